// STREAM-style attainable-bandwidth calibration.  The paper draws its
// roofline with device bandwidth measured by its own STREAM implementation
// (Section 1, Figure perf1); this is the same measurement on gfx950: copy
// (c = a, 2 arrays moved) and triad (a = b + s*c, 3 arrays moved) over
// FP64 arrays far larger than the 256 MB last-level cache, timed with HIP
// events: the best over several passes, grid sizes and kernel shapes is
// reported as attainable.  Shapes: grid-stride (consecutive workgroups touch
// consecutive 4 KB pieces) with 1, 4 or 8 independent 16-byte accesses per
// thread, plain or non-temporal; and contiguous chunks (each workgroup
// streams one long run of each array, the layout the solver kernels use).
// FVPCG_CALIBRATE_VERBOSE=1 prints every variant's rate to stderr.
#include <cstdlib>

#include "common.hpp"

namespace fvpcg {

namespace {

template <bool NT>
__device__ __forceinline__ double2 ld2(const double2* p) {
    if (NT) return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st2(double2* p, double2 v) {
    if (NT) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
    } else {
        *p = v;
    }
}

// Grid-stride copy / triad, U independent 16-byte accesses per thread per
// step (more bytes in flight per wave), optionally non-temporal.
template <int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_copy(const double2* __restrict__ a, double2* __restrict__ c, size_t n2) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + (U - 1) * stride < n2; i += U * stride) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld2<NT>(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) st2<NT>(c + i + u * stride, v[u]);
    }
    for (; i < n2; i += stride) st2<NT>(c + i, ld2<NT>(a + i));
}

template <int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                                  const double2* __restrict__ c, double s, size_t n2) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + (U - 1) * stride < n2; i += U * stride) {
        double2 x[U], y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[u] = ld2<NT>(b + i + u * stride);
            y[u] = ld2<NT>(c + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) st2<NT>(a + i + u * stride, make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y));
    }
    for (; i < n2; i += stride) {
        double2 x = ld2<NT>(b + i), y = ld2<NT>(c + i);
        st2<NT>(a + i, make_double2(x.x + s * y.x, x.y + s * y.y));
    }
}

// Contiguous chunks: workgroup b copies / triads elements [b*len, (b+1)*len)
// with U accesses of 16 bytes in flight per thread, non-temporal.
template <int U>
__global__ __launch_bounds__(kBlock) void k_copy_chunk(const double2* __restrict__ a, double2* __restrict__ c,
                                                      size_t n2, size_t len) {
    const size_t b0 = (size_t)blockIdx.x * len;
    const size_t e = b0 + len < n2 ? b0 + len : n2;
    size_t i = b0 + threadIdx.x;
    for (; i + (U - 1) * kBlock < e; i += U * kBlock) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld2<true>(a + i + u * kBlock);
#pragma unroll
        for (int u = 0; u < U; ++u) st2<true>(c + i + u * kBlock, v[u]);
    }
    for (; i < e; i += kBlock) st2<true>(c + i, ld2<true>(a + i));
}

template <int U>
__global__ __launch_bounds__(kBlock) void k_triad_chunk(double2* __restrict__ a, const double2* __restrict__ b,
                                                       const double2* __restrict__ c, double s, size_t n2,
                                                       size_t len) {
    const size_t b0 = (size_t)blockIdx.x * len;
    const size_t e = b0 + len < n2 ? b0 + len : n2;
    size_t i = b0 + threadIdx.x;
    for (; i + (U - 1) * kBlock < e; i += U * kBlock) {
        double2 x[U], y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[u] = ld2<true>(b + i + u * kBlock);
            y[u] = ld2<true>(c + i + u * kBlock);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) st2<true>(a + i + u * kBlock, make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y));
    }
    for (; i < e; i += kBlock) {
        double2 x = ld2<true>(b + i), y = ld2<true>(c + i);
        st2<true>(a + i, make_double2(x.x + s * y.x, x.y + s * y.y));
    }
}

// Mixed streams: nr arrays read and nw written, every workgroup over one
// contiguous chunk of each (the solver kernels' layout), 16-byte
// non-temporal accesses.  out_j = sum of the inputs; with nw = 0 the sum is
// kept alive by a store that never happens (inputs are filled with 1.0).
constexpr int kMixMaxIn = 16, kMixMaxOut = 8;
struct MixArgs {
    const double2* in[kMixMaxIn];
    double2* out[kMixMaxOut];
    double* sink;
    int nr, nw;
};

// CHUNK: workgroup b streams elements [b len, (b + 1) len); otherwise all
// workgroups sweep the arrays together, workgroup b taking tiles b, b + G, ...
// of kBlock elements (the solver kernels' order).
template <bool CHUNK>
__global__ __launch_bounds__(kBlock) void k_mix(MixArgs m, size_t n2, size_t len) {
    const size_t b0 = CHUNK ? (size_t)blockIdx.x * len : (size_t)blockIdx.x * kBlock;
    const size_t e = CHUNK ? (b0 + len < n2 ? b0 + len : n2) : n2;
    const size_t step = CHUNK ? (size_t)kBlock : (size_t)gridDim.x * kBlock;
    double keep = 0.0;
    for (size_t i = b0 + threadIdx.x; i < e; i += step) {
        double2 v[kMixMaxIn];
#pragma unroll
        for (int k = 0; k < kMixMaxIn; ++k)
            if (k < m.nr) v[k] = ld2<true>(m.in[k] + i);
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < kMixMaxIn; ++k)
            if (k < m.nr) {
                sum.x += v[k].x;
                sum.y += v[k].y;
            }
#pragma unroll
        for (int k = 0; k < kMixMaxOut; ++k)
            if (k < m.nw) st2<true>(m.out[k] + i, sum);
        keep += sum.x + sum.y;
    }
    if (m.nw == 0 && keep == -1.0) m.sink[0] = keep;
}

__global__ __launch_bounds__(kBlock) void k_fill(double2* __restrict__ a, size_t n2, double v) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += (size_t)gridDim.x * kBlock)
        a[i] = make_double2(v, v);
}

}  // namespace

int stream_calibrate(hipStream_t s, uint64_t bytes, double* copy_gbs, double* triad_gbs) {
    if (bytes == 0) bytes = (uint64_t)1 << 30;
    size_t n2 = (size_t)(bytes / sizeof(double2));
    if (n2 < 1024) return set_error(FVPCG_INVALID_ARG, "calibration arrays too small");
    double2 *a = nullptr, *b = nullptr, *c = nullptr;
    int rc;
    if ((rc = dev_alloc(&a, n2, "stream a")) || (rc = dev_alloc(&b, n2, "stream b")) ||
        (rc = dev_alloc(&c, n2, "stream c"))) {
        dev_free(a);
        dev_free(b);
        dev_free(c);
        return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = FVPCG_OK;
    auto body = [&]() -> int {
        FV_HIP(hipEventCreate(&e0));
        FV_HIP(hipEventCreate(&e1));
        int dev = 0;
        FV_HIP(hipGetDevice(&dev));
        int cus = 0;
        FV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int grid = cus * 16;
        hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, s, a, n2, 1.0);
        hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, s, b, n2, 2.0);
        hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, s, c, n2, 0.5);
        FV_LAUNCHED();
        double best_copy = 0, best_triad = 0;
        float ms = 0;
        auto timed = [&](auto&& launch, double bytes, double& best) -> int {
            for (int rep = 0; rep < 4; ++rep) {
                FV_HIP(hipEventRecord(e0, s));
                launch();
                FV_HIP(hipEventRecord(e1, s));
                FV_HIP(hipEventSynchronize(e1));
                FV_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0 && ms > 0) best = std::fmax(best, bytes / (ms * 1e6));
            }
            return FVPCG_OK;
        };
        const double b2 = 2.0 * n2 * sizeof(double2), b3 = 3.0 * n2 * sizeof(double2);
        const char* vb = getenv("FVPCG_CALIBRATE_VERBOSE");
        const bool verbose = vb && vb[0] == '1';
        int rc2;
        auto run = [&](const char* name, int gg, auto&& launch, double bytes, double& best) -> int {
            double mine = 0.0;
            int r = timed(launch, bytes, mine);
            if (verbose) fprintf(stderr, "[calibrate] %-16s grid %5d: %7.1f GB/s\n", name, gg, mine);
            best = std::fmax(best, mine);
            return r;
        };
        for (int gm : {4, 8, 16}) {
            const int gg = cus * gm;
            if ((rc2 = run("copy", gg, [&] { hipLaunchKernelGGL((k_copy<1, false>), dim3(gg), dim3(kBlock), 0, s, a, c, n2); }, b2, best_copy))) return rc2;
            if ((rc2 = run("copy u4", gg, [&] { hipLaunchKernelGGL((k_copy<4, false>), dim3(gg), dim3(kBlock), 0, s, a, c, n2); }, b2, best_copy))) return rc2;
            if ((rc2 = run("copy u4 nt", gg, [&] { hipLaunchKernelGGL((k_copy<4, true>), dim3(gg), dim3(kBlock), 0, s, a, c, n2); }, b2, best_copy))) return rc2;
            if ((rc2 = run("copy u8 nt", gg, [&] { hipLaunchKernelGGL((k_copy<8, true>), dim3(gg), dim3(kBlock), 0, s, a, c, n2); }, b2, best_copy))) return rc2;
            if ((rc2 = run("triad", gg, [&] { hipLaunchKernelGGL((k_triad<1, false>), dim3(gg), dim3(kBlock), 0, s, a, b, c, 0.5, n2); }, b3, best_triad))) return rc2;
            if ((rc2 = run("triad u4", gg, [&] { hipLaunchKernelGGL((k_triad<4, false>), dim3(gg), dim3(kBlock), 0, s, a, b, c, 0.5, n2); }, b3, best_triad))) return rc2;
            if ((rc2 = run("triad u4 nt", gg, [&] { hipLaunchKernelGGL((k_triad<4, true>), dim3(gg), dim3(kBlock), 0, s, a, b, c, 0.5, n2); }, b3, best_triad))) return rc2;
        }
        for (int gm : {1, 2, 4, 8}) {
            const int gg = cus * gm;
            const size_t len = (n2 + gg - 1) / gg;
            if ((rc2 = run("copy chunk u4", gg, [&] { hipLaunchKernelGGL((k_copy_chunk<4>), dim3(gg), dim3(kBlock), 0, s, a, c, n2, len); }, b2, best_copy))) return rc2;
            if ((rc2 = run("copy chunk u8", gg, [&] { hipLaunchKernelGGL((k_copy_chunk<8>), dim3(gg), dim3(kBlock), 0, s, a, c, n2, len); }, b2, best_copy))) return rc2;
            if ((rc2 = run("triad chunk u4", gg, [&] { hipLaunchKernelGGL((k_triad_chunk<4>), dim3(gg), dim3(kBlock), 0, s, a, b, c, 0.5, n2, len); }, b3, best_triad))) return rc2;
        }
        FV_LAUNCHED();
        *copy_gbs = best_copy;
        *triad_gbs = best_triad;
        return FVPCG_OK;
    };
    rc = body();
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(a);
    dev_free(b);
    dev_free(c);
    return rc;
}

int stream_mix(hipStream_t s, uint64_t bytes, int nr, int nw, double* gbs) {
    if (nr < 1 || nr > kMixMaxIn || nw < 0 || nw > kMixMaxOut)
        return set_error(FVPCG_INVALID_ARG, "stream mix: %d arrays read (1..%d) and %d written (0..%d)", nr,
                         kMixMaxIn, nw, kMixMaxOut);
    if (bytes == 0) bytes = (uint64_t)1 << 28;
    const size_t n2 = (size_t)(bytes / sizeof(double2));
    if (n2 < 1024) return set_error(FVPCG_INVALID_ARG, "calibration arrays too small");
    double2* arr[kMixMaxIn + kMixMaxOut] = {};
    double* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto body = [&]() -> int {
        int rc;
        for (int k = 0; k < nr + nw; ++k)
            if ((rc = dev_alloc(&arr[k], n2, "stream mix array"))) return rc;
        if ((rc = dev_alloc(&sink, 1, "stream mix sink"))) return rc;
        FV_HIP(hipEventCreate(&e0));
        FV_HIP(hipEventCreate(&e1));
        int dev = 0, cus = 0;
        FV_HIP(hipGetDevice(&dev));
        FV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        for (int k = 0; k < nr + nw; ++k)
            hipLaunchKernelGGL(k_fill, dim3(cus * 16), dim3(kBlock), 0, s, arr[k], n2, 1.0);
        FV_LAUNCHED();
        MixArgs m{};
        for (int k = 0; k < nr; ++k) m.in[k] = arr[k];
        for (int k = 0; k < nw; ++k) m.out[k] = arr[nr + k];
        m.sink = sink;
        m.nr = nr;
        m.nw = nw;
        const double moved = (double)(nr + nw) * (double)n2 * sizeof(double2);
        const char* vb = getenv("FVPCG_CALIBRATE_VERBOSE");
        const bool verbose = vb && vb[0] == '1';
        double best = 0.0;
        for (int chunk = 1; chunk >= 0; --chunk)
            for (int gm : {1, 2, 4, 8, 16}) {
                const int gg = cus * gm;
                const size_t len = (n2 + gg - 1) / gg;
                double mine = 0.0;
                for (int rep = 0; rep < 4; ++rep) {
                    FV_HIP(hipEventRecord(e0, s));
                    if (chunk)
                        hipLaunchKernelGGL(k_mix<true>, dim3(gg), dim3(kBlock), 0, s, m, n2, len);
                    else
                        hipLaunchKernelGGL(k_mix<false>, dim3(gg), dim3(kBlock), 0, s, m, n2, len);
                    FV_LAUNCHED();
                    FV_HIP(hipEventRecord(e1, s));
                    FV_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    FV_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (rep > 0 && ms > 0) mine = std::fmax(mine, moved / (ms * 1e6));
                }
                if (verbose)
                    fprintf(stderr, "[calibrate] mix %2d in %d out %s grid %5d: %7.1f GB/s\n", nr, nw,
                            chunk ? "chunks" : "sweep ", gg, mine);
                best = std::fmax(best, mine);
            }
        *gbs = best;
        return FVPCG_OK;
    };
    const int rc = body();
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (double2*& a : arr) dev_free(a);
    dev_free(sink);
    return rc;
}

}  // namespace fvpcg
