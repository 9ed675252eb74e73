// STREAM-style attainable-bandwidth calibration.  The paper draws its
// roofline with device bandwidth measured by its own STREAM implementation
// (Section 1, Figure perf1); this is the same measurement on gfx950: copy
// (c = a, 2 arrays moved) and triad (a = b + s*c, 3 arrays moved) over
// FP64 arrays far larger than the 256 MB last-level cache, timed with HIP
// events, best of several passes.
#include "common.hpp"

namespace fvpcg {

namespace {

__global__ __launch_bounds__(kBlock) void k_copy(const double2* __restrict__ a, double2* __restrict__ c, size_t n2) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += (size_t)gridDim.x * kBlock) c[i] = a[i];
}

__global__ __launch_bounds__(kBlock) void k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                                  const double2* __restrict__ c, double s, size_t n2) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += (size_t)gridDim.x * kBlock) {
        double2 x = b[i], y = c[i];
        a[i] = make_double2(x.x + s * y.x, x.y + s * y.y);
    }
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
        for (int rep = 0; rep < 6; ++rep) {
            float ms = 0;
            FV_HIP(hipEventRecord(e0, s));
            hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, s, a, c, n2);
            FV_HIP(hipEventRecord(e1, s));
            FV_HIP(hipEventSynchronize(e1));
            FV_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms > 0) best_copy = std::fmax(best_copy, 2.0 * n2 * sizeof(double2) / (ms * 1e6));
            FV_HIP(hipEventRecord(e0, s));
            hipLaunchKernelGGL(k_triad, dim3(grid), dim3(kBlock), 0, s, a, b, c, 0.5, n2);
            FV_HIP(hipEventRecord(e1, s));
            FV_HIP(hipEventSynchronize(e1));
            FV_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms > 0) best_triad = std::fmax(best_triad, 3.0 * n2 * sizeof(double2) / (ms * 1e6));
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

}  // namespace fvpcg
