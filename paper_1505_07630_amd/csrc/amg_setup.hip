// Smoothed-aggregation AMG: the hierarchy built on the device (the method is
// stated in amg.hpp).
//
// Per level, from the level's CSR operator:
//   k_lvl_diag      diagonal, Gershgorin ratio sum_j |a_ij| / a_ii and its
//                   maximum (an unsigned max over the bit patterns of the
//                   non-negative ratios: exact, order-free);
//   k_strength      the strength mask of every stored entry;
//   k_mis_*         the distance-2 maximal independent set in rounds: two
//                   sweeps of neighbourhood maxima over 64-bit keys (state,
//                   priority, index) give each unknown the largest key within
//                   two strong steps; an undecided unknown whose own key is
//                   that maximum becomes a root, one that sees a root drops
//                   out; the host repeats until none is undecided;
//   k_agg_round1/2  the aggregates (roots numbered by an exclusive scan);
//   P = S P_t, R = P^T, A P, A_c = R (A P): sparse products by a row-wise
//                   k-way merge (one thread per output row keeps a binary heap
//                   of the heads of the rows of the right operand that the
//                   left row selects, keyed by (column, list index); equal
//                   columns are summed in list order, so every entry is summed
//                   in the left row's column order), R by counting, scatter
//                   and a per-row heapsort;
//   last level      dense, inverted by Gauss-Jordan elimination in one
//                   workgroup (SPD: no pivoting; a non-positive pivot is a
//                   breakdown).
// Every result is a function of the operator and the seed: no floating-point
// atomics, integer atomics only for counts and for slot positions that a
// sort puts in order afterwards.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>

#include "amg.hpp"

namespace fvpcg {

namespace {

constexpr int kSetupBs = 256;
constexpr int kScanTile = 1024;  // elements per workgroup in the scan (4 per thread)
constexpr int kMaxMisRounds = 4096;
constexpr uint64_t kKeyMask = (1ull << 62) - 1;  // priority and index below the 2-bit state
constexpr uint64_t kUndecided = 1ull << 62, kRoot = 2ull << 62;

int grid1d(long long work) {
    long long g = (work + kSetupBs - 1) / kSetupBs;
    return (int)std::max(1LL, std::min(g, 65536LL));
}

#define FV_GRID_LOOP(i, n) \
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// One global atomic per workgroup for a value every thread contributes to
// (a count or a maximum over all rows): the workgroup combines its threads'
// values in LDS first.  Same-address atomics from every thread took
// milliseconds per launch at 7M rows.  Every thread of the workgroup must
// call it.
__device__ __forceinline__ void block_atomic_add(int* out, int v) {
    __shared__ int s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    if (v) atomicAdd(&s_sum, v);
    __syncthreads();
    if (threadIdx.x == 0 && s_sum) atomicAdd(out, s_sum);
}
template <typename T>
__device__ __forceinline__ void block_atomic_max(T* out, T v) {  // v >= 0
    __shared__ T s_max;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (v) atomicMax(&s_max, v);
    __syncthreads();
    if (threadIdx.x == 0 && s_max) atomicMax(out, s_max);
}

// Device buffer owned by one setup step.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { dev_free(p); }
    int alloc(size_t count, const char* what) {
        dev_free(p);
        return dev_alloc(&p, count, what);
    }
    void reset() { dev_free(p); }
};

template <typename T>
int read_scalar(T* host, const T* dev, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// ---------------------------------------------------------------- scan
// out[i] = sum_{k < i} in[k] for i <= n (out has n + 1 entries).  Each
// workgroup scans a tile of 1024 (four consecutive elements per thread, the
// thread totals by a Hillis-Steele scan in LDS) and writes its total; the
// tile totals are scanned the same way and added back.
template <typename T>
__global__ __launch_bounds__(kSetupBs) void k_scan_tile(const T* __restrict__ in, long long n, T* __restrict__ out,
                                                        T* __restrict__ tile_sum) {
    __shared__ T s[kSetupBs];
    const long long base = (long long)blockIdx.x * kScanTile + 4 * (long long)threadIdx.x;
    T v[4];
    T t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : T(0);
        t += v[k];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kSetupBs; off <<= 1) {
        const T a = (int)threadIdx.x >= off ? s[threadIdx.x - off] : T(0);
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    T run = s[threadIdx.x] - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kSetupBs - 1) tile_sum[blockIdx.x] = s[kSetupBs - 1];
}

template <typename T>
__global__ __launch_bounds__(kSetupBs) void k_scan_add(T* __restrict__ out, long long n, const T* __restrict__ tile_off) {
    FV_GRID_LOOP(i, n) out[i] += tile_off[i / kScanTile];
}

template <typename T>
__global__ void k_scan_total(T* __restrict__ out, long long n, const T* __restrict__ src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = src[0];
}

template <typename T>
int scan_excl(const T* in, T* out, long long n, hipStream_t s) {
    const long long tiles = std::max(1LL, (n + kScanTile - 1) / kScanTile);
    DevBuf<T> tsum, toff;
    int rc;
    if ((rc = tsum.alloc((size_t)tiles, "scan tile sums"))) return rc;
    hipLaunchKernelGGL((k_scan_tile<T>), dim3((unsigned)tiles), dim3(kSetupBs), 0, s, in, n, out, tsum.p);
    FV_LAUNCHED();
    if (tiles == 1) {
        hipLaunchKernelGGL((k_scan_total<T>), dim3(1), dim3(64), 0, s, out, n, tsum.p);
        FV_LAUNCHED();
        FV_HIP(hipStreamSynchronize(s));  // the tile buffer is freed on return
        return FVPCG_OK;
    }
    if ((rc = toff.alloc((size_t)tiles + 1, "scan tile offsets"))) return rc;
    if ((rc = scan_excl<T>(tsum.p, toff.p, tiles, s))) return rc;
    hipLaunchKernelGGL((k_scan_add<T>), dim3(grid1d(n)), dim3(kSetupBs), 0, s, out, n, toff.p);
    hipLaunchKernelGGL((k_scan_total<T>), dim3(1), dim3(64), 0, s, out, n, toff.p + tiles);
    FV_LAUNCHED();
    FV_HIP(hipStreamSynchronize(s));  // the tile buffers are freed on return
    return FVPCG_OK;
}

// ---------------------------------------------------------------- level 0
// Level 0 as CSR from the ELL layout: the diagonal at its sorted place among
// the row's slots (sorted by column; padding repeats the row and is skipped).
__global__ __launch_bounds__(kSetupBs) void k_l0_count(const int* __restrict__ col, int n, int W, int* __restrict__ cnt) {
    FV_GRID_LOOP(c, n) {
        int k = 1;
        for (int s = 0; s < W; ++s) k += col[(size_t)s * n + c] != (int)c;
        cnt[c] = k;
    }
}

__global__ __launch_bounds__(kSetupBs) void k_l0_fill(const int* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ d, int n, int W,
                                                     const int* __restrict__ ptr, int* __restrict__ ocol,
                                                     double* __restrict__ oval) {
    FV_GRID_LOOP(c, n) {
        int p = ptr[c];
        bool diag = false;
        for (int s = 0; s < W; ++s) {
            const int j = col[(size_t)s * n + c];
            if (j == (int)c) continue;
            if (!diag && j > (int)c) {
                ocol[p] = (int)c;
                oval[p++] = d[c];
                diag = true;
            }
            ocol[p] = j;
            oval[p++] = val[(size_t)s * n + c];
        }
        if (!diag) {
            ocol[p] = (int)c;
            oval[p] = d[c];
        }
    }
}

// ---------------------------------------------------------------- per level
// d_i = a_ii; ratio_i = (sum_j |a_ij|) / a_ii, summed in column order; the
// largest ratio as the maximum of the bit patterns (non-negative doubles
// order like their bits).  bad: a diagonal that is not finite and positive.
__global__ __launch_bounds__(kSetupBs) void k_lvl_diag(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val, int n, double* __restrict__ d,
                                                      unsigned long long* rho_bits, int* bad) {
    unsigned long long mx = 0;
    int b = 0;
    FV_GRID_LOOP(i, n) {
        double di = 0.0, sa = 0.0;
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            if (col[p] == (int)i) di = val[p];
            sa += fabs(val[p]);
        }
        d[i] = di;
        if (!(di > 0.0) || !isfinite(di) || !isfinite(sa)) {
            b = 1;
        } else {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(sa / di);
            mx = bits > mx ? bits : mx;
        }
    }
    block_atomic_max<unsigned long long>(rho_bits, mx);
    if (b) atomicOr(bad, 1);
}

// a_ij / d_j (the coarse levels' column-scaled values)
__global__ __launch_bounds__(kSetupBs) void k_lvl_colscale(const int* __restrict__ col, const double* __restrict__ val,
                                                          const double* __restrict__ d, long long nnz,
                                                          double* __restrict__ cs) {
    FV_GRID_LOOP(p, nnz) cs[p] = val[p] / d[col[p]];
}

// strong[p]: entry p of row i couples i to j = col[p] != i with a_ij != 0
// and |a_ij| >= theta sqrt(|a_ii a_jj|)
__global__ __launch_bounds__(kSetupBs) void k_strength(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val, const double* __restrict__ d,
                                                      int n, double theta, uint8_t* __restrict__ strong) {
    FV_GRID_LOOP(i, n) {
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int j = col[p];
            const double a = val[p];
            strong[p] = (j != (int)i && a != 0.0 && fabs(a) >= theta * sqrt(fabs(d[i] * d[j]))) ? 1 : 0;
        }
    }
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based
// generator: element k of the sequence started at `seed` is the finaliser
// applied to seed + (k + 1) * 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// key = state (2 bits: 0 out, 1 undecided, 2 root) | 31 random bits | index
__global__ __launch_bounds__(kSetupBs) void k_mis_init(int n, uint64_t seed, int level, uint64_t* __restrict__ key) {
    FV_GRID_LOOP(i, n) {
        const uint64_t r = splitmix64_at(seed, ((uint64_t)(uint32_t)level << 32) | (uint64_t)i) >> 33;
        key[i] = kUndecided | (r << 31) | (uint64_t)i;
    }
}

// out_i = max(in_i, in_j over strong neighbours j)
__global__ __launch_bounds__(kSetupBs) void k_mis_max(const int* __restrict__ ptr, const int* __restrict__ col,
                                                     const uint8_t* __restrict__ strong, int n,
                                                     const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
    FV_GRID_LOOP(i, n) {
        uint64_t m = in[i];
        for (int p = ptr[i]; p < ptr[i + 1]; ++p)
            if (strong[p]) {
                const uint64_t v = in[col[p]];
                m = v > m ? v : m;
            }
        out[i] = m;
    }
}

// The same maxima with G lanes per row, for the coarse levels whose rows
// hold tens of entries: the lanes stride through the row and the group's
// maximum is formed by butterfly shuffles within the group.  A maximum is
// exact in any order, so the result is that of k_mis_max.
template <int G>
__global__ __launch_bounds__(kSetupBs) void k_mis_max_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                       const uint8_t* __restrict__ strong, int n,
                                                       const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
    const int lane = threadIdx.x & 63, sub = lane / G, gl = lane % G;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwave = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long base = wave * (64 / G); base < n; base += nwave * (64 / G)) {  // wave-uniform
        const long long i = base + sub;
        unsigned long long m = 0;
        if (i < n) {
            if (gl == 0) m = in[i];
            for (int p = ptr[i] + gl; p < ptr[i + 1]; p += G)
                if (strong[p]) {
                    const unsigned long long v = in[col[p]];
                    m = v > m ? v : m;
                }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            const unsigned long long v = __shfl_xor(m, o, 64);
            m = v > m ? v : m;
        }
        if (i < n && gl == 0) out[i] = m;
    }
}

int mis_group_grid(int n, int G) {
    const long long rows_per_block = (long long)(kSetupBs / 64) * (64 / G);
    return (int)std::max(1LL, std::min(((long long)n + rows_per_block - 1) / rows_per_block, 65536LL));
}

// Level 0 in the matrix's slot layout (slot k of row c at k n + c, padding
// repeating the row with a zero value): the same strength relation, stored
// per slot, and the same maxima, read with coalesced slot loads.
__global__ __launch_bounds__(kSetupBs) void k_strength_ell(const int* __restrict__ col, const double* __restrict__ val,
                                                          const double* __restrict__ d, int n, int W, double theta,
                                                          uint8_t* __restrict__ strong) {
    FV_GRID_LOOP(c, n) {
        for (int k = 0; k < W; ++k) {
            const size_t o = (size_t)k * n + c;
            const int j = col[o];
            const double a = val[o];
            strong[o] = (j != (int)c && a != 0.0 && fabs(a) >= theta * sqrt(fabs(d[c] * d[j]))) ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(kSetupBs) void k_mis_max_ell(const int* __restrict__ col,
                                                         const uint8_t* __restrict__ strong, int n, int W,
                                                         const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
    FV_GRID_LOOP(c, n) {
        uint64_t m = in[c];
        for (int k = 0; k < W; ++k) {
            const size_t o = (size_t)k * n + c;
            if (strong[o]) {
                const uint64_t v = in[col[o]];
                m = v > m ? v : m;
            }
        }
        out[c] = m;
    }
}

// m2_i: the largest key within two strong steps of i.
__global__ __launch_bounds__(kSetupBs) void k_mis_decide(int n, uint64_t* __restrict__ key,
                                                        const uint64_t* __restrict__ m2, int* undecided) {
    int left = 0;
    FV_GRID_LOOP(i, n) {
        const uint64_t k = key[i];
        if ((k & ~kKeyMask) != kUndecided) continue;
        const uint64_t m = m2[i];
        if (m == k)
            key[i] = (k & kKeyMask) | kRoot;
        else if ((m & ~kKeyMask) == kRoot)
            key[i] = k & kKeyMask;
        else
            ++left;
    }
    block_atomic_add(undecided, left);
}

__global__ __launch_bounds__(kSetupBs) void k_root_flags(int n, const uint64_t* __restrict__ key, int* __restrict__ f) {
    FV_GRID_LOOP(i, n) f[i] = (key[i] & ~kKeyMask) == kRoot ? 1 : 0;
}

// round 1: roots take their rank; others the aggregate of a root neighbour
__global__ __launch_bounds__(kSetupBs) void k_agg_round1(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const uint8_t* __restrict__ strong, int n,
                                                        const uint64_t* __restrict__ key, const int* __restrict__ rank,
                                                        int* __restrict__ agg1) {
    FV_GRID_LOOP(i, n) {
        int a = -1;
        if ((key[i] & ~kKeyMask) == kRoot) {
            a = rank[i];
        } else {
            for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
                const int j = col[p];
                if (strong[p] && (key[j] & ~kKeyMask) == kRoot) {
                    a = rank[j];
                    break;
                }
            }
        }
        agg1[i] = a;
    }
}

// round 2: the rest join the round-1 aggregate of the strong neighbour with
// the largest |a_ij| (columns ascend in the row: the first wins ties)
__global__ __launch_bounds__(kSetupBs) void k_agg_round2(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const uint8_t* __restrict__ strong, int n,
                                                        const int* __restrict__ agg1, int* __restrict__ agg,
                                                        int* missing) {
    FV_GRID_LOOP(i, n) {
        int a = agg1[i];
        if (a < 0) {
            double best = -1.0;
            for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
                const int j = col[p];
                if (!strong[p] || agg1[j] < 0) continue;
                const double w = fabs(val[p]);
                if (w > best) {
                    best = w;
                    a = agg1[j];
                }
            }
            if (a < 0) {
                atomicOr(missing, 1);
                a = 0;
            }
        }
        agg[i] = a;
    }
}

// rows of S = I - omega D^-1 A (the pattern of A)
__global__ __launch_bounds__(kSetupBs) void k_smoother_rows(const int* __restrict__ ptr, const int* __restrict__ col,
                                                           const double* __restrict__ val, const double* __restrict__ d,
                                                           int n, double omega, double* __restrict__ sval) {
    FV_GRID_LOOP(i, n) {
        for (int p = ptr[i]; p < ptr[i + 1]; ++p)
            sval[p] = (col[p] == (int)i ? 1.0 : 0.0) - omega * val[p] / d[i];
    }
}

// P_t: row i holds (agg_i, 1)
__global__ __launch_bounds__(kSetupBs) void k_tentative(int n, int* __restrict__ ptr, double* __restrict__ ones) {
    FV_GRID_LOOP(i, n + 1) {
        ptr[i] = (int)i;
        if (i < n) ones[i] = 1.0;
    }
}

// ---------------------------------------------------------------- products
// Upper bound of the entries of row i of X Y: the lengths of the rows of Y
// that row i of X selects.
// Also the longest row of X into *maxlen.
__global__ __launch_bounds__(kSetupBs) void k_gemm_bound(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                        const int* __restrict__ yptr, int rows,
                                                        long long* __restrict__ ub, int* maxlen) {
    int m = 0;
    FV_GRID_LOOP(i, rows) {
        long long t = 0;
        for (int p = xptr[i]; p < xptr[i + 1]; ++p) t += yptr[xcol[p] + 1] - yptr[xcol[p]];
        ub[i] = t;
        m = max(m, xptr[i + 1] - xptr[i]);
    }
    block_atomic_max<int>(maxlen, m);
}

// binary min-heap of keys (column, list index): 64-bit keys (column << 32 |
// index), or 32-bit ones (column << 6 | index) when there are at most 64
// lists and under 2^26 columns; both order the heads alike.
template <typename K>
__device__ __forceinline__ void heap_up(K* H, int i) {
    const K v = H[i];
    while (i > 0) {
        const int q = (i - 1) >> 1;
        const K pv = H[q];
        if (pv <= v) break;
        H[i] = pv;
        i = q;
    }
    H[i] = v;
}

template <typename K>
__device__ __forceinline__ void heap_down(K* H, int h, int i) {
    const K v = H[i];
    for (;;) {
        int c = 2 * i + 1;
        if (c >= h) break;
        K cv = H[c];
        if (c + 1 < h) {
            const K rv = H[c + 1];
            if (rv < cv) {
                ++c;
                cv = rv;
            }
        }
        if (cv >= v) break;
        H[i] = cv;
        i = c;
    }
    H[i] = v;
}

template <typename K>
struct HeapKey;
template <>
struct HeapKey<unsigned long long> {
    static constexpr int kShift = 32;
};
template <>
struct HeapKey<unsigned int> {
    static constexpr int kShift = 6;  // up to 64 lists
};
constexpr int kKey32Lists = 64;
constexpr int kKey32Cols = 1 << 26;

#pragma clang fp contract(off)
// Row i of C = X Y by a k-way merge of the rows Y(k, :) for k in X(i, :):
// the heap H holds (column << 32 | list index) of each list's head, P each
// list's current position; popping yields the columns in ascending order
// and, for equal columns, the lists in X's column order, in which their
// products are summed (each product rounded, then added).  Output: the
// row's distinct columns and sums at off[i] in (tcol, tval), and its count.
template <typename K>
__device__ __forceinline__ void merge_row(long long i, const int* __restrict__ xptr, const int* __restrict__ xcol,
                                          const double* __restrict__ xval, const int* __restrict__ yptr,
                                          const int* __restrict__ ycol, const double* __restrict__ yval,
                                          const long long* __restrict__ off, K* H, int* P,
                                          int* __restrict__ tcol, double* __restrict__ tval, int* __restrict__ cnt) {
    constexpr int kS = HeapKey<K>::kShift;
    constexpr K kMask = ((K)1 << kS) - 1;
    const int base = xptr[i], L = xptr[i + 1] - base;
    int h = 0;
    for (int t = 0; t < L; ++t) {
        const int k = xcol[base + t];
        const int b = yptr[k];
        if (b < yptr[k + 1]) {
            P[t] = b;
            H[h] = ((K)(unsigned)ycol[b] << kS) | (K)(unsigned)t;
            heap_up(H, h);
            ++h;
        }
    }
    const long long o = off[i];
    int out = 0, last = -1;
    double acc = 0.0;
    while (h > 0) {
        const K top = H[0];
        const int c = (int)(top >> kS), t = (int)(top & kMask);
        const int k = xcol[base + t];
        int p = P[t];
        const double v = xval[base + t] * yval[p];
        if (c == last) {
            acc += v;
        } else {
            if (last >= 0) {
                tcol[o + out] = last;
                tval[o + out] = acc;
                ++out;
            }
            last = c;
            acc = v;
        }
        ++p;
        if (p < yptr[k + 1]) {
            P[t] = p;
            H[0] = ((K)(unsigned)ycol[p] << kS) | (K)(unsigned)t;
            heap_down(H, h, 0);
        } else if (--h > 0) {
            H[0] = H[h];
            heap_down(H, h, 0);
        }
    }
    if (last >= 0) {
        tcol[o + out] = last;
        tval[o + out] = acc;
        ++out;
    }
    cnt[i] = out;
}
#pragma clang fp contract(on)

// Row i of C = X Y for rows of X with at most SM entries (level 0's
// products): the heads of the lists Y(k_t, :) stay in registers; each step
// takes the smallest head column and adds, in X's column order t, the
// products of the lists whose head it is (each product rounded, then added,
// the first one taken as it is), then advances those lists.  Every column
// thus receives its products in the heap merge's order, so the sums are
// bitwise the merge's; the loads of the advanced heads are independent of
// each other, where the heap merge waits on one load per product.
constexpr int kShortLists = 8;
#pragma clang fp contract(off)
template <int SM>
__global__ __launch_bounds__(kSetupBs) void k_gemm_short(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                        const double* __restrict__ xval, const int* __restrict__ yptr,
                                                        const int* __restrict__ ycol, const double* __restrict__ yval,
                                                        int rows, const long long* __restrict__ off,
                                                        int* __restrict__ tcol, double* __restrict__ tval,
                                                        int* __restrict__ cnt) {
    constexpr int kNone = 0x7fffffff;
    FV_GRID_LOOP(i, rows) {
        const int base = xptr[i], L = xptr[i + 1] - base;
        int head[SM], pos[SM], end[SM];
        double xv[SM];
#pragma unroll
        for (int t = 0; t < SM; ++t) {
            head[t] = kNone;
            pos[t] = 0;
            end[t] = 0;
            xv[t] = 0.0;
            if (t < L) {
                const int k = xcol[base + t];
                xv[t] = xval[base + t];
                pos[t] = yptr[k];
                end[t] = yptr[k + 1];
                if (pos[t] < end[t]) head[t] = ycol[pos[t]];
            }
        }
        const long long o = off[i];
        int out = 0;
        for (;;) {
            int c = kNone;
#pragma unroll
            for (int t = 0; t < SM; ++t) c = head[t] < c ? head[t] : c;
            if (c == kNone) break;
            double acc = 0.0;
            bool first = true;
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (head[t] == c) {
                    const double v = xv[t] * yval[pos[t]];
                    acc = first ? v : acc + v;
                    first = false;
                    ++pos[t];
                    head[t] = pos[t] < end[t] ? ycol[pos[t]] : kNone;
                }
            }
            tcol[o + out] = c;
            tval[o + out] = acc;
            ++out;
        }
        cnt[i] = out;
    }
}
#pragma clang fp contract(on)

// One row per thread, heap and positions in device memory indexed like X
// (rows whose list count exceeds the LDS budget).
__global__ __launch_bounds__(kSetupBs) void k_gemm_merge(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                        const double* __restrict__ xval, const int* __restrict__ yptr,
                                                        const int* __restrict__ ycol, const double* __restrict__ yval,
                                                        int rows, const long long* __restrict__ off,
                                                        unsigned long long* __restrict__ heap, int* __restrict__ pos,
                                                        int* __restrict__ tcol, double* __restrict__ tval,
                                                        int* __restrict__ cnt) {
    FV_GRID_LOOP(i, rows) {
        const int base = xptr[i];
        merge_row<unsigned long long>(i, xptr, xcol, xval, yptr, ycol, yval, off, heap + base, pos + base, tcol,
                                      tval, cnt);
    }
}

// The same with each thread's heap and positions in LDS (lcap entries of 12
// bytes per row, per_wg rows per workgroup of kLdsBs threads): the merge's
// dependent heap accesses then cost LDS latency instead of device-memory
// latency, which decides the coarse levels' long rows.
constexpr int kLdsBs = 64;
constexpr int kLdsBytes = 65536;
constexpr long long kDenseEntries = 1LL << 27;  // rows x columns of a product accumulated densely (1.2 GB)
template <typename K>
__global__ __launch_bounds__(kLdsBs) void k_gemm_merge_lds(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                          const double* __restrict__ xval,
                                                          const int* __restrict__ yptr, const int* __restrict__ ycol,
                                                          const double* __restrict__ yval, int rows, int per_wg,
                                                          int lcap, const long long* __restrict__ off,
                                                          int* __restrict__ tcol, double* __restrict__ tval,
                                                          int* __restrict__ cnt) {
    extern __shared__ unsigned long long lds_heap_raw[];
    K* lds_heap = reinterpret_cast<K*>(lds_heap_raw);
    const int t = (int)threadIdx.x;
    const long long i = (long long)blockIdx.x * per_wg + t;
    if (t >= per_wg || i >= rows) return;
    K* H = lds_heap + (size_t)t * lcap;
    int* P = reinterpret_cast<int*>(lds_heap + (size_t)per_wg * lcap) + (size_t)t * lcap;
    merge_row<K>(i, xptr, xcol, xval, yptr, ycol, yval, off, H, P, tcol, tval, cnt);
}

// Row i of C = X Y with one wavefront per row and a dense accumulator of
// the row in device memory (acc/touched: nc entries per row), for products
// whose column count nc is small: lane k owns the columns [k w, (k+1) w)
// and walks the rows Y(k_t, :) for t in X's column order, adding the
// products that fall in its columns (found by binary search in each sorted
// Y row).  Every column therefore receives its products in the merge's
// order, so the sums are bitwise the merge's; the touched columns are
// written in ascending order at off[i].
#pragma clang fp contract(off)
__global__ __launch_bounds__(64) void k_gemm_dense(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                  const double* __restrict__ xval, const int* __restrict__ yptr,
                                                  const int* __restrict__ ycol, const double* __restrict__ yval,
                                                  int rows, int nc, const long long* __restrict__ off,
                                                  double* __restrict__ acc_all, uint8_t* __restrict__ touched_all,
                                                  int* __restrict__ tcol, double* __restrict__ tval,
                                                  int* __restrict__ cnt) {
    const int lane = (int)threadIdx.x;
    const int w = (nc + 63) / 64;
    const int c0 = min(lane * w, nc), c1 = min(c0 + w, nc);
    for (long long i = blockIdx.x; i < rows; i += gridDim.x) {
        double* acc = acc_all + (size_t)i * nc;
        uint8_t* touched = touched_all + (size_t)i * nc;
        for (int c = c0; c < c1; ++c) {
            acc[c] = 0.0;
            touched[c] = 0;
        }
        const int base = xptr[i], L = xptr[i + 1] - base;
        for (int t = 0; t < L; ++t) {
            const int k = xcol[base + t];
            const double xv = xval[base + t];
            int lo = yptr[k], hi = yptr[k + 1];
            while (lo < hi) {  // first entry with column >= c0
                const int mid = (lo + hi) >> 1;
                if (ycol[mid] < c0) lo = mid + 1;
                else hi = mid;
            }
            for (int p = lo, e = yptr[k + 1]; p < e; ++p) {
                const int c = ycol[p];
                if (c >= c1) break;
                acc[c] += xv * yval[p];
                touched[c] = 1;
            }
        }
        int mine = 0;
        for (int c = c0; c < c1; ++c) mine += touched[c];
        // exclusive prefix of the lanes' counts (lanes own ascending ranges)
        int incl = mine;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d, 64);
            if (lane >= d) incl += v;
        }
        long long o = off[i] + (incl - mine);
        for (int c = c0; c < c1; ++c)
            if (touched[c]) {
                tcol[o] = c;
                tval[o] = acc[c];
                ++o;
            }
        if (lane == 63) cnt[i] = incl;
    }
}
#pragma clang fp contract(on)

// Row i of C = X Y by one wavefront per row over tiles of kTileCols output
// columns accumulated in LDS, for products whose rows gather many long rows
// of Y (the coarse Galerkin products).  Each list (the row Y(k_t, :) for
// the t-th entry of X's row) keeps a cursor in LDS.  A tile starts at the
// smallest pending column; the lists are visited in X's column order, eight
// at a time with their next 64 entries loaded together, and each list's
// entries inside the tile are added lane by entry (a row's columns are
// distinct, so one pass has no conflicts): the first product of a column is
// stored, later ones added.  Every column therefore receives its products in
// the merge's order and its sum is bitwise the merge's.  The touched columns
// of the tile (a bitmap) are written in ascending order and cleared.
constexpr int kTileCols = 4096;
constexpr int kTileGroup = 8;
constexpr int kTileMaxLists = 4096;
constexpr long long kTileMinWork = 2048;  // mean product entries per row from which the tiles pay

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}

#pragma clang fp contract(off)
__global__ __launch_bounds__(64) void k_gemm_tiled(const int* __restrict__ xptr, const int* __restrict__ xcol,
                                                  const double* __restrict__ xval, const int* __restrict__ yptr,
                                                  const int* __restrict__ ycol, const double* __restrict__ yval,
                                                  int rows, const long long* __restrict__ off,
                                                  int* __restrict__ tcol, double* __restrict__ tval,
                                                  int* __restrict__ cnt) {
    __shared__ double acc[kTileCols];
    __shared__ unsigned int bits[kTileCols / 32];
    __shared__ int cur[kTileMaxLists];
    const int lane = (int)threadIdx.x;
    for (int q = lane; q < kTileCols / 32; q += 64) bits[q] = 0u;
    for (long long i = blockIdx.x; i < rows; i += gridDim.x) {
        const int base = xptr[i], L = xptr[i + 1] - base;
        for (int t = lane; t < L; t += 64) cur[t] = yptr[xcol[base + t]];
        __syncthreads();
        long long o = off[i];
        for (;;) {
            int lo = INT_MAX;
            for (int t = lane; t < L; t += 64) {
                const int p = cur[t];
                if (p < yptr[xcol[base + t] + 1]) lo = min(lo, ycol[p]);
            }
            lo = wave_min_int(lo);
            if (lo == INT_MAX) break;
            const int hi = lo > INT_MAX - kTileCols ? INT_MAX : lo + kTileCols;
            for (int t0 = 0; t0 < L; t0 += kTileGroup) {
                int cc[kTileGroup];
                double vv[kTileGroup];
#pragma unroll
                for (int g = 0; g < kTileGroup; ++g) {
                    cc[g] = INT_MAX;
                    vv[g] = 0.0;
                    const int t = t0 + g;
                    if (t < L) {
                        const int k = xcol[base + t];
                        const int p = cur[t] + lane;
                        if (p < yptr[k + 1]) {
                            cc[g] = ycol[p];
                            vv[g] = xval[base + t] * yval[p];
                        }
                    }
                }
#pragma unroll
                for (int g = 0; g < kTileGroup; ++g) {
                    const int t = t0 + g;
                    if (t >= L) break;
                    int c = cc[g];
                    double v = vv[g];
                    int p0 = cur[t];
                    for (;;) {
                        const bool in = c < hi;
                        if (in) {
                            const int idx = c - lo;
                            const unsigned int m = 1u << (idx & 31);
                            const unsigned int old = atomicOr(&bits[idx >> 5], m);
                            if (old & m)
                                acc[idx] += v;
                            else
                                acc[idx] = v;
                        }
                        const int n_in = __popcll(__ballot(in));
                        p0 += n_in;
                        if (n_in < 64) break;
                        // a full chunk inside the tile: the list's next entries
                        // come before the next list's
                        const int k = xcol[base + t];
                        const int p = p0 + lane;
                        c = INT_MAX;
                        v = 0.0;
                        if (p < yptr[k + 1]) {
                            c = ycol[p];
                            v = xval[base + t] * yval[p];
                        }
                    }
                    if (lane == 0) cur[t] = p0;
                    __syncthreads();
                }
            }
            // the tile's columns in ascending order: lane l owns bitmap words 2l, 2l+1
            const unsigned int w0 = bits[2 * lane], w1 = bits[2 * lane + 1];
            const int mine = __popc(w0) + __popc(w1);
            int incl = mine;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int u = __shfl_up(incl, d, 64);
                if (lane >= d) incl += u;
            }
            long long q = o + (incl - mine);
            for (int h = 0; h < 2; ++h) {
                unsigned int w = h ? w1 : w0;
                while (w) {
                    const int b = __ffs(w) - 1;
                    w &= w - 1;
                    const int idx = (2 * lane + h) * 32 + b;
                    tcol[q] = lo + idx;
                    tval[q] = acc[idx];
                    ++q;
                }
            }
            bits[2 * lane] = 0u;
            bits[2 * lane + 1] = 0u;
            o += __shfl(incl, 63, 64);
            __syncthreads();
        }
        if (lane == 0) cnt[i] = (int)(o - off[i]);
        __syncthreads();
    }
}
#pragma clang fp contract(on)

// the longest row of a CSR matrix
__global__ __launch_bounds__(kSetupBs) void k_max_rowlen(const int* __restrict__ ptr, int rows, int* out) {
    int m = 0;
    FV_GRID_LOOP(i, rows) m = max(m, ptr[i + 1] - ptr[i]);
    block_atomic_max<int>(out, m);
}

// 64-bit copy of a row-pointer array
__global__ __launch_bounds__(kSetupBs) void k_widen(const int* __restrict__ ptr, int n, long long* __restrict__ out) {
    FV_GRID_LOOP(i, n) out[i] = ptr[i];
}

// The rows, written at their upper-bound offsets, copied to C's row
// pointers; G lanes per row so that each row's copy is coalesced.
template <int G>
__global__ __launch_bounds__(kSetupBs) void k_gemm_compact(int rows, const long long* __restrict__ off,
                                                          const int* __restrict__ cnt, const int* __restrict__ cptr,
                                                          const int* __restrict__ tcol, const double* __restrict__ tval,
                                                          int* __restrict__ ccol, double* __restrict__ cval) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int gl = (int)(t % G);
    const long long stride = (long long)gridDim.x * blockDim.x / G;
    for (long long i = t / G; i < rows; i += stride) {
        const long long o = off[i];
        const int q = cptr[i], c = cnt[i];
        for (int k = gl; k < c; k += G) {
            ccol[q + k] = tcol[o + k];
            cval[q + k] = tval[o + k];
        }
    }
}

// ---------------------------------------------------------------- transpose
__global__ __launch_bounds__(kSetupBs) void k_col_count(const int* __restrict__ col, long long nnz, int* __restrict__ cnt) {
    FV_GRID_LOOP(p, nnz) atomicAdd(&cnt[col[p]], 1);
}

__global__ __launch_bounds__(kSetupBs) void k_tr_scatter(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const double* __restrict__ val, int rows,
                                                        const int* __restrict__ tptr, int* __restrict__ cursor,
                                                        int* __restrict__ tcol, double* __restrict__ tval) {
    FV_GRID_LOOP(i, rows) {
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int c = col[p];
            const int q = tptr[c] + atomicAdd(&cursor[c], 1);
            tcol[q] = (int)i;
            tval[q] = val[p];
        }
    }
}

__device__ __forceinline__ void sift_max(int* a, double* v, int i, int n) {
    const int ka = a[i];
    const double kv = v[i];
    for (;;) {
        int c = 2 * i + 1;
        if (c >= n) break;
        if (c + 1 < n && a[c + 1] > a[c]) ++c;
        if (a[c] <= ka) break;
        a[i] = a[c];
        v[i] = v[c];
        i = c;
    }
    a[i] = ka;
    v[i] = kv;
}

__device__ __forceinline__ void heapsort_row(int* a, double* v, int n) {
    for (int s = n / 2 - 1; s >= 0; --s) sift_max(a, v, s, n);
    for (int e = n - 1; e > 0; --e) {
        const int ta = a[0];
        const double tv = v[0];
        a[0] = a[e];
        v[0] = v[e];
        a[e] = ta;
        v[e] = tv;
        sift_max(a, v, 0, e);
    }
}

// each row sorted by column (distinct columns: the order is unique)
__global__ __launch_bounds__(kSetupBs) void k_row_heapsort(const int* __restrict__ ptr, int rows, int* __restrict__ col,
                                                          double* __restrict__ val) {
    FV_GRID_LOOP(i, rows) heapsort_row(col + ptr[i], val + ptr[i], ptr[i + 1] - ptr[i]);
}

// the same with the row copied into LDS first (lcap entries of 12 bytes per
// row, per_wg rows per workgroup)
__global__ __launch_bounds__(kLdsBs) void k_row_heapsort_lds(const int* __restrict__ ptr, int rows, int per_wg,
                                                            int lcap, int* __restrict__ col,
                                                            double* __restrict__ val) {
    extern __shared__ double lds_row[];
    const int t = (int)threadIdx.x;
    const long long i = (long long)blockIdx.x * per_wg + t;
    if (t >= per_wg || i >= rows) return;
    double* v = lds_row + (size_t)t * lcap;
    int* a = reinterpret_cast<int*>(lds_row + (size_t)per_wg * lcap) + (size_t)t * lcap;
    const int b = ptr[i], n = ptr[i + 1] - b;
    for (int k = 0; k < n; ++k) {
        a[k] = col[b + k];
        v[k] = val[b + k];
    }
    heapsort_row(a, v, n);
    for (int k = 0; k < n; ++k) {
        col[b + k] = a[k];
        val[b + k] = v[k];
    }
}

// ---------------------------------------------------------------- last level
__global__ __launch_bounds__(kSetupBs) void k_dense_zero(int n, double* __restrict__ M) {
    FV_GRID_LOOP(e, (long long)n * n) M[e] = 0.0;
}

__global__ __launch_bounds__(kSetupBs) void k_dense_fill(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const double* __restrict__ val, int n, double* __restrict__ M) {
    FV_GRID_LOOP(i, n) {
        for (int p = ptr[i]; p < ptr[i + 1]; ++p) M[(size_t)i * n + col[p]] = val[p];
    }
}

// In-place Gauss-Jordan inverse of an SPD matrix by one workgroup: for each
// pivot k, row k is divided by a_kk (its k-th entry becoming 1 / a_kk), then
// every other row i loses a_ik times the new row k (its k-th entry becoming
// -a_ik / a_kk).  f holds column k before the step.  bad = 1 on a pivot that
// is not finite and positive (every thread reads the same pivot).
constexpr int kGjBs = 1024;
__global__ __launch_bounds__(kGjBs) void k_gauss_jordan(double* __restrict__ M, int n, double* __restrict__ f,
                                                       int* bad) {
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double piv = M[(size_t)k * n + k];
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (threadIdx.x == 0) *bad = 1;
            return;
        }
        for (int i = threadIdx.x; i < n; i += kGjBs) f[i] = M[(size_t)i * n + k];
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += kGjBs) M[(size_t)k * n + j] = (j == k ? 1.0 : M[(size_t)k * n + j]) / piv;
        __syncthreads();
        const long long nn = (long long)n * n;
        for (long long e = threadIdx.x; e < nn; e += kGjBs) {
            const int i = (int)(e / n), j = (int)(e - (long long)i * n);
            if (i == k) continue;
            M[e] = (j == k ? 0.0 : M[e]) - f[i] * M[(size_t)k * n + j];
        }
    }
}

// The same elimination for larger last levels, one pivot per pair of
// launches over the whole grid (one workgroup would stream the matrix
// through a single CU at every step): k_gj_pivot saves column k in f and the
// scaled row k in g (g_k = 1 / a_kk), or flags a bad pivot; k_gj_update
// writes every entry, row k from g and row i != k as (j == k ? 0 : a_ij) -
// f_i g_j, the expressions of k_gauss_jordan.  Both return at once once the
// flag is set.
__global__ __launch_bounds__(kSetupBs) void k_gj_pivot(const double* __restrict__ M, int n, int k,
                                                      double* __restrict__ f, double* __restrict__ g, int* bad) {
    if (*bad) return;
    const double piv = M[(size_t)k * n + k];
    if (!(piv > 0.0) || !isfinite(piv)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *bad = 1;
        return;
    }
    FV_GRID_LOOP(i, n) {
        f[i] = M[(size_t)i * n + k];
        g[i] = (i == k ? 1.0 : M[(size_t)k * n + i]) / piv;
    }
}

__global__ __launch_bounds__(kSetupBs) void k_gj_update(double* __restrict__ M, int n, int k,
                                                       const double* __restrict__ f, const double* __restrict__ g,
                                                       const int* bad) {
    if (*bad) return;
    FV_GRID_LOOP(e, (long long)n * n) {
        const int i = (int)(e / n), j = (int)(e - (long long)i * n);
        M[e] = i == k ? g[j] : (j == k ? 0.0 : M[e]) - f[i] * g[j];
    }
}
constexpr int kGjGridMin = 256;  // last levels from this size use the grid-wide elimination

// ---------------------------------------------------------------- host side

// A level's operator as CSR on the device (not owned).
struct CsrView {
    int n = 0, m = 0;
    long long nnz = 0;
    const int* ptr = nullptr;
    const int* col = nullptr;
    const double* val = nullptr;
};

// Owned CSR result of a product.
struct CsrOut {
    int n = 0, m = 0;
    long long nnz = 0;
    int *ptr = nullptr, *col = nullptr;
    double* val = nullptr;
    void release() {
        dev_free(ptr);
        dev_free(col);
        dev_free(val);
    }
};

// Rows per LDS workgroup for rows of at most m entries of 12 bytes each (0:
// the rows do not fit, use device memory).
void lds_fit(int m, int* lcap, int* per_wg) {
    *lcap = std::max(m, 1);
    *per_wg = std::min(kLdsBs, kLdsBytes / (12 * *lcap));
}

// The longest row of a CSR matrix, and lds_fit for it.
int lds_plan(const int* ptr, int rows, hipStream_t s, int* lcap, int* per_wg) {
    DevBuf<int> mx;
    int rc;
    if ((rc = mx.alloc(1, "row length maximum"))) return rc;
    FV_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_max_rowlen, dim3(grid1d(rows)), dim3(kSetupBs), 0, s, ptr, rows, mx.p);
    FV_LAUNCHED();
    int m = 0;
    if ((rc = read_scalar(&m, mx.p, s))) return rc;
    lds_fit(m, lcap, per_wg);
    return FVPCG_OK;
}

// Launch the product kernel a plan names: every output row i's distinct
// columns and sums at off[i] in (tcol, tval), and its count in cnt[i].
// Scratch (dense accumulators, device-memory heaps) is allocated here and
// freed after a synchronisation.
int spgemm_launch(const CsrView& X, const CsrView& Y, const ProdPlan& plan, const long long* off, int* tcol,
                  double* tval, int* cnt, hipStream_t s) {
    int rc;
    const int rows = X.n;
    DevBuf<double> dacc;
    DevBuf<uint8_t> dtouch;
    DevBuf<unsigned long long> heap;
    DevBuf<int> pos;
    switch (plan.mode) {
        case kProdDense:  // narrow product: dense rows, a wavefront each
            if ((rc = dacc.alloc((size_t)rows * std::max(Y.m, 1), "product accumulators")) ||
                (rc = dtouch.alloc((size_t)rows * std::max(Y.m, 1), "product flags")))
                return rc;
            hipLaunchKernelGGL(k_gemm_dense, dim3((unsigned)std::min(rows, 65536)), dim3(64), 0, s, X.ptr, X.col,
                               X.val, Y.ptr, Y.col, Y.val, rows, Y.m, off, dacc.p, dtouch.p, tcol, tval, cnt);
            break;
        case kProdTiled:  // long rows: LDS column tiles
            hipLaunchKernelGGL(k_gemm_tiled, dim3((unsigned)std::min(rows, 65536)), dim3(64), 0, s, X.ptr, X.col,
                               X.val, Y.ptr, Y.col, Y.val, rows, off, tcol, tval, cnt);
            break;
        case kProdShort:  // rows of X of at most kShortLists entries
            hipLaunchKernelGGL(k_gemm_short<kShortLists>, dim3(grid1d(rows)), dim3(kSetupBs), 0, s, X.ptr, X.col,
                               X.val, Y.ptr, Y.col, Y.val, rows, off, tcol, tval, cnt);
            break;
        case kProdMergeLds: {
            const long long blocks = ((long long)rows + plan.per_wg - 1) / plan.per_wg;
            hipLaunchKernelGGL(k_gemm_merge_lds<unsigned long long>, dim3((unsigned)std::max(blocks, 1LL)),
                               dim3(kLdsBs), (size_t)plan.per_wg * plan.lcap * 12, s, X.ptr, X.col, X.val, Y.ptr,
                               Y.col, Y.val, rows, plan.per_wg, plan.lcap, off, tcol, tval, cnt);
            break;
        }
        case kProdMergeLds32: {  // 32-bit heap keys: 8 bytes of LDS per list, more rows per CU
            const long long blocks = ((long long)rows + plan.per_wg - 1) / plan.per_wg;
            hipLaunchKernelGGL(k_gemm_merge_lds<unsigned int>, dim3((unsigned)std::max(blocks, 1LL)), dim3(kLdsBs),
                               (size_t)plan.per_wg * plan.lcap * 8, s, X.ptr, X.col, X.val, Y.ptr, Y.col, Y.val,
                               rows, plan.per_wg, plan.lcap, off, tcol, tval, cnt);
            break;
        }
        default:
            if ((rc = heap.alloc((size_t)std::max(X.nnz, 1LL), "product heaps")) ||
                (rc = pos.alloc((size_t)std::max(X.nnz, 1LL), "product positions")))
                return rc;
            hipLaunchKernelGGL(k_gemm_merge, dim3(grid1d(rows)), dim3(kSetupBs), 0, s, X.ptr, X.col, X.val, Y.ptr,
                               Y.col, Y.val, rows, off, heap.p, pos.p, tcol, tval, cnt);
            break;
    }
    FV_LAUNCHED();
    if (dacc.p || heap.p) FV_HIP(hipStreamSynchronize(s));  // their scratch is freed on return
    return FVPCG_OK;
}

// C = X Y (rows of X, columns of Y); C's arrays are allocated here, and the
// kernel chosen is recorded in *plan.
int spgemm(const CsrView& X, const CsrView& Y, CsrOut& C, hipStream_t s, ProdPlan* plan) {
    int rc;
    const int rows = X.n;
    DevBuf<long long> ub, off;
    DevBuf<int> cnt, mx;
    if ((rc = ub.alloc((size_t)rows, "product bounds")) || (rc = off.alloc((size_t)rows + 1, "product offsets")) ||
        (rc = cnt.alloc((size_t)rows + 1, "product counts")) || (rc = mx.alloc(1, "row length maximum")))
        return rc;
    FV_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_gemm_bound, dim3(grid1d(rows)), dim3(kSetupBs), 0, s, X.ptr, X.col, Y.ptr, rows, ub.p,
                       mx.p);
    FV_LAUNCHED();
    if ((rc = scan_excl<long long>(ub.p, off.p, rows, s))) return rc;
    long long total = 0;
    if ((rc = read_scalar(&total, off.p + rows, s))) return rc;
    DevBuf<int> tcol;
    DevBuf<double> tval;
    if ((rc = tcol.alloc((size_t)std::max(total, 1LL), "product columns")) ||
        (rc = tval.alloc((size_t)std::max(total, 1LL), "product values")))
        return rc;
    int lcap = 0, per_wg = 0, mlen = 0;
    if ((rc = read_scalar(&mlen, mx.p, s))) return rc;
    lds_fit(mlen, &lcap, &per_wg);
    // Kernel choice: dense rows for narrow products, LDS column tiles for
    // long rows, list heads in registers for rows of X of at most
    // kShortLists entries, else the heap merge (32-bit keys where they
    // fit).  FVPCG_AMG_PRODUCT = merge | merge32 | tiled | dense | short
    // forces one where it applies (all give the same sums); tests use it.
    const char* force = getenv("FVPCG_AMG_PRODUCT");
    const std::string fk = force ? force : "";
    const bool dense_ok = (long long)rows * Y.m <= kDenseEntries, tiled_ok = mlen <= kTileMaxLists;
    const bool use_dense = dense_ok && (fk.empty() || fk == "dense");
    const bool use_tiled = !use_dense && tiled_ok &&
                           (fk == "tiled" || (fk.empty() && (total >= kTileMinWork * (long long)rows || per_wg < 1)));
    const bool use_short = !use_dense && !use_tiled && mlen <= kShortLists && (fk.empty() || fk == "short");
    // the LDS merge with 32-bit keys where the lists and columns fit them:
    // 8 instead of 12 bytes of LDS per list, so more rows share a CU
    const int per_wg32 = std::min(kLdsBs, kLdsBytes / (8 * lcap));
    const bool use_k32 = !use_dense && !use_tiled && !use_short && per_wg >= 1 && mlen <= kKey32Lists &&
                         Y.m < kKey32Cols && (fk.empty() || fk == "merge32");
    plan->mode = use_dense ? kProdDense
                 : use_tiled ? kProdTiled
                 : use_short ? kProdShort
                 : use_k32 ? kProdMergeLds32
                 : per_wg >= 1 ? kProdMergeLds
                               : kProdMerge;
    plan->lcap = lcap;
    plan->per_wg = use_k32 ? per_wg32 : per_wg;
    if ((rc = spgemm_launch(X, Y, *plan, off.p, tcol.p, tval.p, cnt.p, s))) return rc;
    C.n = rows;
    C.m = Y.m;
    if ((rc = dev_alloc(&C.ptr, (size_t)rows + 1, "product row pointers"))) return rc;
    // counts fit in int: a row's distinct columns are at most Y.m
    if ((rc = scan_excl<int>(cnt.p, C.ptr, rows, s))) return rc;
    int nnz = 0;
    if ((rc = read_scalar(&nnz, C.ptr + rows, s))) return rc;
    if (nnz < 0) return set_error(FVPCG_UNSUPPORTED, "AMG: a coarse operator exceeds 2^31 entries");
    C.nnz = nnz;
    if ((rc = dev_alloc(&C.col, (size_t)std::max(nnz, 1), "product columns")) ||
        (rc = dev_alloc(&C.val, (size_t)std::max(nnz, 1), "product values")))
        return rc;
    const double avg = (double)nnz / (double)std::max(rows, 1);
    if (avg <= 5.0)
        hipLaunchKernelGGL(k_gemm_compact<4>, dim3(grid1d(4LL * rows)), dim3(kSetupBs), 0, s, rows, off.p, cnt.p,
                           C.ptr, tcol.p, tval.p, C.col, C.val);
    else if (avg <= 12.0)
        hipLaunchKernelGGL(k_gemm_compact<8>, dim3(grid1d(8LL * rows)), dim3(kSetupBs), 0, s, rows, off.p, cnt.p,
                           C.ptr, tcol.p, tval.p, C.col, C.val);
    else
        hipLaunchKernelGGL(k_gemm_compact<16>, dim3(grid1d(16LL * rows)), dim3(kSetupBs), 0, s, rows, off.p, cnt.p,
                           C.ptr, tcol.p, tval.p, C.col, C.val);
    FV_LAUNCHED();
    FV_HIP(hipStreamSynchronize(s));  // the scratch buffers are freed on return
    return FVPCG_OK;
}

// C's values for new values of X and Y with the patterns unchanged: C's
// pattern is then unchanged too (every product's column set depends on the
// patterns only), so the planned kernel writes each row straight into C at
// its row offsets (off64: C's row pointers widened); the columns it writes
// are the ones C already holds.
int spgemm_numeric(const CsrView& X, const CsrView& Y, int* ccol, double* cval, const long long* off64,
                   const ProdPlan& plan, hipStream_t s) {
    DevBuf<int> cnt;
    int rc;
    if ((rc = cnt.alloc((size_t)X.n + 1, "product counts"))) return rc;
    if ((rc = spgemm_launch(X, Y, plan, off64, ccol, cval, cnt.p, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// T = X^T, rows sorted by column
int transpose(const CsrView& X, CsrOut& T, hipStream_t s) {
    int rc;
    DevBuf<int> cnt, cursor;
    if ((rc = cnt.alloc((size_t)X.m + 1, "transpose counts")) || (rc = cursor.alloc((size_t)X.m, "transpose cursor")))
        return rc;
    FV_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * ((size_t)X.m + 1), s));
    FV_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int) * (size_t)std::max(X.m, 1), s));
    hipLaunchKernelGGL(k_col_count, dim3(grid1d(X.nnz)), dim3(kSetupBs), 0, s, X.col, X.nnz, cnt.p);
    FV_LAUNCHED();
    T.n = X.m;
    T.m = X.n;
    T.nnz = X.nnz;
    if ((rc = dev_alloc(&T.ptr, (size_t)X.m + 1, "transpose rows")) ||
        (rc = dev_alloc(&T.col, (size_t)std::max(X.nnz, 1LL), "transpose columns")) ||
        (rc = dev_alloc(&T.val, (size_t)std::max(X.nnz, 1LL), "transpose values")))
        return rc;
    if ((rc = scan_excl<int>(cnt.p, T.ptr, X.m, s))) return rc;
    hipLaunchKernelGGL(k_tr_scatter, dim3(grid1d(X.n)), dim3(kSetupBs), 0, s, X.ptr, X.col, X.val, X.n, T.ptr,
                       cursor.p, T.col, T.val);
    FV_LAUNCHED();
    int lcap = 0, per_wg = 0;
    if ((rc = lds_plan(T.ptr, T.n, s, &lcap, &per_wg))) return rc;
    if (per_wg >= 1) {
        const long long blocks = ((long long)T.n + per_wg - 1) / per_wg;
        hipLaunchKernelGGL(k_row_heapsort_lds, dim3((unsigned)std::max(blocks, 1LL)), dim3(kLdsBs),
                           (size_t)per_wg * lcap * 12, s, T.ptr, T.n, per_wg, lcap, T.col, T.val);
    } else {
        hipLaunchKernelGGL(k_row_heapsort, dim3(grid1d(T.n)), dim3(kSetupBs), 0, s, T.ptr, T.n, T.col, T.val);
    }
    FV_LAUNCHED();
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

CsrView view(const CsrOut& c) { return {c.n, c.m, c.nnz, c.ptr, c.col, c.val}; }

// The inverse of the last level (n at most kAmgMaxCoarse) into cinv (n x n,
// row-major) by Gauss-Jordan: one workgroup below kGjGridMin unknowns, one
// pair of grid-wide launches per pivot from there.
int invert_last(const CsrView& cur, double* cinv, int* bad, hipStream_t s) {
    int rc;
    const int nl = cur.n;
    DevBuf<double> f, g;
    if ((rc = f.alloc((size_t)nl, "AMG elimination column")) || (rc = g.alloc((size_t)nl, "AMG elimination row")))
        return rc;
    FV_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_dense_zero, dim3(grid1d((long long)nl * nl)), dim3(kSetupBs), 0, s, nl, cinv);
    hipLaunchKernelGGL(k_dense_fill, dim3(grid1d(nl)), dim3(kSetupBs), 0, s, cur.ptr, cur.col, cur.val, nl, cinv);
    if (nl < kGjGridMin) {
        hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(kGjBs), 0, s, cinv, nl, f.p, bad);
    } else {
        for (int k = 0; k < nl; ++k) {
            hipLaunchKernelGGL(k_gj_pivot, dim3(grid1d(nl)), dim3(kSetupBs), 0, s, cinv, nl, k, f.p, g.p, bad);
            hipLaunchKernelGGL(k_gj_update, dim3(grid1d((long long)nl * nl)), dim3(kSetupBs), 0, s, cinv, nl, k, f.p,
                               g.p, bad);
        }
    }
    FV_LAUNCHED();
    int hbad = 0;
    if ((rc = read_scalar(&hbad, bad, s))) return rc;
    if (hbad) return set_error(FVPCG_BREAKDOWN, "AMG: the last level is not positive definite");
    return FVPCG_OK;
}

// R = P^T's values for new values of P (the patterns kept): the entry
// (c, i) of R takes P's entry (i, c), found by a binary search in R's row c.
__global__ __launch_bounds__(kSetupBs) void k_tr_refresh(const int* __restrict__ pptr, const int* __restrict__ pcol,
                                                        const double* __restrict__ pval, int rows,
                                                        const int* __restrict__ rptr, const int* __restrict__ rcol,
                                                        double* __restrict__ rval) {
    FV_GRID_LOOP(i, rows) {
        for (int p = pptr[i]; p < pptr[i + 1]; ++p) {
            const int c = pcol[p];
            int lo = rptr[c], hi = rptr[c + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rcol[mid] < (int)i) lo = mid + 1;
                else hi = mid;
            }
            rval[lo] = pval[p];
        }
    }
}

// The aggregates of one level (agg: n entries, owned by the level); returns
// the aggregate count in *na.
// ell: level 0's slot layout (columns, values, W) for the rounds' maxima, or
// nullptr.
struct EllView {
    const int* col;
    const double* val;
    const double* d;
    int W;
};

int aggregate_level(const CsrView& A, const double* d, double theta, uint64_t seed, int level, int* agg, int* na,
                    const EllView* ell, hipStream_t s) {
    int rc;
    const int n = A.n;
    DevBuf<uint8_t> strong;
    DevBuf<uint64_t> key, m1, m2;
    DevBuf<int> counter, flags, rank, agg1;
    if ((rc = strong.alloc((size_t)std::max(A.nnz, 1LL), "AMG strength")) ||
        (rc = key.alloc((size_t)n, "AMG keys")) || (rc = m1.alloc((size_t)n, "AMG key maxima")) ||
        (rc = m2.alloc((size_t)n, "AMG key maxima")) || (rc = counter.alloc(2, "AMG counters")))
        return rc;
    const int g = grid1d(n);
    hipLaunchKernelGGL(k_strength, dim3(g), dim3(kSetupBs), 0, s, A.ptr, A.col, A.val, d, n, theta, strong.p);
    hipLaunchKernelGGL(k_mis_init, dim3(g), dim3(kSetupBs), 0, s, n, seed, level, key.p);
    FV_LAUNCHED();
    DevBuf<uint8_t> strong_ell;
    if (ell) {
        if ((rc = strong_ell.alloc((size_t)ell->W * n, "AMG slot strength"))) return rc;
        hipLaunchKernelGGL(k_strength_ell, dim3(g), dim3(kSetupBs), 0, s, ell->col, ell->val, ell->d, n, ell->W,
                           theta, strong_ell.p);
        FV_LAUNCHED();
    }
    const double avg_row = (double)A.nnz / (double)std::max(n, 1);
    int left = 1, rounds = 0;
    while (left > 0) {
        if (++rounds > kMaxMisRounds)
            return set_error(FVPCG_DEVICE_ERROR, "AMG: the independent set did not settle in %d rounds", kMaxMisRounds);
        FV_HIP(hipMemsetAsync(counter.p, 0, sizeof(int), s));
        if (ell) {
            hipLaunchKernelGGL(k_mis_max_ell, dim3(g), dim3(kSetupBs), 0, s, ell->col, strong_ell.p, n, ell->W,
                               key.p, m1.p);
            hipLaunchKernelGGL(k_mis_max_ell, dim3(g), dim3(kSetupBs), 0, s, ell->col, strong_ell.p, n, ell->W,
                               m1.p, m2.p);
        } else if (avg_row > 6.0) {
            hipLaunchKernelGGL(k_mis_max_g<16>, dim3(mis_group_grid(n, 16)), dim3(kSetupBs), 0, s, A.ptr, A.col,
                               strong.p, n, key.p, m1.p);
            hipLaunchKernelGGL(k_mis_max_g<16>, dim3(mis_group_grid(n, 16)), dim3(kSetupBs), 0, s, A.ptr, A.col,
                               strong.p, n, m1.p, m2.p);
        } else {
            hipLaunchKernelGGL(k_mis_max, dim3(g), dim3(kSetupBs), 0, s, A.ptr, A.col, strong.p, n, key.p, m1.p);
            hipLaunchKernelGGL(k_mis_max, dim3(g), dim3(kSetupBs), 0, s, A.ptr, A.col, strong.p, n, m1.p, m2.p);
        }
        hipLaunchKernelGGL(k_mis_decide, dim3(g), dim3(kSetupBs), 0, s, n, key.p, m2.p, counter.p);
        FV_LAUNCHED();
        if ((rc = read_scalar(&left, counter.p, s))) return rc;
    }
    if ((rc = flags.alloc((size_t)n, "AMG root flags")) || (rc = rank.alloc((size_t)n + 1, "AMG root ranks")) ||
        (rc = agg1.alloc((size_t)n, "AMG round-1 aggregates")))
        return rc;
    hipLaunchKernelGGL(k_root_flags, dim3(g), dim3(kSetupBs), 0, s, n, key.p, flags.p);
    FV_LAUNCHED();
    if ((rc = scan_excl<int>(flags.p, rank.p, n, s))) return rc;
    if ((rc = read_scalar(na, rank.p + n, s))) return rc;
    hipLaunchKernelGGL(k_agg_round1, dim3(g), dim3(kSetupBs), 0, s, A.ptr, A.col, strong.p, n, key.p, rank.p, agg1.p);
    FV_HIP(hipMemsetAsync(counter.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_agg_round2, dim3(g), dim3(kSetupBs), 0, s, A.ptr, A.col, A.val, strong.p, n, agg1.p, agg,
                       counter.p);
    FV_LAUNCHED();
    int missing = 0;
    if ((rc = read_scalar(&missing, counter.p, s))) return rc;
    if (missing) return set_error(FVPCG_DEVICE_ERROR, "AMG: an unknown was left out of every aggregate");
    return FVPCG_OK;
}

}  // namespace

int amg_build(fvpcg_amg* h, const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, uint64_t seed,
              hipStream_t s) {
    int rc;
    const fvpcg_mesh* msh = A->mesh;
    const int n0 = msh->n, W = msh->W;
    h->generation = A->generation;
    max_levels = std::max(1, std::min(max_levels, kAmgMaxLevels));
    // level 0 as CSR (freed once level 1 exists; the cycle uses the ELL layout)
    CsrOut A0;
    struct Release {
        CsrOut* c;
        ~Release() { c->release(); }
    } rel0{&A0};
    {
        DevBuf<int> cnt;
        if ((rc = cnt.alloc((size_t)n0, "level-0 row lengths"))) return rc;
        hipLaunchKernelGGL(k_l0_count, dim3(grid1d(n0)), dim3(kSetupBs), 0, s, msh->col, n0, W, cnt.p);
        FV_LAUNCHED();
        if ((rc = dev_alloc(&A0.ptr, (size_t)n0 + 1, "level-0 rows"))) return rc;
        if ((rc = scan_excl<int>(cnt.p, A0.ptr, n0, s))) return rc;
        int nnz = 0;
        if ((rc = read_scalar(&nnz, A0.ptr + n0, s))) return rc;
        A0.n = A0.m = n0;
        A0.nnz = nnz;
        if ((rc = dev_alloc(&A0.col, (size_t)std::max(nnz, 1), "level-0 columns")) ||
            (rc = dev_alloc(&A0.val, (size_t)std::max(nnz, 1), "level-0 values")))
            return rc;
        hipLaunchKernelGGL(k_l0_fill, dim3(grid1d(n0)), dim3(kSetupBs), 0, s, msh->col, A->val, A->d, n0, W, A0.ptr,
                           A0.col, A0.val);
        FV_LAUNCHED();
        FV_HIP(hipStreamSynchronize(s));
    }
    CsrView cur = view(A0);
    DevBuf<double> d0;  // level 0's diagonal as the CSR holds it
    DevBuf<unsigned long long> rho_bits;
    DevBuf<int> bad;
    if ((rc = rho_bits.alloc(1, "AMG spectral bound")) || (rc = bad.alloc(1, "AMG flag"))) return rc;
    double th = theta;
    int l = 0;
    for (;;) {
        AmgLevel& v = h->lev[l];
        v.n = cur.n;
        v.nnz = cur.nnz;
        double* d = nullptr;
        if (l == 0) {
            if ((rc = d0.alloc((size_t)cur.n, "AMG level diagonal"))) return rc;
            d = d0.p;
        } else {
            if ((rc = dev_alloc(&v.d, (size_t)cur.n, "AMG level diagonal"))) return rc;
            d = v.d;
        }
        FV_HIP(hipMemsetAsync(rho_bits.p, 0, sizeof(unsigned long long), s));
        FV_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_lvl_diag, dim3(grid1d(cur.n)), dim3(kSetupBs), 0, s, cur.ptr, cur.col, cur.val, cur.n, d,
                           rho_bits.p, bad.p);
        FV_LAUNCHED();
        unsigned long long rb = 0;
        int hbad = 0;
        if ((rc = read_scalar(&rb, rho_bits.p, s)) || (rc = read_scalar(&hbad, bad.p, s))) return rc;
        double rho;
        std::memcpy(&rho, &rb, sizeof(rho));
        if (hbad || !(rho > 0.0) || !std::isfinite(rho))
            return set_error(FVPCG_BREAKDOWN, "AMG: level %d has a diagonal entry that is not finite and positive", l);
        v.omega = 4.0 / (3.0 * rho);
        v.ga = lanes_for((size_t)cur.nnz, cur.n);
        if (l > 0) {
            if ((rc = dev_alloc(&v.a_val_cs, (size_t)std::max(cur.nnz, 1LL), "AMG level scaled values"))) return rc;
            hipLaunchKernelGGL(k_lvl_colscale, dim3(grid1d(cur.nnz)), dim3(kSetupBs), 0, s, cur.col, cur.val, d,
                               cur.nnz, v.a_val_cs);
            FV_LAUNCHED();
        }
        const size_t nv = (size_t)std::max(v.n, 1);
        if ((rc = dev_alloc(&v.b, nv, "AMG work")) || (rc = dev_alloc(&v.x, nv, "AMG work")) ||
            (rc = dev_alloc(&v.r, nv, "AMG work")) || (rc = dev_alloc(&v.y, nv, "AMG work")))
            return rc;
        if (cur.n <= coarse_size || l + 1 == max_levels) break;
        if ((rc = dev_alloc(&v.agg, (size_t)cur.n, "AMG aggregates"))) return rc;
        int na = 0;
        const EllView ell0{msh->col, A->val, A->d, W};
        if ((rc = aggregate_level(cur, d, th, seed, l, v.agg, &na, l == 0 ? &ell0 : nullptr, s))) return rc;
        if ((double)na > 0.6 * (double)cur.n) {  // aggregation no longer coarsens: this is the last level
            dev_free(v.agg);
            break;
        }
        // P = S P_t
        CsrOut P, R, AP, Ac;
        struct ReleaseAll {
            CsrOut* c[2];
            ~ReleaseAll() {
                for (CsrOut* x : c) x->release();
            }
        } relt{{&AP, &Ac}};
        {
            DevBuf<double> sval, ones;
            DevBuf<int> pt_ptr;
            if ((rc = sval.alloc((size_t)std::max(cur.nnz, 1LL), "AMG smoother rows")) ||
                (rc = ones.alloc((size_t)cur.n, "AMG tentative prolongator")) ||
                (rc = pt_ptr.alloc((size_t)cur.n + 1, "AMG tentative prolongator")))
                return rc;
            hipLaunchKernelGGL(k_smoother_rows, dim3(grid1d(cur.n)), dim3(kSetupBs), 0, s, cur.ptr, cur.col, cur.val,
                               d, cur.n, v.omega, sval.p);
            hipLaunchKernelGGL(k_tentative, dim3(grid1d((long long)cur.n + 1)), dim3(kSetupBs), 0, s, cur.n, pt_ptr.p,
                               ones.p);
            FV_LAUNCHED();
            const CsrView S{cur.n, cur.n, cur.nnz, cur.ptr, cur.col, sval.p};
            const CsrView Pt{cur.n, na, cur.n, pt_ptr.p, v.agg, ones.p};
            rc = spgemm(S, Pt, P, s, &v.plan_p);
            v.p_ptr = P.ptr;
            v.p_col = P.col;
            v.p_val = P.val;  // owned by the level from here on
            if (rc) return rc;
        }
        if ((rc = transpose(view(P), R, s))) {
            v.r_ptr = R.ptr;
            v.r_col = R.col;
            v.r_val = R.val;
            return rc;
        }
        v.r_ptr = R.ptr;
        v.r_col = R.col;
        v.r_val = R.val;
        if ((rc = spgemm(cur, view(P), AP, s, &v.plan_ap))) return rc;
        if ((rc = spgemm(view(R), view(AP), Ac, s, &v.plan_c))) return rc;
        // kept for the numeric refresh: A P, and the three products' row
        // offsets widened to 64 bits
        v.ap_ptr = AP.ptr;
        v.ap_col = AP.col;
        v.ap_val = AP.val;
        v.ap_nnz = AP.nnz;
        AP.ptr = nullptr;
        AP.col = nullptr;
        AP.val = nullptr;
        if ((rc = dev_alloc(&v.p_off, (size_t)cur.n + 1, "AMG product offsets")) ||
            (rc = dev_alloc(&v.ap_off, (size_t)cur.n + 1, "AMG product offsets")) ||
            (rc = dev_alloc(&v.c_off, (size_t)na + 1, "AMG product offsets")))
            return rc;
        hipLaunchKernelGGL(k_widen, dim3(grid1d((long long)cur.n + 1)), dim3(kSetupBs), 0, s, v.p_ptr, cur.n + 1,
                           v.p_off);
        hipLaunchKernelGGL(k_widen, dim3(grid1d((long long)cur.n + 1)), dim3(kSetupBs), 0, s, v.ap_ptr, cur.n + 1,
                           v.ap_off);
        hipLaunchKernelGGL(k_widen, dim3(grid1d((long long)na + 1)), dim3(kSetupBs), 0, s, Ac.ptr, na + 1, v.c_off);
        FV_LAUNCHED();
        v.nc = na;
        v.p_nnz = P.nnz;
        v.gp = lanes_for((size_t)P.nnz, P.n);
        v.gr = lanes_for((size_t)R.nnz, R.n);
        AmgLevel& next = h->lev[l + 1];
        next.a_ptr = Ac.ptr;
        next.a_col = Ac.col;
        next.a_val = Ac.val;
        Ac.ptr = nullptr;
        Ac.col = nullptr;
        Ac.val = nullptr;
        cur = CsrView{na, na, Ac.nnz, next.a_ptr, next.a_col, next.a_val};
        if (l == 0) d0.reset();  // level 0's CSR diagonal is no longer needed
        th *= 0.5;  // theta_l = theta / 2^l
        ++l;
    }
    h->nlev = l + 1;
    h->nlast = cur.n;
    if (cur.n > kAmgMaxCoarse)
        return set_error(FVPCG_UNSUPPORTED, "AMG: last level has %d unknowns (at most %d are solved exactly)", cur.n,
                         kAmgMaxCoarse);
    // the last level's inverse
    if (!h->cinv && (rc = dev_alloc(&h->cinv, (size_t)cur.n * cur.n, "AMG coarse inverse"))) return rc;
    if ((rc = invert_last(cur, h->cinv, bad.p, s))) return rc;
    // level 0's CSR is kept for the numeric refresh
    h->a0_ptr = A0.ptr;
    h->a0_col = A0.col;
    h->a0_val = A0.val;
    h->a0_nnz = A0.nnz;
    A0.ptr = nullptr;
    A0.col = nullptr;
    A0.val = nullptr;
    FV_HIP(hipStreamSynchronize(s));
    const size_t nn0 = (size_t)std::max(n0, 1);
    if ((rc = dev_alloc(&h->r, nn0, "AMG-PCG vectors")) || (rc = dev_alloc(&h->z, nn0, "AMG-PCG vectors")) ||
        (rc = dev_alloc(&h->p, nn0, "AMG-PCG vectors")) || (rc = dev_alloc(&h->q, nn0, "AMG-PCG vectors")) ||
        (rc = dev_alloc(&h->st, 1, "AMG-PCG state")) || (rc = dev_alloc(&h->partials, (size_t)4 * kMaxGrid, "partials")))
        return rc;
    if (hipHostMalloc((void**)&h->hst, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        h->hst = nullptr;
        return set_error(FVPCG_OUT_OF_MEMORY, "pinned allocation failed");
    }
    FV_HIP(hipMemsetAsync(h->st, 0, sizeof(DevState), s));
    hipEvent_t* evs[] = {&h->t_begin, &h->t_end, &h->t_it0, &h->t_it1};
    for (hipEvent_t* e : evs) FV_HIP(hipEventCreate(e));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

int amg_refresh(fvpcg_amg* h, hipStream_t s) {
    int rc;
    const fvpcg_matrix* A = h->mat;
    const fvpcg_mesh* msh = A->mesh;
    const int n0 = msh->n, W = msh->W;
    h->generation = kStaleGeneration;  // until the refresh completes
    // level 0's values into the kept CSR (the ELL pattern gives the same columns)
    hipLaunchKernelGGL(k_l0_fill, dim3(grid1d(n0)), dim3(kSetupBs), 0, s, msh->col, A->val, A->d, n0, W, h->a0_ptr,
                       h->a0_col, h->a0_val);
    FV_LAUNCHED();
    CsrView cur{n0, n0, h->a0_nnz, h->a0_ptr, h->a0_col, h->a0_val};
    DevBuf<double> d0;
    DevBuf<unsigned long long> rho_bits;
    DevBuf<int> bad;
    if ((rc = d0.alloc((size_t)n0, "AMG level diagonal")) || (rc = rho_bits.alloc(1, "AMG spectral bound")) ||
        (rc = bad.alloc(1, "AMG flag")))
        return rc;
    const int last = h->nlev - 1;
    for (int l = 0; l <= last; ++l) {
        AmgLevel& v = h->lev[l];
        double* d = l == 0 ? d0.p : v.d;
        FV_HIP(hipMemsetAsync(rho_bits.p, 0, sizeof(unsigned long long), s));
        FV_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_lvl_diag, dim3(grid1d(cur.n)), dim3(kSetupBs), 0, s, cur.ptr, cur.col, cur.val, cur.n, d,
                           rho_bits.p, bad.p);
        FV_LAUNCHED();
        unsigned long long rb = 0;
        int hbad = 0;
        if ((rc = read_scalar(&rb, rho_bits.p, s)) || (rc = read_scalar(&hbad, bad.p, s))) return rc;
        double rho;
        std::memcpy(&rho, &rb, sizeof(rho));
        if (hbad || !(rho > 0.0) || !std::isfinite(rho))
            return set_error(FVPCG_BREAKDOWN, "AMG: level %d has a diagonal entry that is not finite and positive", l);
        v.omega = 4.0 / (3.0 * rho);
        if (l > 0) {
            hipLaunchKernelGGL(k_lvl_colscale, dim3(grid1d(cur.nnz)), dim3(kSetupBs), 0, s, cur.col, cur.val, d,
                               cur.nnz, v.a_val_cs);
            FV_LAUNCHED();
        }
        if (l == last) break;
        {  // P = S P_t with the kept aggregates
            DevBuf<double> sval, ones;
            DevBuf<int> pt_ptr;
            if ((rc = sval.alloc((size_t)std::max(cur.nnz, 1LL), "AMG smoother rows")) ||
                (rc = ones.alloc((size_t)cur.n, "AMG tentative prolongator")) ||
                (rc = pt_ptr.alloc((size_t)cur.n + 1, "AMG tentative prolongator")))
                return rc;
            hipLaunchKernelGGL(k_smoother_rows, dim3(grid1d(cur.n)), dim3(kSetupBs), 0, s, cur.ptr, cur.col, cur.val,
                               d, cur.n, v.omega, sval.p);
            hipLaunchKernelGGL(k_tentative, dim3(grid1d((long long)cur.n + 1)), dim3(kSetupBs), 0, s, cur.n, pt_ptr.p,
                               ones.p);
            FV_LAUNCHED();
            const CsrView S{cur.n, cur.n, cur.nnz, cur.ptr, cur.col, sval.p};
            const CsrView Pt{cur.n, v.nc, cur.n, pt_ptr.p, v.agg, ones.p};
            if ((rc = spgemm_numeric(S, Pt, v.p_col, v.p_val, v.p_off, v.plan_p, s))) return rc;
        }
        hipLaunchKernelGGL(k_tr_refresh, dim3(grid1d(cur.n)), dim3(kSetupBs), 0, s, v.p_ptr, v.p_col, v.p_val, cur.n,
                           v.r_ptr, v.r_col, v.r_val);
        FV_LAUNCHED();
        const CsrView P{cur.n, v.nc, v.p_nnz, v.p_ptr, v.p_col, v.p_val};
        const CsrView R{v.nc, cur.n, v.p_nnz, v.r_ptr, v.r_col, v.r_val};
        const CsrView AP{cur.n, v.nc, v.ap_nnz, v.ap_ptr, v.ap_col, v.ap_val};
        AmgLevel& next = h->lev[l + 1];
        if ((rc = spgemm_numeric(cur, P, v.ap_col, v.ap_val, v.ap_off, v.plan_ap, s)) ||
            (rc = spgemm_numeric(R, AP, next.a_col, next.a_val, v.c_off, v.plan_c, s)))
            return rc;
        cur = CsrView{v.nc, v.nc, next.nnz, next.a_ptr, next.a_col, next.a_val};
    }
    if ((rc = invert_last(cur, h->cinv, bad.p, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    h->generation = A->generation;
    return FVPCG_OK;
}

}  // namespace fvpcg

