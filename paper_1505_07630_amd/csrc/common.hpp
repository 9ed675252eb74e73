// Internal definitions shared by the fvpcg HIP sources: handle layouts,
// launch geometry, device-side reductions and error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "fvpcg.h"

namespace fvpcg {

#ifndef FVPCG_BLOCK
#define FVPCG_BLOCK 256
#endif
constexpr int kBlock = FVPCG_BLOCK;   // threads per workgroup (wave64s)
constexpr int kWaves = kBlock / 64;
#ifndef FVPCG_MAX_GRID
#define FVPCG_MAX_GRID 256
#endif
constexpr int kMaxGrid = FVPCG_MAX_GRID;  // row-parallel workgroups per launch
constexpr int kMaxChunk = 64;         // iterations enqueued between convergence checks
// FP32 pipelined inner solve of the mixed solver: residual replacement period
// and the number of replacements without a new minimum that ends it.
constexpr int kReplaceEvery = 20;
constexpr int kStagnationChecks = 5;
// Reliable-update mixed solve: stop once the FP64 residual has had no new
// minimum for max(kReliableWindow, 10 * update period) FP32 iterations (CG
// residual norms are not monotone, so the window is long).
constexpr int kReliableWindow = 500;

// ---------------------------------------------------------------------------
// Solver scalars living in device memory.  Written only by the last
// workgroup of a reducing kernel (one thread), read by every workgroup of the
// next kernel on the stream.
struct alignas(128) DevState {
    double gamma;     // (r, M^-1 r) of the current iterate
    double delta;     // (p, A p) [standard] or (w, u) [pipelined]
    double rho;       // (r, r)
    double alpha;     // step of the next update
    double beta;      // direction coefficient of the next update
    double bnorm;     // ||b||
    double tol_abs;   // tol * ||b||
    double r0norm;    // ||r0||
    double true_rr;   // ||b - A x||^2 at exit
    double scale;     // mixed solver: ||r|| of the current outer residual
    double gamma_old; // gamma and alpha of the previous iteration (pipelined
    double alpha_old; //   recurrences, re-formed after a residual replacement)
    double best;      // smallest replaced (true) ||r||^2 so far
    double scale_prev; // mixed solver: ||r|| before the last correction
    int32_t no_min;   // replacements since the last new minimum
    int32_t iter;     // completed updates of x
    int32_t maxit;
    int32_t done;     // 1 once converged, out of iterations or broken down
    int32_t status;   // fvpcg_status
    int32_t zero_b;   // 1 if b == 0 (host writes x = 0)
    int32_t undo;     // mixed solver: the last correction increased ||r||
    uint32_t ticket;  // last-workgroup detection counter
    uint32_t pad1;
};

// Rows [blk*R, min(n, blk*R + R)) per workgroup; R is a multiple of 64.
struct Geom {
    int grid;
    int rows;
};

// Iterations to enqueue before the host next looks at a solver state.  The
// chunk doubles up to `cap`; once a state seen after `seen` iterations shows
// the residual norm below its initial one, the chunk is also capped by the
// iterations that the mean rate of decrease so far still needs to reach the
// target (10% margin, one more), less the `in_flight` iterations already
// enqueued after that state.  0: those in flight are expected to finish.
// Kernels launched after a solve has stopped return at once, so this only
// trades empty launches against host round trips; results do not depend on it.
inline int next_chunk(int chunk, int cap, double rnorm, double r0norm, double target, int seen, int in_flight) {
    const int grown = chunk * 2 < cap ? chunk * 2 : cap;
    if (!(seen >= 2 && target > 0.0 && rnorm > target && rnorm < r0norm)) return grown;
    const double rate = std::log(rnorm / r0norm) / (double)seen;  // < 0
    const double need = std::ceil(1.1 * std::log(target / rnorm) / rate) + 1.0;
    const double left = need - (double)in_flight;
    if (left <= 0.0) return 0;
    return left < (double)grown ? (int)left : grown;
}

inline Geom make_geom(int n, int max_grid = kMaxGrid) {
    if (n < 1) n = 1;
    int g = (n + kBlock - 1) / kBlock;
    if (g > max_grid) g = max_grid;
    int r = (n + g - 1) / g;
    r = (r + 63) / 64 * 64;
    g = (n + r - 1) / r;
    return {g, r};
}

// ---------------------------------------------------------------------------
// Handles.

struct fvpcg_mesh_impl;

struct Work;  // per-matrix solve workspace (solve.hip)

// ---------------------------------------------------------------------------
// Error reporting: thread-local message, return codes only.

int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define FV_HIP(expr)                                                       \
    do {                                                                   \
        hipError_t fv_e_ = (expr);                                         \
        if (fv_e_ != hipSuccess) return ::fvpcg::hip_fail(fv_e_, #expr, __FILE__, __LINE__); \
    } while (0)

#define FV_LAUNCHED()                                                      \
    do {                                                                   \
        hipError_t fv_e_ = hipGetLastError();                              \
        if (fv_e_ != hipSuccess) return ::fvpcg::hip_fail(fv_e_, "kernel launch", __FILE__, __LINE__); \
    } while (0)

template <typename T>
int dev_alloc(T** p, size_t count, const char* what) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(FVPCG_OUT_OF_MEMORY, "hipMalloc of %zu bytes for %s failed: %s", count * sizeof(T),
                         what, hipGetErrorString(e));
    }
    return FVPCG_OK;
}

template <typename T>
void dev_free(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// ---------------------------------------------------------------------------
// Device helpers.

// v from the lane K places lower in the same row of 16 lanes, 0 for the
// first K lanes of each row (DPP row_shr:K with bound_ctrl zero fill; the
// two 32-bit halves move separately).
template <int K>
__device__ __forceinline__ double row_shr(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x110 + K, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x110 + K, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a wave (all lanes active): an inclusive scan
// within each row of 16 lanes by DPP row shifts (ALU cross-lane moves, no LDS
// round trips), then the four row totals, read from lanes 15, 31, 47 and 63,
// added in that order.  Every lane returns the same, order-fixed sum.
__device__ __forceinline__ double wave_sum(double v) {
    v += row_shr<1>(v);
    v += row_shr<2>(v);
    v += row_shr<4>(v);
    v += row_shr<8>(v);
    return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// Sum NV values over a workgroup of BS threads; the result is valid in thread 0.
template <int BS, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    constexpr int kW = BS / 64;
    __shared__ double lds[NV][kW];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kW; ++w) s += lds[k][w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// One device-wide reduction in a single pass: each workgroup publishes its
// partial sums (layout [NV][G]) and takes a ticket; the workgroup that draws
// the last ticket sums all partials in a fixed order and returns true with
// the totals in thread 0's `tot`.  Deterministic for a given G.
template <int BS, int NV>
__device__ __forceinline__ bool device_reduce(double (&v)[NV], double* partials, uint32_t* ticket, int blk,
                                              int G, double (&tot)[NV]) {
    __shared__ int s_last;
    block_sum<BS, NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            __hip_atomic_store(&partials[(size_t)k * G + blk], v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == (uint32_t)(G - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < G; i += BS) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            acc[k] += __hip_atomic_load(&partials[(size_t)k * G + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<BS, NV>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = acc[k];
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// Loads and stores of data used once per kernel (matrix slots, the row's own
// vector entries): marked non-temporal so they do not evict the gathered
// neighbour values from L2.
#ifndef FVPCG_NT_LOADS
#define FVPCG_NT_LOADS 1
#endif
#ifndef FVPCG_NT_STORES
#define FVPCG_NT_STORES 1
#endif
template <typename T>
__device__ __forceinline__ T ld_once(const T* p) {
#if FVPCG_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
__device__ __forceinline__ void st_once(T* p, T v) {
#if FVPCG_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Tiles of BS rows handled by workgroup b of G (see FV_ROWS): b, b + G,
// b + 2G, ...
struct TileRange {
    int first, end, step;
};
template <int BS>
__device__ __forceinline__ TileRange block_tiles(int b, int G, int n) {
    return {b, (n + BS - 1) / BS, G};
}

}  // namespace fvpcg
