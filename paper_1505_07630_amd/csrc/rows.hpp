// Row-parallel building blocks shared by the solver kernels: the ELL slot
// gather, the interleaved tile loop, the layout dispatch and the per-solver
// workgroup geometry.
#pragma once

#include "handles.hpp"

namespace fvpcg {

// Column of slot (k, c): int32 column, or int16 offset from the row when the
// mesh's bandwidth fits (12 fewer bytes per hexahedral row per product).
__device__ __forceinline__ int slot_col(const int* p, size_t o, int) { return ld_once(p + o); }
__device__ __forceinline__ int slot_col(const int16_t* p, size_t o, int c) { return c + (int)ld_once(p + o); }

// The same with a plain (caching) load: for a kernel launched again and
// again whose slot columns, with its other small read-only arrays, fit in
// the chip's 256 MB last-level cache beside its gathered vector.
__device__ __forceinline__ int slot_col_keep(const int* p, size_t o, int) { return p[o]; }
__device__ __forceinline__ int slot_col_keep(const int16_t* p, size_t o, int c) { return c + (int)p[o]; }

// acc + sum_k val[k][c] * v[col[k][c]] over the WT slots of row c (KEEP:
// columns loaded with slot_col_keep).
template <typename T, int WT, typename CI, bool KEEP = false>
__device__ __forceinline__ T row_gather(const CI* __restrict__ col, const T* __restrict__ val, int n, int c,
                                        const T* __restrict__ v, T acc) {
    int j[WT];
    T a[WT];
#pragma unroll
    for (int k = 0; k < WT; ++k) {
        size_t o = (size_t)k * n + c;
        j[k] = KEEP ? slot_col_keep(col, o, c) : slot_col(col, o, c);
        a[k] = ld_once(val + o);
    }
#pragma unroll
    for (int k = 0; k < WT; ++k) acc += a[k] * v[j[k]];
    return acc;
}

// Tiles of BS rows (BS = the kernel's workgroup size), interleaved over the
// G workgroups: workgroup b takes tiles b, b + G, ..., so all G workgroups
// sweep the rows together, one window of G tiles at a time.  The hardware
// deals consecutive workgroups to the 8 XCDs in turn, so each XCD's L2 sees
// every eighth tile of the window; the neighbour values a row gathers from
// tiles another XCD owns come from the chip's last-level cache.  Measured on
// MI355X at 7.08M cells, this order is 3-7% faster for every row-parallel
// solver kernel than giving each XCD one contiguous band of tiles (which
// keeps the gathers in the XCD's own L2).
#define FV_ROWS(blk)                                                          \
    const int blk = (int)blockIdx.x;                                         \
    const TileRange tr_ = block_tiles<BS>(blk, g.grid, n);                   \
    for (int t_ = tr_.first; t_ < tr_.end; t_ += tr_.step)                   \
        for (int c = t_ * BS + (int)threadIdx.x; c < n && c < (t_ + 1) * BS; c += n)


// The tile loop of FV_ROWS with the slots of the thread's next row loaded
// before the current row is processed: the slot loads of one tile are in
// flight together with the own-row loads and neighbour gathers of the
// previous one, so a tile waits for one memory round trip instead of two
// (slots, then gathers).  Two slot buffers alternate (the loop is unrolled
// twice) so that no register holding a load in flight is copied, and the
// slots stay as loaded (int16 offsets unconverted) until the row uses them.
// The prefetch past the last tile reads row n - 1 again and is discarded.
// body(c, raw, a) handles row c; slot_abs(raw[k], c) is the column of slot k.
// Measured at 7.08M cells: it pays where a row gathers several vectors (the
// multi-component BiCGSTAB products, 5%) and costs 2-4% where it gathers one.
__device__ __forceinline__ int slot_abs(int raw, int) { return raw; }
__device__ __forceinline__ int slot_abs(int16_t raw, int c) { return c + (int)raw; }

template <typename T, int WT, typename CI>
__device__ __forceinline__ void load_slots_raw(const CI* __restrict__ col, const T* __restrict__ val, int n, int c,
                                               CI (&j)[WT], T (&a)[WT]) {
#pragma unroll
    for (int k = 0; k < WT; ++k) {
        const size_t o = (size_t)k * n + c;
        j[k] = ld_once(col + o);
        a[k] = ld_once(val + o);
    }
}

template <int BS, typename T, int WT, typename CI, typename Body>
__device__ __forceinline__ void rows_prefetched(const CI* __restrict__ col, const T* __restrict__ val, int n, Geom g,
                                                Body&& body) {
    const TileRange tr = block_tiles<BS>((int)blockIdx.x, g.grid, n);
    const int last = n - 1;
    int t = tr.first;
    CI ja[WT], jb[WT];
    T aa[WT], ab[WT];
    if (t >= tr.end) return;
    int c = t * BS + (int)threadIdx.x;
    load_slots_raw<T, WT, CI>(col, val, n, c < n ? c : last, ja, aa);
    for (;;) {
        int cn = (t + tr.step) * BS + (int)threadIdx.x;
        load_slots_raw<T, WT, CI>(col, val, n, cn < n ? cn : last, jb, ab);
        if (c < n) body(c, ja, aa);
        t += tr.step;
        if (t >= tr.end) break;
        c = cn;
        cn = (t + tr.step) * BS + (int)threadIdx.x;
        load_slots_raw<T, WT, CI>(col, val, n, cn < n ? cn : last, ja, aa);
        if (c < n) body(c, jb, ab);
        t += tr.step;
        if (t >= tr.end) break;
        c = cn;
    }
}

#define FV_WT_SWITCH(WT, ...)                                                        \
    switch (WT) {                                                                    \
        case 4: { constexpr int W_ = 4; __VA_ARGS__; } break;                        \
        case 6: { constexpr int W_ = 6; __VA_ARGS__; } break;                        \
        case 8: { constexpr int W_ = 8; __VA_ARGS__; } break;                        \
        case 16: { constexpr int W_ = 16; __VA_ARGS__; } break;                      \
        default: { constexpr int W_ = 32; __VA_ARGS__; } break;                      \
    }

// Dispatch on the mesh layout: W_ = slot count, CI_ = column type, cols_ =
// the column array (int16 offsets when the bandwidth fits, else int32).
#define FV_LAYOUT(M, ...)                                                            \
    if ((M)->col16) {                                                                \
        using CI_ = int16_t;                                                         \
        const CI_* cols_ = (M)->col16;                                               \
        (void)cols_;                                                                 \
        FV_WT_SWITCH((M)->WT, __VA_ARGS__);                                          \
    } else {                                                                         \
        using CI_ = int;                                                             \
        const CI_* cols_ = (M)->col;                                                 \
        (void)cols_;                                                                 \
        FV_WT_SWITCH((M)->WT, __VA_ARGS__);                                          \
    }

inline const void* mesh_cols(const fvpcg_mesh* m) {
    return m->col16 ? (const void*)m->col16 : (const void*)m->col;
}

// Workgroup size per solver (measured on MI355X at 7.08M cells: the fused
// pipelined iteration is fastest with 512-thread workgroups, the standard-CG
// and FP32 kernels with 1024) and the workgroup count (one per CU: each
// workgroup streams long runs of every array; more concurrent workgroups only
// add concurrent HBM streams).
#ifndef FVPCG_BS_PIPE
#define FVPCG_BS_PIPE 512
#endif
#ifndef FVPCG_BS_CG
#define FVPCG_BS_CG 1024
#endif
#ifndef FVPCG_BS_MIXED
#define FVPCG_BS_MIXED 1024
#endif
#ifndef FVPCG_BS_MISC
#define FVPCG_BS_MISC 512
#endif
constexpr int kBsPipe = FVPCG_BS_PIPE, kBsCg = FVPCG_BS_CG, kBsMixed = FVPCG_BS_MIXED, kBsMisc = FVPCG_BS_MISC;

inline Geom geom_for(int n, int bs) {
    if (n < 1) n = 1;
    int g = (n + bs - 1) / bs;
    if (g > kMaxGrid) g = kMaxGrid;
    return {g, bs};
}


// The pipelined recurrences' scalars, formed once by the workgroup that
// finishes the reduction: the stopping test on rho = (r, r), then
// beta = gamma / gamma_prev and alpha = gamma / (delta - beta gamma /
// alpha_prev) (first: beta = 0, alpha = gamma / delta), with breakdown when
// the denominator is not positive or a scalar is not finite.
__device__ __forceinline__ void pipe_scalars(DevState* st, double gamma, double delta, double rho, bool first) {
    if (first) {
        st->iter = 0;
        st->r0norm = sqrt(rho);
    } else {
        st->iter = st->iter + 1;
    }
    st->rho = rho;
    if (sqrt(rho) <= st->tol_abs) {
        st->done = 1;
        st->status = FVPCG_OK;
        return;
    }
    if (st->iter >= st->maxit) {
        st->done = 1;
        st->status = FVPCG_NOT_CONVERGED;
        return;
    }
    double beta, den;
    if (first) {
        beta = 0.0;
        den = delta;
    } else {
        beta = gamma / st->gamma;
        den = delta - beta * gamma / st->alpha;
    }
    const double alpha = gamma / den;
    if (!(den > 0.0) || !isfinite(den) || !isfinite(alpha) || !isfinite(beta)) {
        st->done = 1;
        st->status = FVPCG_BREAKDOWN;
        return;
    }
    st->gamma_old = st->gamma;
    st->alpha_old = st->alpha;
    st->gamma = gamma;
    st->delta = delta;
    st->alpha = alpha;
    st->beta = beta;
}

}  // namespace fvpcg
