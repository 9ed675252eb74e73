// Krylov solves on the device: the LDU/ELL matrix-vector product, standard
// preconditioned CG (Section 2: a sparse product, an optional
// preconditioner, three inner products and vector updates per iteration),
// the pipelined CG of Ghysels and Vanroose that the paper implements
// (Section 4.1: one reduction per iteration, overlapped with the product),
// the FP32/FP64 refinement and the adjoint gradients.
//
// Every row-parallel kernel walks tiles of its workgroup size, interleaved
// over the workgroups (FV_ROWS), one row per lane.
// Inner products are accumulated per thread in row order, then per wave
// (DPP scan), per workgroup (fixed order) and finally by the last workgroup
// over all workgroup partials in index order: results are bitwise
// reproducible for a given mesh.  The scalars of the recurrences (alpha,
// beta, the stopping test, breakdown) are computed once, by that last
// workgroup, and read by the next kernel from device memory; the host only
// reads the `done` flag back at chunk boundaries.
#include <climits>

#include <algorithm>

#include "handles.hpp"
#include <chrono>
#include <mutex>

#include "rows.hpp"

namespace fvpcg {

// ===========================================================================
// Row kernels' building blocks

// ===========================================================================
// y = A v

template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_spmv(const CI* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ d, int n, Geom g,
                                                 const double* __restrict__ v, double* __restrict__ y) {
    FV_ROWS(blk) { y[c] = row_gather<double, WT, CI>(col, val, n, c, v, d[c] * v[c]); }
}

// ||b - A x||^2 into st->true_rr (the true residual reported at exit).
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_true_residual(const CI* __restrict__ col, const double* __restrict__ val,
                                                          const double* __restrict__ d, int n, Geom g,
                                                          const double* __restrict__ b, const double* __restrict__ x,
                                                          DevState* st, double* partials) {
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        double r = b[c] - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        acc[0] += r * r;
    }
    double tot[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, tot) && threadIdx.x == 0) st->true_rr = tot[0];
}

// ===========================================================================
// Standard preconditioned CG

// r = b - A x, z = M^-1 r, p = z; gamma = (r,z), rho = (r,r), (b,b).
template <int BS, int WT, typename CI, bool JAC>
__global__ __launch_bounds__(BS) void k_cg_init(const CI* __restrict__ col, const double* __restrict__ val,
                                                    const double* __restrict__ d, int n, Geom g,
                                                    const double* __restrict__ b, const double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p, DevState* st,
                                                    double* partials) {
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        double bc = b[c];
        double dc = d[c];
        double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, dc * x[c]);
        double zc = JAC ? rc / dc : rc;
        r[c] = rc;
        p[c] = zc;
        acc[0] += rc * zc;
        acc[1] += rc * rc;
        acc[2] += bc * bc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const double bb = t[2];
        st->iter = 0;
        st->bnorm = sqrt(bb);
        if (bb == 0.0) {
            st->zero_b = 1;
            st->done = 1;
            st->status = FVPCG_OK;
            st->rho = 0.0;
            return;
        }
        st->tol_abs *= st->bnorm;
        st->gamma = t[0];
        st->rho = t[1];
        st->r0norm = sqrt(t[1]);
        if (st->r0norm <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (st->maxit <= 0) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// q = A p; delta = (p, q); alpha = gamma / delta.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_cg_spmv(const CI* __restrict__ col, const double* __restrict__ val,
                                                    const double* __restrict__ d, int n, Geom g,
                                                    const double* __restrict__ p, double* __restrict__ q, DevState* st,
                                                    double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        double pc = p[c];
        double qc = row_gather<double, WT, CI>(col, val, n, c, p, d[c] * pc);
        q[c] = qc;
        acc[0] += pc * qc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const double delta = t[0];
        st->delta = delta;
        if (!(delta > 0.0) || !isfinite(delta) || !isfinite(st->gamma)) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->alpha = st->gamma / delta;
    }
}

// r -= alpha q; z = M^-1 r; gamma' = (r, z), rho = (r, r); stopping test;
// beta = gamma' / gamma.
template <int BS, bool JAC>
__global__ __launch_bounds__(BS) void k_cg_update_r(double* __restrict__ r, const double* __restrict__ q,
                                                        const double* __restrict__ d, int n, Geom g, DevState* st,
                                                        double* partials) {
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    FV_ROWS(blk) {
        double rc = r[c] - alpha * q[c];
        r[c] = rc;
        double zc = JAC ? rc / d[c] : rc;
        acc[0] += rc * zc;
        acc[1] += rc * rc;
    }
    double t[2];
    if (device_reduce<BS, 2>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->rho = t[1];
        if (sqrt(t[1]) <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (it >= st->maxit) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        } else {
            st->beta = t[0] / st->gamma;
            st->gamma = t[0];
        }
    }
}

// x += alpha p (if iteration `it` updated r); p = z + beta p unless done.
template <int BS, bool JAC>
__global__ __launch_bounds__(BS) void k_cg_update_xp(double* __restrict__ x, double* __restrict__ p,
                                                         const double* __restrict__ r, const double* __restrict__ d,
                                                         int n, Geom g, int it, const DevState* st) {
    if (st->iter != it + 1) return;
    const double alpha = st->alpha, beta = st->beta;
    const bool more = !st->done;
    FV_ROWS(blk) {
        const double pc = p[c];
        x[c] += alpha * pc;
        if (more) {
            const double rc = r[c];
            const double zc = JAC ? rc / d[c] : rc;
            p[c] = zc + beta * pc;
        }
    }
}

// ===========================================================================
// Pipelined CG (Ghysels-Vanroose).  One kernel per iteration i does, per row:
//   nv = A m_i with m_i = M^-1 w_i (gathered from w_i; with Jacobi
//        A D^-1 w = w + sum_j (a_cj / d_j) w_j uses the column-scaled values)
//   z = nv + beta z;  s = w + beta s;  p = u + beta p;  [literal: q = m + beta q]
//   x += alpha p;  r -= alpha s;  w' = w - alpha z;   [literal: u -= alpha q]
// and the partial sums of gamma = (r,u), delta = (w',u), rho = (r,r) of
// the new iterate (folded: u = r/d).  w is double-buffered because
// neighbouring rows still gather w_i while w_{i+1} is written.  The last
// workgroup finishes the one reduction and forms alpha_{i+1}, beta_{i+1}:
//   beta = gamma / gamma_prev,
//   alpha = gamma / (delta - beta * gamma / alpha_prev).

template <typename T>
struct PipeVec {
    const void* col;  // int32 columns or int16 offsets (the kernel's CI)
    const T* val;  // column-scaled with Jacobi, plain otherwise
    const T* d;
    const T* w_in;
    T* w_out;
    T* z;
    T* s;
    T* p;
    T* x;
    T* r;
    T* u;  // literal only
    T* q;  // literal only
};


// r = b - A x; (b, b) -> bnorm and the absolute tolerance; clears the
// pipelined recurrences (z, s, p[, q]) and sets u = M^-1 r (literal).
template <int BS, int WT, typename CI, bool JAC, bool LIT>
__global__ __launch_bounds__(BS) void k_pipe_init_r(const CI* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ d, int n, Geom g,
                                                        const double* __restrict__ b, const double* __restrict__ x,
                                                        double* __restrict__ r, double* __restrict__ z,
                                                        double* __restrict__ s, double* __restrict__ p,
                                                        double* __restrict__ u, double* __restrict__ q, DevState* st,
                                                        double* partials) {
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        double bc = b[c];
        double dc = d[c];
        double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, dc * x[c]);
        r[c] = rc;
        z[c] = 0.0;
        s[c] = 0.0;
        p[c] = 0.0;
        if (LIT) {
            u[c] = JAC ? rc / dc : rc;
            q[c] = 0.0;
        }
        acc[0] += bc * bc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->iter = 0;
        st->bnorm = sqrt(t[0]);
        st->tol_abs *= st->bnorm;
        if (t[0] == 0.0) {
            st->zero_b = 1;
            st->done = 1;
            st->status = FVPCG_OK;
        }
    }
}

// w0 = A M^-1 r0 and the first reduction (gamma_0, delta_0, rho_0).
template <int BS, typename T, int WT, typename CI, bool JAC>
__global__ __launch_bounds__(BS) void k_pipe_init_w(const CI* __restrict__ col, const T* __restrict__ val,
                                                        const T* __restrict__ d, int n, Geom g,
                                                        const T* __restrict__ r, T* __restrict__ w, DevState* st,
                                                        double* partials) {
    if (st->done) return;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        T rc = r[c];
        T dc = d[c];
        T wc = row_gather<T, WT, CI>(col, val, n, c, r, JAC ? rc : dc * rc);
        w[c] = wc;
        T uc = JAC ? rc / dc : rc;
        acc[0] += (double)rc * (double)uc;
        acc[1] += (double)wc * (double)uc;
        acc[2] += (double)rc * (double)rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], true);
}

// FP64 folded form: x is needed only at exit, so it is updated every second
// iteration: on odd iterations x += alpha_{i-1} p_{i-1} + alpha_i p_i (p_{i-1}
// is read anyway; the two products are added in order, giving the same x as
// two separate updates); k_x_fixup adds a pending alpha_i p_i after an even
// last iteration.  Saves two vector passes every other iteration.
// d and the slot columns are read-only and re-read every launch; together
// with w (read and written every launch) they fit in the chip's 256 MB
// last-level cache at 7M cells, so they are loaded with caching loads and
// the other streams non-temporally (measured: 2-3% faster than all
// non-temporal; caching r or z or s as well is slower).
template <typename T, bool LIT>
struct PairX {
    static constexpr bool value = !LIT && sizeof(T) == 8;
};

template <int BS, typename T, int WT, typename CI, bool JAC, bool LIT>
__global__ __launch_bounds__(BS) void k_pipe_iter(PipeVec<T> a, int n, Geom g, DevState* st, double* partials) {
    if (st->done) return;
    constexpr bool PAIR = PairX<T, LIT>::value;
    const T alpha = (T)st->alpha, beta = (T)st->beta;
    const T alpha_prev = (T)st->alpha_old;
    const bool odd = (st->iter & 1) != 0;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const T wc = a.w_in[c];
        const T dc = a.d[c];
        const T nv = row_gather<T, WT, CI, true>((const CI*)a.col, a.val, n, c, a.w_in, JAC ? wc : dc * wc);
        const T zc = nv + beta * ld_once(a.z + c);
        const T sc = wc + beta * ld_once(a.s + c);
        T rc = ld_once(a.r + c);
        T uc;
        if (LIT) {
            const T mc = JAC ? wc / dc : wc;
            const T qc = mc + beta * ld_once(a.q + c);
            uc = ld_once(a.u + c);
            const T pc = uc + beta * ld_once(a.p + c);
            st_once(a.q + c, qc);
            st_once(a.p + c, pc);
            st_once(a.x + c, ld_once(a.x + c) + alpha * pc);
            uc -= alpha * qc;
            st_once(a.u + c, uc);
        } else {
            uc = JAC ? rc / dc : rc;
            const T pold = ld_once(a.p + c);
            const T pc = uc + beta * pold;
            st_once(a.p + c, pc);
            if (!PAIR) {
                st_once(a.x + c, ld_once(a.x + c) + alpha * pc);
            } else if (odd) {
                const T xa = ld_once(a.x + c) + alpha_prev * pold;
                st_once(a.x + c, xa + alpha * pc);
            }
        }
        rc -= alpha * sc;
        const T wn = wc - alpha * zc;
        st_once(a.z + c, zc);
        st_once(a.s + c, sc);
        st_once(a.r + c, rc);
        a.w_out[c] = wn;
        if (!LIT) uc = JAC ? rc / dc : rc;
        acc[0] += (double)rc * (double)uc;
        acc[1] += (double)wn * (double)uc;
        acc[2] += (double)rc * (double)rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], false);
}

// x += alpha p when the last pipelined iteration (an even one) left its
// update pending (see PairX).
template <int BS>
__global__ __launch_bounds__(BS) void k_x_fixup(double* __restrict__ x, const double* __restrict__ p, int n, Geom g,
                                                const DevState* st) {
    if ((st->iter & 1) == 0) return;
    const double alpha = st->alpha;
    FV_ROWS(blk) { x[c] += alpha * p[c]; }
}

// ===========================================================================
// Residual replacement for the FP32 pipelined inner solve: the recurrence
// vectors are re-formed from their definitions,
//   r = b - A x,  s = A p          (k_replace_rs)
//   w = A D^-1 r, z = A D^-1 s     (k_replace_wz, + the iteration's dots)
// and the scalars of the next update are formed again from the new dots and
// the previous iteration's gamma and alpha.  The inner solve ends once
// kStagnationChecks replacements in a row bring no new minimum of ||r||.

template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_replace_rs(const CI* __restrict__ col, const float* __restrict__ val,
                                                       const float* __restrict__ d, int n, Geom g,
                                                       const float* __restrict__ b, const float* __restrict__ x,
                                                       const float* __restrict__ p, float* __restrict__ r,
                                                       float* __restrict__ s, const DevState* st) {
    if (st->done) return;
    FV_ROWS(blk) {
        const float dc = d[c];
        r[c] = b[c] - row_gather<float, WT, CI>(col, val, n, c, x, dc * x[c]);
        s[c] = row_gather<float, WT, CI>(col, val, n, c, p, dc * p[c]);
    }
}

// RELIABLE: replacement within the reliable-update mixed solve (r comes from
// the FP64 residual; no stagnation or tolerance test here: the FP64 side
// decides, and `outer` done skips the kernel).
template <int BS, int WT, typename CI, bool RELIABLE>
__global__ __launch_bounds__(BS) void k_replace_wz(const CI* __restrict__ col, const float* __restrict__ val_cs,
                                                       const float* __restrict__ d, int n, Geom g,
                                                       const float* __restrict__ r, const float* __restrict__ s,
                                                       float* __restrict__ w, float* __restrict__ z, DevState* st,
                                                       const DevState* outer, double* partials) {
    if (st->done || (RELIABLE && outer->done)) return;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const float rc = r[c];
        const float wc = row_gather<float, WT, CI>(col, val_cs, n, c, r, rc);
        z[c] = row_gather<float, WT, CI>(col, val_cs, n, c, s, s[c]);
        w[c] = wc;
        const float uc = rc / d[c];
        acc[0] += (double)rc * (double)uc;
        acc[1] += (double)wc * (double)uc;
        acc[2] += (double)rc * (double)rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const double gamma = t[0], delta = t[1], rho = t[2];
        st->rho = rho;
        if (!RELIABLE) {
            if (rho < st->best) {
                st->best = rho;
                st->no_min = 0;
            } else if (++st->no_min >= kStagnationChecks) {
                st->done = 1;
                st->status = FVPCG_NOT_CONVERGED;
                return;
            }
            if (sqrt(rho) <= st->tol_abs) {
                st->done = 1;
                st->status = FVPCG_OK;
                return;
            }
        }
        const double beta = gamma / st->gamma_old;
        const double den = delta - beta * gamma / st->alpha_old;
        const double alpha = gamma / den;
        if (!(den > 0.0) || !isfinite(den) || !isfinite(alpha) || !isfinite(beta)) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->gamma = gamma;
        st->delta = delta;
        st->alpha = alpha;
        st->beta = beta;
    }
}

// ===========================================================================
// Mixed precision: FP64 residual and its norm, scaled FP32 right-hand side,
// FP64 correction.

// r = b - A x (FP64); outer stopping test on ||r||.  `j` = corrections so far.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_mixed_residual(const CI* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ d, int n, Geom g,
                                                           const double* __restrict__ b, const double* __restrict__ x,
                                                           double* __restrict__ r, int j, DevState* st,
                                                           double* partials) {
    double acc[2] = {0.0, 0.0};
    FV_ROWS(blk) {
        double bc = b[c];
        double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        r[c] = rc;
        acc[0] += rc * rc;
        acc[1] += bc * bc;
    }
    double t[2];
    if (device_reduce<BS, 2>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->iter = j;
        const double rn = sqrt(t[0]);
        const double prev = st->scale;
        st->scale_prev = prev;
        st->scale = rn;
        st->rho = t[0];
        st->true_rr = t[0];
        if (j == 0) {
            st->bnorm = sqrt(t[1]);
            st->tol_abs *= st->bnorm;
            st->r0norm = rn;
            if (t[1] == 0.0) {
                st->zero_b = 1;
                st->done = 1;
                st->status = FVPCG_OK;
                return;
            }
        }
        if (rn <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (!isfinite(rn)) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
        } else if (j > 0 && rn >= prev) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
            st->undo = 1;
        } else if (j >= st->maxit) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// r32 = fp32(r / ||r||), c = 0, recurrences cleared; inner ||rhs|| and
// inner absolute tolerance.
template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_cast(const double* __restrict__ r, int n, Geom g,
                                                       const DevState* st_out, float* __restrict__ r32,
                                                       float* __restrict__ b32, float* __restrict__ c32, float* __restrict__ z32,
                                                       float* __restrict__ s32, float* __restrict__ p32,
                                                       DevState* st_in, double* partials) {
    const double inv = 1.0 / st_out->scale;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        float v = (float)(r[c] * inv);
        r32[c] = v;
        b32[c] = v;
        c32[c] = 0.0f;
        z32[c] = 0.0f;
        s32[c] = 0.0f;
        p32[c] = 0.0f;
        acc[0] += (double)v * (double)v;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st_in->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st_in->iter = 0;
        st_in->bnorm = sqrt(t[0]);
        st_in->tol_abs *= st_in->bnorm;
    }
}

// x += ||r|| c; with `undo`, x -= ||r_prev|| c takes the last correction back.
template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_correct(double* __restrict__ x, const float* __restrict__ c32, int n,
                                                          Geom g, const DevState* st_out, int undo) {
    const double sc = undo ? -st_out->scale_prev : st_out->scale;
    FV_ROWS(blk) { x[c] += sc * (double)c32[c]; }
}

// ===========================================================================
// Mixed precision with reliable updates (residual replacement in the sense
// of van der Vorst and Ye, applied to the pipelined recurrences as by Cools
// et al.): the FP32 pipelined recurrences are never restarted; every K
// iterations the FP64 side accumulates x and recomputes b - A x, from which
// the FP32 r is re-formed, with s = A p (here) and w, z (k_replace_wz).

// x += scale * c; c = 0.
template <int BS>
__global__ __launch_bounds__(BS) void k_ru_accumulate(double* __restrict__ x, float* __restrict__ c32, int n, Geom g,
                                                          const DevState* so) {
    if (so->done) return;
    const double sc = so->scale;
    FV_ROWS(blk) {
        x[c] += sc * (double)c32[c];
        c32[c] = 0.0f;
    }
}

// r64 = b - A x with the FP64 matrix; r32 = fp32(r64 / scale); s32 = A32 p32,
// or, when the FP32 recurrences have stopped (breakdown), p32 = s32 = z32 = 0
// for a restart.  Outer tests on ||r64||: tolerance, non-finite, FP32
// iteration limit, no new minimum for `window` iterations.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_ru_residual(const CI* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ d, const float* __restrict__ val32,
                                                        const float* __restrict__ d32, int n, Geom g,
                                                        const double* __restrict__ b, const double* __restrict__ x,
                                                        float* __restrict__ r32, float* __restrict__ s32,
                                                        float* __restrict__ p32, float* __restrict__ z32,
                                                        DevState* so, const DevState* si, int it_offset, int maxit,
                                                        int window, int j, double* partials) {
    if (so->done) return;
    const double inv = 1.0 / so->scale;
    const bool restart = si->done != 0;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double rc = b[c] - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        r32[c] = (float)(rc * inv);
        if (restart) {
            s32[c] = 0.0f;
            p32[c] = 0.0f;
            z32[c] = 0.0f;
        } else {
            s32[c] = row_gather<float, WT, CI>(col, val32, n, c, p32, d32[c] * p32[c]);
        }
        acc[0] += rc * rc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &so->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const double rn = sqrt(t[0]);
        const int total = it_offset + si->iter;
        so->iter = j;
        so->rho = t[0];
        so->true_rr = t[0];
        if (rn <= so->tol_abs) {
            so->done = 1;
            so->status = FVPCG_OK;
        } else if (!isfinite(rn)) {
            so->done = 1;
            so->status = FVPCG_BREAKDOWN;
        } else if (total >= maxit) {
            so->done = 1;
            so->status = FVPCG_NOT_CONVERGED;
        } else {
            const double best = so->best < so->r0norm ? so->best : so->r0norm;
            if (rn < best) {
                so->best = rn;
                so->no_min = total;
            } else if (total - so->no_min >= window) {
                so->done = 1;
                so->status = FVPCG_NOT_CONVERGED;
            }
        }
    }
}

// ===========================================================================
// Adjoint gradients on the LDU pattern.

__global__ void k_grad_cells(const double* __restrict__ x, const double* __restrict__ lam, int n,
                             double* __restrict__ gd, double* __restrict__ gb) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        double l = lam[c];
        if (gd) gd[c] = -l * x[c];
        if (gb && gb != lam) gb[c] = l;
    }
}

__global__ void k_grad_faces(const int* __restrict__ owner, const int* __restrict__ nb, int F,
                             const double* __restrict__ x, const double* __restrict__ lam, double* __restrict__ gu,
                             double* __restrict__ gl, int sym) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) {
        const int o = owner[f], m = nb[f];
        const double up = -lam[o] * x[m];
        const double lo = -lam[m] * x[o];
        if (sym) {
            if (gu) gu[f] = up + lo;
        } else {
            if (gu) gu[f] = up;
            if (gl) gl[f] = lo;
        }
    }
}

// Reset a solver state on the device (the no-allocation path has no pinned
// host copy to send it from).
__global__ void k_state_reset(DevState* st, double tol_rel, int maxit) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState h = {};
    h.tol_abs = tol_rel;
    h.maxit = maxit;
    h.best = HUGE_VAL;
    h.status = FVPCG_NOT_CONVERGED;
    *st = h;
}

// ===========================================================================
// Host side

int work_init(Work& w, int n) {
    if (w.st) return FVPCG_OK;
    w.n = n;
    w.geom = make_geom(n);
    int rc;
    if ((rc = dev_alloc(&w.partials, (size_t)4 * kMaxGrid, "reduction partials"))) return rc;
    if ((rc = dev_alloc(&w.st, 2, "solver state"))) return rc;
    FV_HIP(hipMemset(w.st, 0, 2 * sizeof(DevState)));
    hipError_t e = hipHostMalloc((void**)&w.hst, 4 * sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess) {
        w.hst = nullptr;
        return set_error(FVPCG_OUT_OF_MEMORY, "pinned host allocation failed: %s", hipGetErrorString(e));
    }
    for (auto& ev : w.ev) FV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    FV_HIP(hipEventCreate(&w.t_begin));
    FV_HIP(hipEventCreate(&w.t_end));
    FV_HIP(hipEventCreate(&w.t_it0));
    FV_HIP(hipEventCreate(&w.t_it1));
    return FVPCG_OK;
}

int work_need_cg(Work& w) {
    if (w.have_cg) return FVPCG_OK;
    int rc;
    if (!w.r && (rc = dev_alloc(&w.r, (size_t)w.n, "r"))) return rc;
    if (!w.p && (rc = dev_alloc(&w.p, (size_t)w.n, "p"))) return rc;
    if (!w.q && (rc = dev_alloc(&w.q, (size_t)w.n, "q"))) return rc;
    w.have_cg = true;
    return FVPCG_OK;
}

int work_need_pipe(Work& w, bool literal) {
    int rc;
    if (!w.have_pipe) {
        if (!w.r && (rc = dev_alloc(&w.r, (size_t)w.n, "r"))) return rc;
        if (!w.p && (rc = dev_alloc(&w.p, (size_t)w.n, "p"))) return rc;
        if (!w.z && (rc = dev_alloc(&w.z, (size_t)w.n, "z"))) return rc;
        if (!w.s && (rc = dev_alloc(&w.s, (size_t)w.n, "s"))) return rc;
        if (!w.w[0] && (rc = dev_alloc(&w.w[0], (size_t)w.n, "w0"))) return rc;
        if (!w.w[1] && (rc = dev_alloc(&w.w[1], (size_t)w.n, "w1"))) return rc;
        w.have_pipe = true;
    }
    if (literal && !w.have_lit) {
        if (!w.u && (rc = dev_alloc(&w.u, (size_t)w.n, "u"))) return rc;
        if (!w.qq && (rc = dev_alloc(&w.qq, (size_t)w.n, "q"))) return rc;
        w.have_lit = true;
    }
    return FVPCG_OK;
}

int work_need_mixed(Work& w) {
    if (w.have_mixed) return FVPCG_OK;
    int rc;
    if (!w.r && (rc = dev_alloc(&w.r, (size_t)w.n, "r"))) return rc;
    if ((rc = dev_alloc(&w.r32, (size_t)w.n, "r32"))) return rc;
    if ((rc = dev_alloc(&w.r32b, (size_t)w.n, "b32"))) return rc;
    if ((rc = dev_alloc(&w.w32[0], (size_t)w.n, "w32a"))) return rc;
    if ((rc = dev_alloc(&w.w32[1], (size_t)w.n, "w32b"))) return rc;
    if ((rc = dev_alloc(&w.z32, (size_t)w.n, "z32"))) return rc;
    if ((rc = dev_alloc(&w.s32, (size_t)w.n, "s32"))) return rc;
    if ((rc = dev_alloc(&w.p32, (size_t)w.n, "p32"))) return rc;
    if ((rc = dev_alloc(&w.c32, (size_t)w.n, "c32"))) return rc;
    w.have_mixed = true;
    return FVPCG_OK;
}

void work_free(Work& w) {
    double* dv[] = {w.r, w.p, w.q, w.z, w.s, w.w[0], w.w[1], w.u, w.qq, w.lam, w.partials};
    for (double* p : dv)
        if (p) (void)hipFree(p);
    float* fv[] = {w.r32, w.r32b, w.w32[0], w.w32[1], w.z32, w.s32, w.p32, w.c32};
    for (float* p : fv)
        if (p) (void)hipFree(p);
    if (w.st) (void)hipFree(w.st);
    if (w.hst) (void)hipHostFree(w.hst);
    for (auto ev : w.ev)
        if (ev) (void)hipEventDestroy(ev);
    hipEvent_t te[] = {w.t_begin, w.t_end, w.t_it0, w.t_it1};
    for (auto ev : te)
        if (ev) (void)hipEventDestroy(ev);
    w = Work();
}

namespace {

// Reset the device state of slot `k` for a new solve.
int state_reset(Work& w, int k, double tol_rel, int maxit, hipStream_t s) {
    if (!w.hst) {
        hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, &w.st[k], tol_rel, maxit);
        FV_LAUNCHED();
        return FVPCG_OK;
    }
    DevState* h = &w.hst[2 + k];
    *h = DevState();
    h->tol_abs = tol_rel;
    h->maxit = maxit;
    h->best = HUGE_VAL;
    h->status = FVPCG_NOT_CONVERGED;
    FV_HIP(hipMemcpyAsync(&w.st[k], h, sizeof(DevState), hipMemcpyHostToDevice, s));
    return FVPCG_OK;
}

int state_read(Work& w, int k, DevState* out, hipStream_t s) {
    if (!w.hst) {  // no pinned mirror: copy into the caller's variable and wait
        FV_HIP(hipMemcpyAsync(out, &w.st[k], sizeof(DevState), hipMemcpyDeviceToHost, s));
        FV_HIP(hipStreamSynchronize(s));
        return FVPCG_OK;
    }
    FV_HIP(hipMemcpyAsync(&w.hst[k], &w.st[k], sizeof(DevState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    *out = w.hst[k];
    return FVPCG_OK;
}

// Both states (outer, inner) with one copy and one wait.
int state_read_both(Work& w, DevState* h0, DevState* h1, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(&w.hst[0], &w.st[0], 2 * sizeof(DevState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    *h0 = w.hst[0];
    *h1 = w.hst[1];
    return FVPCG_OK;
}

// Enqueue iterations in chunks; after each chunk the state is copied to
// pinned memory, and the previous chunk's copy is inspected while the current
// chunk runs.  Chunks grow geometrically and are capped by the iterations the
// residual's rate so far still needs (next_chunk); when the chunk in flight is
// expected to finish the solve, its state is waited for before anything more
// is enqueued.  Kernels launched after convergence return at once.  Without a
// pinned mirror (the no-allocation path) each chunk's state is read and
// waited for before the next chunk is enqueued.
template <typename Launch>
int iterate(Work& w, int k, int maxit, hipStream_t s, Launch&& launch_iter) {
    int launched = 0, chunk = 2, pending = -1, slot = 0;
    auto next = [&](const DevState& h, int in_flight) {
        return next_chunk(chunk, kMaxChunk, std::sqrt(h.rho), h.r0norm, h.tol_abs, h.iter, in_flight);
    };
    if (!w.hst) {
        while (launched < maxit) {
            const int cnt = chunk < maxit - launched ? chunk : maxit - launched;
            for (int i = 0; i < cnt; ++i) launch_iter(launched + i);
            FV_LAUNCHED();
            launched += cnt;
            DevState h;
            int rc = state_read(w, k, &h, s);
            if (rc) return rc;
            if (h.done) break;
            chunk = std::max(next(h, 0), 1);
        }
        return FVPCG_OK;
    }
    while (launched < maxit) {
        const int cnt = chunk < maxit - launched ? chunk : maxit - launched;
        for (int i = 0; i < cnt; ++i) launch_iter(launched + i);
        FV_LAUNCHED();
        launched += cnt;
        FV_HIP(hipMemcpyAsync(&w.hst[slot], &w.st[k], sizeof(DevState), hipMemcpyDeviceToHost, s));
        FV_HIP(hipEventRecord(w.ev[slot], s));
        if (pending < 0) {  // nothing to inspect yet
            if (launched == cnt) chunk = chunk * 2 < kMaxChunk ? chunk * 2 : kMaxChunk;
            pending = slot;
            slot ^= 1;
            continue;
        }
        FV_HIP(hipEventSynchronize(w.ev[pending]));
        const DevState& h = w.hst[pending];
        if (h.done) break;
        const int c = next(h, launched - h.iter);
        if (c > 0) {
            chunk = c;
            pending = slot;
            slot ^= 1;
            continue;
        }
        // the chunk in flight should end the solve: wait for it
        FV_HIP(hipEventSynchronize(w.ev[slot]));
        const DevState& g = w.hst[slot];
        if (g.done) break;
        chunk = std::max(next(g, 0), 1);
        pending = -1;
    }
    return FVPCG_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

}  // namespace

int spmv(const fvpcg_matrix* A, const double* v, double* y, hipStream_t s) {
    const fvpcg_mesh* m = A->mesh;
    const Geom gm = geom_for(m->n, kBsMisc);
    FV_LAYOUT(m, hipLaunchKernelGGL((k_spmv<kBsMisc, W_, CI_>), dim3(gm.grid), dim3(kBsMisc), 0, s, cols_, A->val, A->d, m->n,
                                           gm, v, y));
    FV_LAUNCHED();
    return FVPCG_OK;
}

namespace {

// HIP events on the stream when the work has them, else the host clock
// (after a synchronisation) for the no-allocation path.
struct Clock {
    Work& w;
    std::chrono::steady_clock::time_point h0, h1, h2;
    int mark(hipEvent_t e, std::chrono::steady_clock::time_point& t, hipStream_t s) {
        if (e) FV_HIP(hipEventRecord(e, s));
        else t = std::chrono::steady_clock::now();
        return FVPCG_OK;
    }
};

int solve_core(const fvpcg_matrix* A, Work& w, const double* b, double* x, double tol, int maxit, int method,
               int precond, hipStream_t s, fvpcg_stats* stats);

}  // namespace

int solve(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
          hipStream_t s, fvpcg_stats* stats) {
    Work& w = *A->work;
    int rc;
    if ((rc = work_init(w, A->mesh->n))) return rc;
    if (method == FVPCG_PIPECG_LITERAL && precond != FVPCG_PRECOND_JACOBI) method = FVPCG_PIPECG;
    if (method == FVPCG_CG) {
        if ((rc = work_need_cg(w))) return rc;
    } else {
        if ((rc = work_need_pipe(w, method == FVPCG_PIPECG_LITERAL))) return rc;
    }
    return solve_core(A, w, b, x, tol, maxit, method, precond, s, stats);
}

namespace {

int solve_core(const fvpcg_matrix* A, Work& w, const double* b, double* x, double tol, int maxit, int method,
               int precond, hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    const bool jac = precond == FVPCG_PRECOND_JACOBI;
    int rc;
    Clock clk{w, {}, {}, {}};
    const Geom gm = geom_for(n, kBsMisc), gc = geom_for(n, kBsCg), gp = geom_for(n, kBsPipe),
               gx = geom_for(n, kBsMixed);
    (void)gc; (void)gp; (void)gx; (void)gm;
    if (method == FVPCG_PIPECG_LITERAL && !jac) method = FVPCG_PIPECG;  // identical recurrences when M = I
    if ((rc = clk.mark(w.t_begin, clk.h0, s))) return rc;
    if ((rc = state_reset(w, 0, tol, maxit, s))) return rc;
    DevState* st = &w.st[0];
    double* part = w.partials;

    if (method == FVPCG_CG) {
        FV_LAYOUT(m,
                     if (jac) hipLaunchKernelGGL((k_cg_init<kBsCg, W_, CI_, true>), dim3(gc.grid), dim3(kBsCg), 0, s, cols_,
                                                 A->val, A->d, n, gc, b, x, w.r, w.p, st, part);
                     else hipLaunchKernelGGL((k_cg_init<kBsCg, W_, CI_, false>), dim3(gc.grid), dim3(kBsCg), 0, s, cols_, A->val,
                                             A->d, n, gc, b, x, w.r, w.p, st, part));
    } else {
        const bool lit = method == FVPCG_PIPECG_LITERAL;
        FV_LAYOUT(
            m,
            if (jac && lit) hipLaunchKernelGGL((k_pipe_init_r<kBsPipe, W_, CI_, true, true>), dim3(gp.grid), dim3(kBsPipe), 0, s,
                                               cols_, A->val, A->d, n, gp, b, x, w.r, w.z, w.s, w.p, w.u, w.qq, st,
                                               part);
            else if (jac) hipLaunchKernelGGL((k_pipe_init_r<kBsPipe, W_, CI_, true, false>), dim3(gp.grid), dim3(kBsPipe), 0, s,
                                             cols_, A->val, A->d, n, gp, b, x, w.r, w.z, w.s, w.p, w.u, w.qq, st,
                                             part);
            else hipLaunchKernelGGL((k_pipe_init_r<kBsPipe, W_, CI_, false, false>), dim3(gp.grid), dim3(kBsPipe), 0, s, cols_,
                                    A->val, A->d, n, gp, b, x, w.r, w.z, w.s, w.p, w.u, w.qq, st, part);
            if (jac) hipLaunchKernelGGL((k_pipe_init_w<kBsPipe, double, W_, CI_, true>), dim3(gp.grid), dim3(kBsPipe), 0, s, cols_,
                                        A->val_cs, A->d, n, gp, w.r, w.w[0], st, part);
            else hipLaunchKernelGGL((k_pipe_init_w<kBsPipe, double, W_, CI_, false>), dim3(gp.grid), dim3(kBsPipe), 0, s, cols_,
                                    A->val, A->d, n, gp, w.r, w.w[0], st, part));
    }
    FV_LAUNCHED();
    DevState h;
    if ((rc = state_read(w, 0, &h, s))) return rc;
    std::chrono::steady_clock::time_point t_it0;
    if ((rc = clk.mark(w.t_it0, t_it0, s))) return rc;
    if (h.zero_b) {
        FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    } else if (!h.done) {
        if (method == FVPCG_CG) {
            rc = iterate(w, 0, maxit, s, [&](int it) {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_cg_spmv<kBsCg, W_, CI_>), dim3(gc.grid), dim3(kBsCg), 0, s, cols_,
                                                       A->val, A->d, n, gc, w.p, w.q, st, part));
                if (jac) {
                    hipLaunchKernelGGL((k_cg_update_r<kBsCg, true>), dim3(gc.grid), dim3(kBsCg), 0, s, w.r, w.q, A->d, n, gc,
                                       st, part);
                    hipLaunchKernelGGL((k_cg_update_xp<kBsCg, true>), dim3(gc.grid), dim3(kBsCg), 0, s, x, w.p, w.r, A->d, n,
                                       gc, it, st);
                } else {
                    hipLaunchKernelGGL((k_cg_update_r<kBsCg, false>), dim3(gc.grid), dim3(kBsCg), 0, s, w.r, w.q, A->d, n, gc,
                                       st, part);
                    hipLaunchKernelGGL((k_cg_update_xp<kBsCg, false>), dim3(gc.grid), dim3(kBsCg), 0, s, x, w.p, w.r, A->d, n,
                                       gc, it, st);
                }
            });
        } else {
            const bool lit = method == FVPCG_PIPECG_LITERAL;
            rc = iterate(w, 0, maxit, s, [&](int it) {
                PipeVec<double> a{mesh_cols(m), jac ? A->val_cs : A->val, A->d, w.w[it & 1], w.w[(it + 1) & 1], w.z,
                                  w.s, w.p, x, w.r, w.u, w.qq};
                FV_LAYOUT(
                    m,
                    if (jac && lit) hipLaunchKernelGGL((k_pipe_iter<kBsPipe, double, W_, CI_, true, true>), dim3(gp.grid),
                                                       dim3(kBsPipe), 0, s, a, n, gp, st, part);
                    else if (jac) hipLaunchKernelGGL((k_pipe_iter<kBsPipe, double, W_, CI_, true, false>), dim3(gp.grid),
                                                       dim3(kBsPipe), 0, s, a, n, gp, st, part);
                    else hipLaunchKernelGGL((k_pipe_iter<kBsPipe, double, W_, CI_, false, false>), dim3(gp.grid), dim3(kBsPipe), 0,
                                            s, a, n, gp, st, part));
            });
        }
        if (rc) return rc;
    }
    if (method == FVPCG_PIPECG && !h.zero_b && !h.done) {
        hipLaunchKernelGGL((k_x_fixup<kBsPipe>), dim3(gp.grid), dim3(kBsPipe), 0, s, x, w.p, n, gp, st);
        FV_LAUNCHED();
    }
    std::chrono::steady_clock::time_point t_it1;
    if ((rc = clk.mark(w.t_it1, t_it1, s))) return rc;
    FV_LAYOUT(m, hipLaunchKernelGGL((k_true_residual<kBsMisc, W_, CI_>), dim3(gm.grid), dim3(kBsMisc), 0, s, cols_, A->val,
                                           A->d, n, gm, b, x, st, part));
    FV_LAUNCHED();
    if (w.t_end) FV_HIP(hipEventRecord(w.t_end, s));
    if ((rc = state_read(w, 0, &h, s))) return rc;
    if (!w.t_end) clk.h2 = std::chrono::steady_clock::now();
    if (stats) {
        stats->iters = h.iter;
        stats->outer_iters = 0;
        stats->status = h.status;
        stats->b_norm = h.bnorm;
        stats->r0_norm = h.r0norm;
        stats->rel_res = h.bnorm > 0 ? sqrt(h.rho) / h.bnorm : 0.0;
        stats->true_rel_res = h.bnorm > 0 ? sqrt(h.true_rr) / h.bnorm : 0.0;
        if (w.t_begin) {
            stats->device_ms = elapsed(w.t_begin, w.t_end);
            stats->iter_ms = elapsed(w.t_it0, w.t_it1);
        } else {  // host clock: the whole call, and from the first state read to the end
            stats->device_ms = std::chrono::duration<double, std::milli>(clk.h2 - clk.h0).count();
            stats->iter_ms = std::chrono::duration<double, std::milli>(clk.h2 - t_it0).count();
        }
    }
    return h.status;
}

}  // namespace

// ---------------------------------------------------------------------------
// The solve for callers that cannot allocate: every work buffer (the solver
// vectors, the reduction partials and the device state) lives in `scratch`,
// a file-scope device array each GPU holds once the library is loaded, sized
// for FVPCG_NOALLOC_MAX_CELLS cells.  Its address on the current device is
// looked up once per device (hipGetSymbolAddress; the array's name itself is
// a host-side stand-in) and passed to the kernels like any other buffer.
// Every call on one GPU shares the array: calls that overlap on a GPU race.
// vectors: r, p, z (standard CG's q), s, w0, w1, u, q (literal pipelined);
// standard CG uses r, p, q, the folded pipelined form the first six
constexpr int kNoAllocVectors = 8;
constexpr size_t kNoAllocStride = ((size_t)FVPCG_NOALLOC_MAX_CELLS + 63) / 64 * 64;
constexpr size_t kNoAllocStateDoubles = (2 * sizeof(DevState) + sizeof(double) - 1) / sizeof(double);
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocVectors * kNoAllocStride + 4 * (size_t)kMaxGrid +
                                   kNoAllocStateDoubles;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

int scratch_on_current_device(double** out) {
    int dev = 0;
    FV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(FVPCG_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        FV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return FVPCG_OK;
}
}  // namespace

int solve_noalloc(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
                  hipStream_t s, fvpcg_stats* stats) {
    const int n = A->mesh->n;
    if (n > FVPCG_NOALLOC_MAX_CELLS)
        return set_error(FVPCG_INVALID_ARG, "fvpcg_solve_noalloc: %d cells exceed its fixed work space of %d cells",
                         n, FVPCG_NOALLOC_MAX_CELLS);
    int dev = 0;
    FV_HIP(hipGetDevice(&dev));
    if (dev != A->mesh->device)
        return set_error(FVPCG_INVALID_ARG, "fvpcg_solve_noalloc: the current device (%d) is not the matrix's (%d)",
                         dev, A->mesh->device);
    double* base = nullptr;
    int rc;
    if ((rc = scratch_on_current_device(&base))) return rc;
    Work w;  // a view of the scratch array: no pinned mirror, no events
    w.n = n;
    w.geom = make_geom(n);
    double** vec[kNoAllocVectors] = {&w.r, &w.p, &w.z, &w.s, &w.w[0], &w.w[1], &w.u, &w.qq};
    for (int k = 0; k < kNoAllocVectors; ++k) *vec[k] = base + (size_t)k * kNoAllocStride;
    w.q = w.z;  // standard CG's q; the pipelined forms' z
    w.partials = base + (size_t)kNoAllocVectors * kNoAllocStride;
    w.st = reinterpret_cast<DevState*>(w.partials + 4 * (size_t)kMaxGrid);
    return solve_core(A, w, b, x, tol, maxit, method, precond, s, stats);
}

int solve_mixed(const fvpcg_matrix* A, const double* b, double* x, double outer_tol, double inner_tol, int max_outer,
                int max_inner, hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    Work& w = *A->work;
    int rc;
    if ((rc = work_init(w, n)) || (rc = work_need_mixed(w))) return rc;
    const Geom gm = geom_for(n, kBsMisc), gc = geom_for(n, kBsCg), gp = geom_for(n, kBsPipe),
               gx = geom_for(n, kBsMixed);
    (void)gc; (void)gp; (void)gx; (void)gm;
    FV_HIP(hipEventRecord(w.t_begin, s));
    if ((rc = state_reset(w, 0, outer_tol, max_outer, s))) return rc;
    DevState* so = &w.st[0];
    DevState* si = &w.st[1];
    double* part = w.partials;
    DevState h, hi;
    int inner_total = 0, j = 0;
    float iter_ms = 0.f;
    for (j = 0;; ++j) {
        FV_LAYOUT(m, hipLaunchKernelGGL((k_mixed_residual<kBsMixed, W_, CI_>), dim3(gx.grid), dim3(kBsMixed), 0, s, cols_,
                                               A->val, A->d, n, gx, b, x, w.r, j, so, part));
        FV_LAUNCHED();
        if ((rc = state_read(w, 0, &h, s))) return rc;
        if (h.undo) {
            hipLaunchKernelGGL((k_mixed_correct<kBsMixed>), dim3(gx.grid), dim3(kBsMixed), 0, s, x, w.c32, n, gx, so, 1);
            FV_LAUNCHED();
            h.scale = h.scale_prev;
        }
        if (h.done) break;
        if ((rc = state_reset(w, 1, inner_tol, max_inner, s))) return rc;
        FV_HIP(hipEventRecord(w.t_it0, s));
        hipLaunchKernelGGL((k_mixed_cast<kBsMixed>), dim3(gx.grid), dim3(kBsMixed), 0, s, w.r, n, gx, so, w.r32, w.r32b, w.c32, w.z32, w.s32,
                           w.p32, si, part);
        FV_LAYOUT(m, hipLaunchKernelGGL((k_pipe_init_w<kBsMixed, float, W_, CI_, true>), dim3(gx.grid), dim3(kBsMixed), 0, s,
                                               cols_, A->val32_cs, A->d32, n, gx, w.r32, w.w32[0], si, part));
        FV_LAUNCHED();
        rc = iterate(w, 1, max_inner, s, [&](int it) {
            PipeVec<float> a{mesh_cols(m), A->val32_cs, A->d32, w.w32[it & 1], w.w32[(it + 1) & 1], w.z32, w.s32,
                             w.p32, w.c32, w.r32, nullptr, nullptr};
            FV_LAYOUT(m, hipLaunchKernelGGL((k_pipe_iter<kBsMixed, float, W_, CI_, true, false>), dim3(gx.grid), dim3(kBsMixed),
                                                   0, s, a, n, gx, si, part));
            if ((it + 1) % kReplaceEvery == 0) {
                float* w_cur = w.w32[(it + 1) & 1];
                FV_LAYOUT(m,
                             hipLaunchKernelGGL((k_replace_rs<kBsMixed, W_, CI_>), dim3(gx.grid), dim3(kBsMixed), 0, s, cols_, A->val32,
                                                A->d32, n, gx, w.r32b, w.c32, w.p32, w.r32, w.s32, si);
                             hipLaunchKernelGGL((k_replace_wz<kBsMixed, W_, CI_, false>), dim3(gx.grid), dim3(kBsMixed), 0, s, cols_,
                                                A->val32_cs, A->d32, n, gx, w.r32, w.s32, w_cur, w.z32, si, nullptr, part));
            }
        });
        if (rc) return rc;
        hipLaunchKernelGGL((k_mixed_correct<kBsMixed>), dim3(gx.grid), dim3(kBsMixed), 0, s, x, w.c32, n, gx, so, 0);
        FV_LAUNCHED();
        FV_HIP(hipEventRecord(w.t_it1, s));
        if ((rc = state_read(w, 1, &hi, s))) return rc;
        iter_ms += elapsed(w.t_it0, w.t_it1);
        inner_total += hi.iter;
        if (hi.status == FVPCG_BREAKDOWN && hi.iter == 0) {
            FV_HIP(hipEventRecord(w.t_end, s));
            if ((rc = state_read(w, 0, &h, s))) return rc;
            h.status = FVPCG_BREAKDOWN;
            break;
        }
    }
    if (h.zero_b) FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    FV_HIP(hipEventRecord(w.t_end, s));
    FV_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = inner_total;
        stats->outer_iters = h.iter;
        stats->status = h.status;
        stats->b_norm = h.bnorm;
        stats->r0_norm = h.r0norm;
        stats->rel_res = h.bnorm > 0 ? h.scale / h.bnorm : 0.0;
        stats->true_rel_res = stats->rel_res;
        stats->device_ms = elapsed(w.t_begin, w.t_end);
        stats->iter_ms = iter_ms;
    }
    return h.status;
}

// Mixed precision with reliable updates.  Stats: iters = FP32 iterations,
// outer_iters = FP64 updates; status as the FP64 side decides it.
int solve_mixed_reliable(const fvpcg_matrix* A, const double* b, double* x, double tol, int update_every, int maxit,
                         hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    Work& w = *A->work;
    int rc;
    if ((rc = work_init(w, n)) || (rc = work_need_mixed(w))) return rc;
    const Geom gx = geom_for(n, kBsMixed);
    const int K = update_every;
    const int window = std::max(kReliableWindow, 10 * K);
    FV_HIP(hipEventRecord(w.t_begin, s));
    if ((rc = state_reset(w, 0, tol, INT_MAX, s)) || (rc = state_reset(w, 1, 0.0, maxit, s))) return rc;
    DevState* so = &w.st[0];
    DevState* si = &w.st[1];
    double* part = w.partials;
    DevState h, hi;
    // r = b - A x0, ||b||, scale = ||r0||; r32 = fp32(r / scale), c = z = s = p = 0
    FV_LAYOUT(m, hipLaunchKernelGGL((k_mixed_residual<kBsMixed, W_, CI_>), dim3(gx.grid), dim3(kBsMixed), 0, s, cols_,
                                    A->val, A->d, n, gx, b, x, w.r, 0, so, part));
    FV_LAUNCHED();
    if ((rc = state_read(w, 0, &h, s))) return rc;
    int offset = 0, updates = 0, wi = 0;
    FV_HIP(hipEventRecord(w.t_it0, s));
    if (!h.done) {
        hipLaunchKernelGGL((k_mixed_cast<kBsMixed>), dim3(gx.grid), dim3(kBsMixed), 0, s, w.r, n, gx, so, w.r32, w.r32b,
                           w.c32, w.z32, w.s32, w.p32, si, part);
        FV_LAYOUT(m, hipLaunchKernelGGL((k_pipe_init_w<kBsMixed, float, W_, CI_, true>), dim3(gx.grid), dim3(kBsMixed), 0,
                                        s, cols_, A->val32_cs, A->d32, n, gx, w.r32, w.w32[wi], si, part));
        FV_LAUNCHED();
        for (;;) {
            for (int k = 0; k < K; ++k) {
                PipeVec<float> a{mesh_cols(m), A->val32_cs, A->d32, w.w32[wi], w.w32[wi ^ 1], w.z32, w.s32, w.p32,
                                 w.c32, w.r32, nullptr, nullptr};
                FV_LAYOUT(m, hipLaunchKernelGGL((k_pipe_iter<kBsMixed, float, W_, CI_, true, false>), dim3(gx.grid),
                                                dim3(kBsMixed), 0, s, a, n, gx, si, part));
                wi ^= 1;
            }
            ++updates;
            hipLaunchKernelGGL((k_ru_accumulate<kBsMixed>), dim3(gx.grid), dim3(kBsMixed), 0, s, x, w.c32, n, gx, so);
            FV_LAYOUT(m, hipLaunchKernelGGL((k_ru_residual<kBsMixed, W_, CI_>), dim3(gx.grid), dim3(kBsMixed), 0, s,
                                            cols_, A->val, A->d, A->val32, A->d32, n, gx, b, x, w.r32, w.s32, w.p32,
                                            w.z32, so, si, offset, maxit, window, updates, part);
                         hipLaunchKernelGGL((k_replace_wz<kBsMixed, W_, CI_, true>), dim3(gx.grid), dim3(kBsMixed), 0,
                                            s, cols_, A->val32_cs, A->d32, n, gx, w.r32, w.s32, w.w32[wi], w.z32, si,
                                            so, part));
            FV_LAUNCHED();
            if ((rc = state_read_both(w, &h, &hi, s))) return rc;
            if (h.done) break;
            if (hi.done) {
                // the FP32 recurrences stopped (breakdown): restart them from
                // the replaced residual; a breakdown in a restart's first
                // iteration ends the solve
                if (hi.iter == 0) {
                    h.status = FVPCG_BREAKDOWN;
                    break;
                }
                offset += hi.iter;
                if ((rc = state_reset(w, 1, 0.0, maxit - offset, s))) return rc;
                FV_LAYOUT(m, hipLaunchKernelGGL((k_pipe_init_w<kBsMixed, float, W_, CI_, true>), dim3(gx.grid),
                                                dim3(kBsMixed), 0, s, cols_, A->val32_cs, A->d32, n, gx, w.r32,
                                                w.w32[wi], si, part));
                FV_LAUNCHED();
            }
        }
    }
    if (h.zero_b) FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    FV_HIP(hipEventRecord(w.t_it1, s));
    FV_HIP(hipEventRecord(w.t_end, s));
    FV_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = updates == 0 ? 0 : offset + hi.iter;
        stats->outer_iters = updates;
        stats->status = h.status;
        stats->b_norm = h.bnorm;
        stats->r0_norm = h.r0norm;
        stats->rel_res = h.bnorm > 0 ? sqrt(h.rho) / h.bnorm : 0.0;
        stats->true_rel_res = stats->rel_res;
        stats->device_ms = elapsed(w.t_begin, w.t_end);
        stats->iter_ms = elapsed(w.t_it0, w.t_it1);
    }
    return h.status;
}

int adjoint_grads(const fvpcg_matrix* A, const double* x, const double* lam, double* grad_b, double* grad_diag,
                  double* grad_upper, double* grad_lower, hipStream_t s) {
    const fvpcg_mesh* m = A->mesh;
    int gc = (int)((m->n + kBlock - 1) / kBlock);
    if (gc > 65536) gc = 65536;
    int gf = (int)((m->F + kBlock - 1) / kBlock);
    if (gf > 65536) gf = 65536;
    if (gf < 1) gf = 1;
    if (grad_diag || (grad_b && grad_b != lam))
        hipLaunchKernelGGL(k_grad_cells, dim3(gc), dim3(kBlock), 0, s, x, lam, m->n, grad_diag, grad_b);
    if ((grad_upper || grad_lower) && m->F > 0)
        hipLaunchKernelGGL(k_grad_faces, dim3(gf), dim3(kBlock), 0, s, m->owner, m->nb, m->F, x, lam, grad_upper,
                           grad_lower, A->sym ? 1 : 0);
    FV_LAUNCHED();
    return FVPCG_OK;
}

int solve_backward(const fvpcg_matrix* A, const double* x, const double* g, double* grad_b, double* grad_diag,
                   double* grad_upper, double* grad_lower, double tol, int maxit, int method, int precond,
                   hipStream_t s, fvpcg_stats* stats) {
    Work& w = *A->work;
    int rc;
    if ((rc = work_init(w, A->mesh->n))) return rc;
    double* lam = grad_b;
    if (!lam) {
        if (!w.lam && (rc = dev_alloc(&w.lam, (size_t)A->mesh->n, "adjoint solution"))) return rc;
        lam = w.lam;
    }
    FV_HIP(hipMemsetAsync(lam, 0, sizeof(double) * (size_t)A->mesh->n, s));
    int st = solve(A, g, lam, tol, maxit, method, precond, s, stats);
    if (st < 0) return st;
    if ((rc = adjoint_grads(A, x, lam, nullptr, grad_diag, grad_upper, grad_lower, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    return st;
}

}  // namespace fvpcg
