// Smoothed-aggregation AMG preconditioner and AMG-preconditioned CG: the
// device cycle and the solvers.  The hierarchy (aggregation, prolongators,
// Galerkin operators, last-level inverse) is built on the device by
// amg_setup.hip; amg.hpp states the method.
//
// The cycle runs entirely on the device: level 0 uses the matrix's ELL layout
// (the pre-smoothing and residual in one pass through the column-scaled
// values), coarser levels CSR with 1, 16 or 64 lanes per row, the last level
// a dense inverse.  The cycle is symmetric positive definite, so standard CG
// can use it as M^-1.
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "amg.hpp"
#include "rows.hpp"

namespace fvpcg {

namespace {

// ---------------------------------------------------------------- kernels

// Level 0, from x = 0: x = omega b / d and r = b - A x in one pass.  With
// x_j = omega b_j / d_j the product is omega (b_c + sum_j (a_cj / d_j) b_j),
// the column-scaled values' gather of b.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_amg_pre0(const CI* __restrict__ col, const double* __restrict__ val_cs,
                                                  const double* __restrict__ d, int n, Geom g, double w,
                                                  const double* __restrict__ b, double* __restrict__ x,
                                                  double* __restrict__ r, const DevState* st) {
    if (st->done) return;
    FV_ROWS(blk) {
        const double bc = b[c];
        const double t = row_gather<double, WT, CI>(col, val_cs, n, c, b, bc);
        x[c] = w * bc / d[c];
        r[c] = bc - w * t;
    }
}

// Level 0: y = x + omega (b - A x) / d; with DOT, also gamma' = (b, y) (b is
// the CG residual, y the preconditioned one): the first cycle sets gamma and
// beta = 0, later ones beta = gamma' / gamma.
template <int BS, int WT, typename CI, bool DOT>
__global__ __launch_bounds__(BS) void k_amg_post0(const CI* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ d, int n, Geom g, double w,
                                                   const double* __restrict__ b, const double* __restrict__ x,
                                                   double* __restrict__ y, int first, DevState* st,
                                                   double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double xc = x[c], dc = d[c], bc = b[c];
        const double ax = row_gather<double, WT, CI>(col, val, n, c, x, dc * xc);
        const double yc = xc + w * (bc - ax) / dc;
        y[c] = yc;
        if (DOT) acc[0] += bc * yc;
    }
    if (!DOT) return;
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        if (first) {
            st->beta = 0.0;
        } else {
            st->beta = t[0] / st->gamma;
        }
        st->gamma = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
        }
    }
}

// CSR levels, one row per thread.
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_pre(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val_cs, const double* __restrict__ d,
                                                      int n, double w, const double* __restrict__ b,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val_cs[k] * b[col[k]];
        const double bi = b[i];
        x[i] = w * bi / d[i];
        r[i] = bi - w * s;
    }
}

__global__ __launch_bounds__(kAmgCsrBs) void k_amg_post(const int* __restrict__ ptr, const int* __restrict__ col,
                                                       const double* __restrict__ val, const double* __restrict__ d,
                                                       int n, double w, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = x[i] + w * (b[i] - s) / d[i];
    }
}

// y = M v (restriction), or y += M v (prolongation, ADD)
template <bool ADD>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_csr_mv(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const double* __restrict__ val, int n,
                                                         const double* __restrict__ v, double* __restrict__ y,
                                                         const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * v[col[k]];
        y[i] = ADD ? y[i] + s : s;
    }
}

// The same CSR operations with G lanes per row (G = 16: four rows per
// wavefront; G = 64: one), for operators whose rows are long (the coarse
// levels of smoothed aggregation hold tens to hundreds of entries per row):
// the lanes stride through the row, coalesced, and the row sum is an
// inclusive DPP scan within each 16-lane row of the wave (plus, for G = 64,
// the sum of the four row totals).  Rows are taken in wave-uniform blocks so
// every lane of a wave takes part in the scan.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    v += row_shr<1>(v);
    v += row_shr<2>(v);
    v += row_shr<4>(v);
    v += row_shr<8>(v);
    if (G == 64) return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
    return v;  // the group's sum in its last lane
}

#define AMG_GROUP_ROWS(G)                                                                  \
    const int lane_ = threadIdx.x & 63, sub_ = lane_ / (G), gl_ = lane_ % (G);              \
    const bool lead_ = (G) == 64 ? lane_ == 0 : gl_ == (G) - 1;                             \
    const int wave_ = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);                  \
    const int nwave_ = (int)((gridDim.x * blockDim.x) >> 6);                                \
    for (int base_ = wave_ * (64 / (G)); base_ < n; base_ += nwave_ * (64 / (G)))

// x = omega b / d; r = b - A x with A x = omega sum_j (a_ij / d_j) b_j
template <int G>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_pre_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const double* __restrict__ val_cs,
                                                        const double* __restrict__ d, int n, double w,
                                                        const double* __restrict__ b, double* __restrict__ x,
                                                        double* __restrict__ r, const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val_cs[k] * b[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) {
            const double bi = b[i];
            x[i] = w * bi / d[i];
            r[i] = bi - w * s;
        }
    }
}

template <int G>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_post_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const double* __restrict__ val, const double* __restrict__ d,
                                                         int n, double w, const double* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val[k] * x[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) y[i] = x[i] + w * (b[i] - s) / d[i];
    }
}

template <int G, bool ADD>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_csr_mv_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                           const double* __restrict__ val, int n,
                                                           const double* __restrict__ v, double* __restrict__ y,
                                                           const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val[k] * v[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) y[i] = ADD ? y[i] + s : s;
    }
}

// last level: y = A^-1 b with the dense inverse, one wavefront per row
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_coarse_w(const double* __restrict__ inv, int n,
                                                           const double* __restrict__ b, double* __restrict__ y,
                                                           const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(64) {
        const int i = base_;
        double s = 0.0;
        for (int k = gl_; k < n; k += 64) s += inv[(size_t)i * n + k] * b[k];
        s = group_sum<64>(s);
        if (lead_) y[i] = s;
    }
}

// gamma' = (r, z) when the hierarchy has a single level (no post-smoothing)
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_dot(const double* __restrict__ r, const double* __restrict__ z, int n,
                                                 Geom g, int first, DevState* st, double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) { acc[0] += r[c] * z[c]; }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->beta = first ? 0.0 : t[0] / st->gamma;
        st->gamma = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
        }
    }
}

// r = b - A x; (b, b), (r, r); stopping test before the first iteration.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_init(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  double* __restrict__ r, DevState* st, double* partials) {
    double acc[2] = {0.0, 0.0};
    FV_ROWS(blk) {
        const double bc = b[c];
        const double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        r[c] = rc;
        acc[0] += bc * bc;
        acc[1] += rc * rc;
    }
    double t[2];
    if (device_reduce<BS, 2>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->iter = 0;
        st->bnorm = sqrt(t[0]);
        st->rho = t[1];
        st->r0norm = sqrt(t[1]);
        if (t[0] == 0.0) {
            st->zero_b = 1;
            st->done = 1;
            st->status = FVPCG_OK;
            return;
        }
        st->tol_abs *= st->bnorm;
        if (st->r0norm <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (st->maxit <= 0) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// p = z (first) or p = z + beta p
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_p(const double* __restrict__ z, double* __restrict__ p, int n, Geom g,
                                               int first, const DevState* st) {
    if (st->done) return;
    const double beta = st->beta;
    FV_ROWS(blk) { p[c] = first ? z[c] : z[c] + beta * p[c]; }
}

// q = A p; delta = (p, q); alpha = gamma / delta.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_spmv(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ p, double* __restrict__ q, DevState* st,
                                                  double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double pc = p[c];
        const double qc = row_gather<double, WT, CI>(col, val, n, c, p, d[c] * pc);
        q[c] = qc;
        acc[0] += pc * qc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->delta = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->alpha = st->gamma / t[0];
    }
}

// x += alpha p; r -= alpha q; rho = (r, r); iteration count and stopping test.
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_xr(double* __restrict__ x, const double* __restrict__ p,
                                                double* __restrict__ r, const double* __restrict__ q, int n, Geom g,
                                                DevState* st, double* partials) {
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        x[c] += alpha * p[c];
        const double rc = r[c] - alpha * q[c];
        r[c] = rc;
        acc[0] += rc * rc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->rho = t[0];
        if (sqrt(t[0]) <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (it >= st->maxit) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// Pipelined CG (Ghysels and Vanroose, Section 4.1) with the AMG cycle as
// M^-1, literal recurrences: w0 = A u0 and the first reduction.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apipe_init_w(const CI* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ d, int n, Geom g,
                                                     const double* __restrict__ r, const double* __restrict__ u,
                                                     double* __restrict__ w, DevState* st, double* partials) {
    if (st->done) return;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const double uc = u[c], rc = r[c];
        const double wc = row_gather<double, WT, CI>(col, val, n, c, u, d[c] * uc);
        w[c] = wc;
        acc[0] += rc * uc;
        acc[1] += wc * uc;
        acc[2] += rc * rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], true);
}

// One iteration, m = M^-1 w already formed by a cycle:
//   n = A m; z = n + beta z; q = m + beta q; s = w + beta s; p = u + beta p;
//   x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z;
// and the reduction (r, u), (w, u), (r, r) of the new iterate.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apipe_iter(const CI* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ d, int n, Geom g,
                                                   const double* __restrict__ m, double* __restrict__ w,
                                                   double* __restrict__ z, double* __restrict__ q,
                                                   double* __restrict__ s, double* __restrict__ p,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ u, DevState* st, double* partials) {
    if (st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const double mc = m[c];
        const double nv = row_gather<double, WT, CI>(col, val, n, c, m, d[c] * mc);
        const double zc = nv + beta * z[c];
        const double qc = mc + beta * q[c];
        const double wc = w[c];
        const double sc = wc + beta * s[c];
        double uc = u[c];
        const double pc = uc + beta * p[c];
        z[c] = zc;
        q[c] = qc;
        s[c] = sc;
        p[c] = pc;
        x[c] += alpha * pc;
        const double rc = r[c] - alpha * sc;
        r[c] = rc;
        uc -= alpha * qc;
        u[c] = uc;
        const double wn = wc - alpha * zc;
        w[c] = wn;
        acc[0] += rc * uc;
        acc[1] += wn * uc;
        acc[2] += rc * rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], false);
}

// zero the pipelined recurrences z, q, s, p before the first iteration
template <int BS>
__global__ __launch_bounds__(BS) void k_apipe_clear(double* __restrict__ z, double* __restrict__ q,
                                                    double* __restrict__ s, double* __restrict__ p, int n, Geom g) {
    FV_ROWS(blk) {
        z[c] = 0.0;
        q[c] = 0.0;
        s[c] = 0.0;
        p[c] = 0.0;
    }
}

// ||b - A x||^2 at exit
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_true(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  DevState* st, double* partials) {
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double rc = b[c] - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        acc[0] += rc * rc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) st->true_rr = t[0];
}

int csr_grid(int n) { return std::max(1, std::min((n + kAmgCsrBs - 1) / kAmgCsrBs, 4096)); }
// blocks for G lanes per row: 64 / G rows per wavefront, 4 wavefronts per block
int group_grid(int n, int G) {
    const int rows_per_block = (kAmgCsrBs / 64) * (64 / G);
    return std::max(1, std::min((n + rows_per_block - 1) / rows_per_block, 8192));
}

void launch_pre(const AmgLevel& v, const double* b, const DevState* st, hipStream_t s) {
    if (v.ga == 1)
        hipLaunchKernelGGL(k_amg_pre, dim3(csr_grid(v.n)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col, v.a_val_cs, v.d,
                           v.n, v.omega, b, v.x, v.r, st);
    else if (v.ga == 16)
        hipLaunchKernelGGL((k_amg_pre_g<16>), dim3(group_grid(v.n, 16)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val_cs, v.d, v.n, v.omega, b, v.x, v.r, st);
    else
        hipLaunchKernelGGL((k_amg_pre_g<64>), dim3(group_grid(v.n, 64)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val_cs, v.d, v.n, v.omega, b, v.x, v.r, st);
}

void launch_post(const AmgLevel& v, const DevState* st, hipStream_t s) {
    if (v.ga == 1)
        hipLaunchKernelGGL(k_amg_post, dim3(csr_grid(v.n)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col, v.a_val, v.d,
                           v.n, v.omega, v.b, v.x, v.y, st);
    else if (v.ga == 16)
        hipLaunchKernelGGL((k_amg_post_g<16>), dim3(group_grid(v.n, 16)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val, v.d, v.n, v.omega, v.b, v.x, v.y, st);
    else
        hipLaunchKernelGGL((k_amg_post_g<64>), dim3(group_grid(v.n, 64)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val, v.d, v.n, v.omega, v.b, v.x, v.y, st);
}

template <bool ADD>
void launch_mv(const int* ptr, const int* col, const double* val, int rows, int G, const double* in, double* out,
               const DevState* st, hipStream_t s) {
    if (G == 1)
        hipLaunchKernelGGL((k_amg_csr_mv<ADD>), dim3(csr_grid(rows)), dim3(kAmgCsrBs), 0, s, ptr, col, val, rows, in,
                           out, st);
    else if (G == 16)
        hipLaunchKernelGGL((k_amg_csr_mv_g<16, ADD>), dim3(group_grid(rows, 16)), dim3(kAmgCsrBs), 0, s, ptr, col,
                           val, rows, in, out, st);
    else
        hipLaunchKernelGGL((k_amg_csr_mv_g<64, ADD>), dim3(group_grid(rows, 64)), dim3(kAmgCsrBs), 0, s, ptr, col,
                           val, rows, in, out, st);
}

// Enqueue one cycle y0 = M^-1 b0 on `s`; kernels skip once st->done.
int enqueue_cycle(const fvpcg_amg* h, const double* b0, double* y0, bool dot, bool first, DevState* st,
                  hipStream_t s) {
    const fvpcg_matrix* A = h->mat;
    const fvpcg_mesh* m = A->mesh;
    const int n0 = m->n;
    const Geom g0 = geom_for(n0, kAmgBs);
    const int L = h->nlev;
    if (L == 1) {
        hipLaunchKernelGGL(k_amg_coarse_w, dim3(group_grid(n0, 64)), dim3(kAmgCsrBs), 0, s, h->cinv, n0, b0, y0, st);
        if (dot)
            hipLaunchKernelGGL((k_apcg_dot<kAmgBs>), dim3(g0.grid), dim3(kAmgBs), 0, s, b0, y0, n0, g0, first ? 1 : 0,
                               st, h->partials);
        FV_LAUNCHED();
        return FVPCG_OK;
    }
    for (int l = 0; l + 1 < L; ++l) {
        const AmgLevel& v = h->lev[l];
        const double* b = l == 0 ? b0 : v.b;
        if (l == 0) {
            FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_pre0<kAmgBs, W_, CI_>), dim3(g0.grid), dim3(kAmgBs), 0, s, cols_,
                                            A->val_cs, A->d, n0, g0, v.omega, b, v.x, v.r, st));
        } else {
            launch_pre(v, b, st, s);
        }
        launch_mv<false>(v.r_ptr, v.r_col, v.r_val, v.nc, v.gr, v.r, h->lev[l + 1].b, st, s);
    }
    const AmgLevel& last = h->lev[L - 1];
    hipLaunchKernelGGL(k_amg_coarse_w, dim3(group_grid(last.n, 64)), dim3(kAmgCsrBs), 0, s, h->cinv, last.n, last.b,
                       last.y, st);
    for (int l = L - 2; l >= 0; --l) {
        const AmgLevel& v = h->lev[l];
        launch_mv<true>(v.p_ptr, v.p_col, v.p_val, v.n, v.gp, h->lev[l + 1].y, v.x, st, s);
        if (l == 0) {
            if (dot) {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_post0<kAmgBs, W_, CI_, true>), dim3(g0.grid), dim3(kAmgBs), 0,
                                                s, cols_, A->val, A->d, n0, g0, v.omega, b0, v.x, y0, first ? 1 : 0,
                                                st, h->partials));
            } else {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_post0<kAmgBs, W_, CI_, false>), dim3(g0.grid), dim3(kAmgBs),
                                                0, s, cols_, A->val, A->d, n0, g0, v.omega, b0, v.x, y0, 0, st,
                                                h->partials));
            }
        } else {
            launch_post(v, st, s);
        }
    }
    FV_LAUNCHED();
    return FVPCG_OK;
}

int state_put(fvpcg_amg* h, double tol, int maxit, hipStream_t s) {
    DevState* hs = &h->hst[1];
    *hs = DevState();
    hs->tol_abs = tol;
    hs->maxit = maxit;
    hs->status = FVPCG_NOT_CONVERGED;
    FV_HIP(hipMemcpyAsync(h->st, hs, sizeof(DevState), hipMemcpyHostToDevice, s));
    return FVPCG_OK;
}

int state_get(fvpcg_amg* h, DevState* out, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(&h->hst[0], h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    *out = h->hst[0];
    return FVPCG_OK;
}

}  // namespace

void amg_free(fvpcg_amg* h) {
    if (!h) return;
    for (AmgLevel& v : h->lev) {
        dev_free(v.a_ptr);
        dev_free(v.a_col);
        dev_free(v.a_val);
        dev_free(v.a_val_cs);
        dev_free(v.d);
        dev_free(v.p_ptr);
        dev_free(v.p_col);
        dev_free(v.p_val);
        dev_free(v.r_ptr);
        dev_free(v.r_col);
        dev_free(v.r_val);
        dev_free(v.b);
        dev_free(v.x);
        dev_free(v.r);
        dev_free(v.y);
        dev_free(v.agg);
        dev_free(v.ap_ptr);
        dev_free(v.ap_col);
        dev_free(v.ap_val);
        dev_free(v.p_off);
        dev_free(v.ap_off);
        dev_free(v.c_off);
    }
    dev_free(h->cinv);
    dev_free(h->a0_ptr);
    dev_free(h->a0_col);
    dev_free(h->a0_val);
    dev_free(h->r);
    dev_free(h->z);
    dev_free(h->p);
    dev_free(h->q);
    dev_free(h->u);
    dev_free(h->w);
    dev_free(h->m);
    dev_free(h->s);
    dev_free(h->st);
    dev_free(h->partials);
    if (h->hst) (void)hipHostFree(h->hst);
    hipEvent_t* evs[] = {&h->t_begin, &h->t_end, &h->t_it0, &h->t_it1};
    for (hipEvent_t* e : evs)
        if (*e) (void)hipEventDestroy(*e);
    delete h;
}

int amg_create(const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, uint64_t seed, hipStream_t s,
               fvpcg_amg** out) {
    fvpcg_amg* h = new (std::nothrow) fvpcg_amg();
    if (!h) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    h->mat = A;
    int rc;
    try {
        rc = amg_build(h, A, theta, max_levels, coarse_size, seed, s);
    } catch (const std::bad_alloc&) {
        rc = set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed during the AMG setup");
    }
    if (rc) {
        amg_free(h);
        return rc;
    }
    *out = h;
    return FVPCG_OK;
}

// fvpcg_amg_refresh: the matrix's checks of fvpcg_amg_create, then the
// numeric refresh
int amg_update(fvpcg_amg* h, hipStream_t s) {
    const fvpcg_matrix* mat = h->mat;
    if (!mat->diag_ok) return set_error(FVPCG_BREAKDOWN, "AMG needs a finite positive diagonal");
    if (!mat->vals_sym)
        return set_error(FVPCG_UNSUPPORTED, "AMG needs a symmetric matrix (lower == upper on every face)");
    try {
        return amg_refresh(h, s);
    } catch (const std::bad_alloc&) {
        h->generation = kStaleGeneration;
        return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed during the AMG refresh");
    }
}

int amg_levels(const fvpcg_amg* h) { return h->nlev; }
int amg_level_n(const fvpcg_amg* h, int l) { return h->lev[l].n; }
long long amg_level_nnz(const fvpcg_amg* h, int l) { return h->lev[l].nnz; }
int amg_level_agg(const fvpcg_amg* h, int l, int* host_out, hipStream_t s) {
    if (!h->lev[l].agg) return set_error(FVPCG_INVALID_ARG, "level %d has no aggregates", l);
    FV_HIP(hipMemcpyAsync(host_out, h->lev[l].agg, sizeof(int) * (size_t)h->lev[l].n, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// Level l's operator (which 0, levels >= 1), prolongator (1) or restriction
// (2) as CSR into host arrays (NULL arrays: sizes only).
int amg_export(const fvpcg_amg* h, int l, int which, int* rows, int* cols, long long* nnz, int* ptr, int* col,
               double* val, hipStream_t s) {
    const AmgLevel& v = h->lev[l];
    const int *dp, *dc;
    const double* dv;
    if (which == 0) {
        if (l == 0) return set_error(FVPCG_INVALID_ARG, "level 0's operator is the matrix itself (ELL layout)");
        *rows = *cols = v.n;
        *nnz = v.nnz;
        dp = v.a_ptr, dc = v.a_col, dv = v.a_val;
    } else if (l + 1 < h->nlev && (which == 1 || which == 2)) {
        *rows = which == 1 ? v.n : v.nc;
        *cols = which == 1 ? v.nc : v.n;
        *nnz = v.p_nnz;
        dp = which == 1 ? v.p_ptr : v.r_ptr;
        dc = which == 1 ? v.p_col : v.r_col;
        dv = which == 1 ? v.p_val : v.r_val;
    } else {
        return set_error(FVPCG_INVALID_ARG, "level %d has no %s", l, which == 1 || which == 2 ? "coarser level" : "such operator");
    }
    if (ptr) FV_HIP(hipMemcpyAsync(ptr, dp, sizeof(int) * ((size_t)*rows + 1), hipMemcpyDeviceToHost, s));
    if (col) FV_HIP(hipMemcpyAsync(col, dc, sizeof(int) * (size_t)*nnz, hipMemcpyDeviceToHost, s));
    if (val) FV_HIP(hipMemcpyAsync(val, dv, sizeof(double) * (size_t)*nnz, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// The hierarchy holds coarse operators formed from the coefficients at
// setup; after the matrix is updated they describe another operator.
static int check_generation(const fvpcg_amg* h) {
    if (h->generation != h->mat->generation)
        return set_error(FVPCG_INVALID_ARG,
                         "the matrix was updated after this AMG hierarchy was built (or its refresh failed); refresh or create it");
    return FVPCG_OK;
}

// z = M^-1 r (one cycle)
int amg_apply(const fvpcg_amg* ch, const double* r, double* z, hipStream_t s) {
    fvpcg_amg* h = const_cast<fvpcg_amg*>(ch);
    int rc;
    if ((rc = check_generation(h))) return rc;
    if ((rc = state_put(h, 0.0, 1, s))) return rc;
    if ((rc = enqueue_cycle(h, r, z, false, false, h->st, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// Standard PCG (Section 2) with one AMG cycle as M^-1.
int solve_amg(const fvpcg_amg* ch, const double* b, double* x, double tol, int maxit, int method, hipStream_t s,
              fvpcg_stats* stats) {
    fvpcg_amg* h = const_cast<fvpcg_amg*>(ch);
    const fvpcg_matrix* A = h->mat;
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    const Geom g = geom_for(n, kAmgBs);
    DevState* st = h->st;
    int rc;
    if ((rc = check_generation(h))) return rc;
    FV_HIP(hipEventRecord(h->t_begin, s));
    if ((rc = state_put(h, tol, maxit, s))) return rc;
    FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_init<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, h->r, st, h->partials));
    FV_LAUNCHED();
    DevState hs;
    if ((rc = state_get(h, &hs, s))) return rc;
    FV_HIP(hipEventRecord(h->t_it0, s));
    const bool pipe = method == FVPCG_PIPECG;
    if (pipe && !h->u) {
        const size_t nn = (size_t)std::max(n, 1);
        if ((rc = dev_alloc(&h->u, nn, "AMG pipelined vectors")) || (rc = dev_alloc(&h->w, nn, "AMG pipelined vectors")) ||
            (rc = dev_alloc(&h->m, nn, "AMG pipelined vectors")) || (rc = dev_alloc(&h->s, nn, "AMG pipelined vectors")))
            return rc;
    }
    if (!hs.done && pipe) {
        // u = M^-1 r; z = q = s = p = 0; w = A u and the first reduction
        if ((rc = enqueue_cycle(h, h->r, h->u, false, false, st, s))) return rc;
        hipLaunchKernelGGL((k_apipe_clear<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->q, h->s, h->p, n, g);
        FV_LAYOUT(m, hipLaunchKernelGGL((k_apipe_init_w<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_,
                                        A->val, A->d, n, g, h->r, h->u, h->w, st, h->partials));
        FV_LAUNCHED();
        int launched = 0, chunk = 1;
        while (launched < maxit) {
            const int cnt = std::min(chunk, maxit - launched);
            for (int k = 0; k < cnt; ++k) {
                if ((rc = enqueue_cycle(h, h->w, h->m, false, false, st, s))) return rc;
                FV_LAYOUT(m, hipLaunchKernelGGL((k_apipe_iter<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s,
                                                cols_, A->val, A->d, n, g, h->m, h->w, h->z, h->q, h->s, h->p, x,
                                                h->r, h->u, st, h->partials));
                FV_LAUNCHED();
            }
            launched += cnt;
            if ((rc = state_get(h, &hs, s))) return rc;
            if (hs.done) break;
            chunk = std::max(next_chunk(chunk, 16, std::sqrt(hs.rho), hs.r0norm, hs.tol_abs, hs.iter, 0), 1);
        }
    } else if (!hs.done) {
        // z = M^-1 r, gamma = (r, z), p = z
        if ((rc = enqueue_cycle(h, h->r, h->z, true, true, st, s))) return rc;
        hipLaunchKernelGGL((k_apcg_p<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->p, n, g, 1, st);
        FV_LAUNCHED();
        int launched = 0, chunk = 1;
        while (launched < maxit) {
            const int cnt = std::min(chunk, maxit - launched);
            for (int k = 0; k < cnt; ++k) {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_spmv<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s,
                                                cols_, A->val, A->d, n, g, h->p, h->q, st, h->partials));
                hipLaunchKernelGGL((k_apcg_xr<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, x, h->p, h->r, h->q, n, g,
                                   st, h->partials);
                if ((rc = enqueue_cycle(h, h->r, h->z, true, false, st, s))) return rc;
                hipLaunchKernelGGL((k_apcg_p<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->p, n, g, 0, st);
                FV_LAUNCHED();
            }
            launched += cnt;
            if ((rc = state_get(h, &hs, s))) return rc;
            if (hs.done) break;
            chunk = std::max(next_chunk(chunk, 16, std::sqrt(hs.rho), hs.r0norm, hs.tol_abs, hs.iter, 0), 1);
        }
    }
    FV_HIP(hipEventRecord(h->t_it1, s));
    if (hs.zero_b) FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_true<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, st, h->partials));
    FV_LAUNCHED();
    FV_HIP(hipEventRecord(h->t_end, s));
    if ((rc = state_get(h, &hs, s))) return rc;
    if (stats) {
        stats->iters = hs.iter;
        stats->outer_iters = 0;
        stats->status = hs.status;
        stats->b_norm = hs.bnorm;
        stats->r0_norm = hs.r0norm;
        stats->rel_res = hs.bnorm > 0 ? sqrt(hs.rho) / hs.bnorm : 0.0;
        stats->true_rel_res = hs.bnorm > 0 ? sqrt(hs.true_rr) / hs.bnorm : 0.0;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, h->t_begin, h->t_end);
        stats->device_ms = ms;
        (void)hipEventElapsedTime(&ms, h->t_it0, h->t_it1);
        stats->iter_ms = ms;
    }
    return hs.status;
}

}  // namespace fvpcg
