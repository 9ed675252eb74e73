// BiCGSTAB for non-symmetric LDU matrices (lower != upper): the solver the
// paper names for icoFoam's momentum equation (Section 2).  van der Vorst's
// Bi-CGSTAB with M = I or Jacobi applied to the search directions (right
// preconditioning: r stays the residual of A x = b), shadow residual
// rhat = r0.
//
// Each iteration needs three global reductions (alpha; omega; the stopping
// test), so it runs as three row-parallel kernels, each ending in the
// single-pass reduction whose last workgroup forms the next scalars.  With
// Jacobi the products use the column-scaled values A D^-1 (unit diagonal), so
// neither phat = D^-1 p nor shat = D^-1 s is ever stored:
//
//   k_bi_pv     v = A D^-1 p;  (rhat, v) -> alpha
//   k_bi_st     s = r - alpha v (formed on the fly, also for the gathered
//               neighbours), t = A D^-1 s;  (t, s), (t, t), (s, s), (rhat, s),
//               (rhat, t) -> omega (or the half-step exit) and
//               rho' = (rhat, r') = (rhat, s) - omega (rhat, t), so
//               beta = (rho'/rho)(alpha/omega) is known one kernel early
//   k_bi_update x += D^-1 (alpha p + omega s), r' = s - omega t,
//               p' = r' + beta (p - omega v);  (r', r') -> stop
//
// rho' is the inner product of rhat with r' = s - omega t split by linearity
// (the vectors are the computed ones; only the rounding order differs from
// forming r' first).  Knowing beta before the update lets that kernel store
// p' itself, so the first product gathers one vector.  Per iteration the
// kernels move 128 n + 48 F bytes (int32 columns) against 2 x 24 F for the
// two products alone.
#include "handles.hpp"
#include "rows.hpp"

namespace fvpcg {

// Scalars of the recurrences, written by the last workgroup of each kernel.
struct alignas(128) BiState {
    double rho;      // (rhat, r) of the current iterate
    double rho_next; // (rhat, r') of the iterate being formed
    double alpha;
    double omega;    // 0 after a half-step exit
    double beta;
    double rr;       // (r, r)
    double bnorm;
    double tol_abs;  // tol * ||b||
    double r0norm;
    double true_rr;  // ||b - A x||^2 at exit
    int32_t iter;    // iterations that formed alpha
    int32_t maxit;
    int32_t done;
    int32_t status;
    int32_t zero_b;
    int32_t half;    // ||s|| met the tolerance: x += alpha phat ends the solve
    uint32_t ticket;
    uint32_t pad;
};

struct BiWork {
    int n = 0;
    double* r = nullptr;
    double* rhat = nullptr;
    double* p = nullptr;
    double* v = nullptr;
    double* t = nullptr;
    double* partials = nullptr;  // [5][kBiMaxGrid]
    BiState* st = nullptr;
    BiState* hst = nullptr;  // pinned [3]: two chunk slots and the reset image
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t_begin = nullptr, t_end = nullptr, t_it0 = nullptr, t_it1 = nullptr;
};

namespace {

#ifndef FVPCG_BS_BICG
#define FVPCG_BS_BICG 512
#endif
#ifndef FVPCG_GRID_BICG
#define FVPCG_GRID_BICG 256
#endif
constexpr int kBsBi = FVPCG_BS_BICG;
constexpr int kBiMaxGrid = FVPCG_GRID_BICG;  // workgroups per launch at most

Geom bi_geom(int n) {
    if (n < 1) n = 1;
    int g = (n + kBsBi - 1) / kBsBi;
    if (g > kBiMaxGrid) g = kBiMaxGrid;
    return {g, kBsBi};
}

// s = r - alpha v with one rounding: the row that owns an entry and every
// row that gathers it compute the same bits.
__device__ __forceinline__ double bi_half(double r, double v, double alpha) { return fma(-alpha, v, r); }

// acc + sum_k val[k][c] * s[j] over the WT slots of row c, with s = r - alpha v
// formed from the gathered r[j] and v[j].
template <int WT, typename CI>
__device__ __forceinline__ double gather_s(const CI* __restrict__ col, const double* __restrict__ val, int n, int c,
                                           const double* __restrict__ r, const double* __restrict__ v, double alpha,
                                           double acc) {
    int j[WT];
    double m[WT];
#pragma unroll
    for (int i = 0; i < WT; ++i) {
        const size_t o = (size_t)i * n + c;
        j[i] = slot_col(col, o, c);
        m[i] = ld_once(val + o);
    }
#pragma unroll
    for (int i = 0; i < WT; ++i) acc += m[i] * bi_half(r[j[i]], v[j[i]], alpha);
    return acc;
}

// r = b - A x, rhat = r, p = r; (r, r) and (b, b) -> the tolerance and
// rho_1 = (rhat, r) = (r, r).
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_bi_init(const CI* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ d, int n, Geom g,
                                                const double* __restrict__ b, const double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ rhat,
                                                double* __restrict__ p, BiState* st, double* partials) {
    double acc[2] = {0.0, 0.0};
    FV_ROWS(blk) {
        const double bc = b[c];
        const double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        r[c] = rc;
        st_once(rhat + c, rc);
        p[c] = rc;
        acc[0] += rc * rc;
        acc[1] += bc * bc;
    }
    double t[2];
    if (device_reduce<BS, 2>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->iter = 0;
        st->bnorm = sqrt(t[1]);
        if (t[1] == 0.0) {
            st->zero_b = 1;
            st->done = 1;
            st->status = FVPCG_OK;
            st->rr = 0.0;
            return;
        }
        st->tol_abs *= st->bnorm;
        st->rr = t[0];
        st->rho = t[0];
        st->r0norm = sqrt(t[0]);
        if (st->r0norm <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (st->maxit <= 0) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// v = A M^-1 p; alpha = rho / (rhat, v).
template <int BS, int WT, typename CI, bool JAC>
__global__ __launch_bounds__(BS) void k_bi_pv(const CI* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ d, int n, Geom g,
                                              const double* __restrict__ p, const double* __restrict__ rhat,
                                              double* __restrict__ v, BiState* st, double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double pc = p[c];
        const double vc = row_gather<double, WT, CI>(col, val, n, c, p, JAC ? pc : ld_once(d + c) * pc);
        v[c] = vc;
        acc[0] += ld_once(rhat + c) * vc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const double rv = t[0];
        const double alpha = st->rho / rv;
        if (rv == 0.0 || !isfinite(alpha)) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->alpha = alpha;
    }
}

// t = A M^-1 s with s = r - alpha v; omega = (t, s) / (t, t), or omega = 0
// and the half-step exit when ||s|| meets the tolerance; rho' and beta.
template <int BS, int WT, typename CI, bool JAC>
__global__ __launch_bounds__(BS) void k_bi_st(const CI* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ d, int n, Geom g,
                                              const double* __restrict__ r, const double* __restrict__ v,
                                              const double* __restrict__ rhat, double* __restrict__ t, BiState* st,
                                              double* partials) {
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const double sc = bi_half(r[c], v[c], alpha);
        const double tc = gather_s<WT, CI>(col, val, n, c, r, v, alpha, JAC ? sc : ld_once(d + c) * sc);
        const double hc = ld_once(rhat + c);
        st_once(t + c, tc);
        acc[0] += tc * sc;
        acc[1] += tc * tc;
        acc[2] += sc * sc;
        acc[3] += hc * sc;
        acc[4] += hc * tc;
    }
    double tot[5];
    if (device_reduce<BS, 5>(acc, partials, &st->ticket, blk, g.grid, tot) && threadIdx.x == 0) {
        if (sqrt(tot[2]) <= st->tol_abs) {
            st->omega = 0.0;
            st->beta = 0.0;
            st->half = 1;
            return;
        }
        const double omega = tot[0] / tot[1];
        if (tot[1] == 0.0 || omega == 0.0 || !isfinite(omega)) {
            st->iter = st->iter + 1;
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        const double rho_next = tot[3] - omega * tot[4];
        st->omega = omega;
        st->rho_next = rho_next;
        st->beta = (rho_next / st->rho) * (alpha / omega);
    }
}

// x += M^-1 (alpha p + omega s), r' = s - omega t, p' = r' + beta (p - omega v);
// (r', r'): stopping test; breakdown if rho' is zero or a scalar not finite.
template <int BS, bool JAC>
__global__ __launch_bounds__(BS) void k_bi_update(double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ p, const double* __restrict__ v,
                                                  const double* __restrict__ t, const double* __restrict__ d, int n,
                                                  Geom g, BiState* st, double* partials) {
    if (st->done) return;
    const double alpha = st->alpha, omega = st->omega, beta = st->beta;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double rc = ld_once(r + c), vc = ld_once(v + c), pc = ld_once(p + c);
        const double sc = bi_half(rc, vc, alpha);
        const double dx = alpha * pc + omega * sc;
        st_once(x + c, ld_once(x + c) + (JAC ? dx / ld_once(d + c) : dx));
        const double rn = sc - omega * ld_once(t + c);
        r[c] = rn;
        p[c] = rn + beta * (pc - omega * vc);
        acc[0] += rn * rn;
    }
    double tot[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, tot) && threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->rr = tot[0];
        if (st->half || sqrt(tot[0]) <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
            return;
        }
        if (it >= st->maxit) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
            return;
        }
        const double rho = st->rho_next;
        if (rho == 0.0 || !isfinite(rho) || !isfinite(beta)) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->rho = rho;
    }
}

// ||b - A x||^2 at exit.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_bi_true(const CI* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ d, int n, Geom g,
                                                const double* __restrict__ b, const double* __restrict__ x,
                                                BiState* st, double* partials) {
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double rc = b[c] - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        acc[0] += rc * rc;
    }
    double tot[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, tot) && threadIdx.x == 0)
        st->true_rr = tot[0];
}

void bi_release(BiWork* w) {
    if (!w) return;
    dev_free(w->r);
    dev_free(w->rhat);
    dev_free(w->p);
    dev_free(w->v);
    dev_free(w->t);
    dev_free(w->partials);
    dev_free(w->st);
    if (w->hst) (void)hipHostFree(w->hst);
    for (auto ev : w->ev)
        if (ev) (void)hipEventDestroy(ev);
    hipEvent_t te[] = {w->t_begin, w->t_end, w->t_it0, w->t_it1};
    for (auto ev : te)
        if (ev) (void)hipEventDestroy(ev);
    delete w;
}

int bi_alloc(BiWork* w, int n) {
    w->n = n;
    int rc;
    const size_t m = (size_t)n;
    if ((rc = dev_alloc(&w->r, m, "BiCGSTAB r")) || (rc = dev_alloc(&w->rhat, m, "BiCGSTAB rhat")) ||
        (rc = dev_alloc(&w->p, m, "BiCGSTAB p")) || (rc = dev_alloc(&w->v, m, "BiCGSTAB v")) ||
        (rc = dev_alloc(&w->t, m, "BiCGSTAB t")) ||
        (rc = dev_alloc(&w->partials, (size_t)5 * kBiMaxGrid, "BiCGSTAB partials")) ||
        (rc = dev_alloc(&w->st, 1, "BiCGSTAB state")))
        return rc;
    FV_HIP(hipMemset(w->st, 0, sizeof(BiState)));
    hipError_t e = hipHostMalloc((void**)&w->hst, 3 * sizeof(BiState), hipHostMallocDefault);
    if (e != hipSuccess) {
        w->hst = nullptr;
        return set_error(FVPCG_OUT_OF_MEMORY, "pinned host allocation failed: %s", hipGetErrorString(e));
    }
    for (auto& ev : w->ev) FV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    FV_HIP(hipEventCreate(&w->t_begin));
    FV_HIP(hipEventCreate(&w->t_end));
    FV_HIP(hipEventCreate(&w->t_it0));
    FV_HIP(hipEventCreate(&w->t_it1));
    return FVPCG_OK;
}

// The matrix's BiCGSTAB workspace, allocated on first use (all or nothing).
int bi_work(BiWork*& w, int n) {
    if (w) return FVPCG_OK;
    BiWork* nw = new BiWork();
    const int rc = bi_alloc(nw, n);
    if (rc) {
        bi_release(nw);
        return rc;
    }
    w = nw;
    return FVPCG_OK;
}

float bi_elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

int bi_state_read(BiWork& w, int slot, BiState* out, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(&w.hst[slot], w.st, sizeof(BiState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    *out = w.hst[slot];
    return FVPCG_OK;
}

}  // namespace

void bicgstab_free(fvpcg_matrix* A) {
    bi_release(A->bi);
    A->bi = nullptr;
}

int solve_bicgstab(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int precond,
                   hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    const bool jac = precond == FVPCG_PRECOND_JACOBI;
    int rc;
    if ((rc = bi_work(A->bi, n))) return rc;
    BiWork& w = *A->bi;
    const Geom g = bi_geom(n);
    BiState* st = w.st;
    double* part = w.partials;
    const double* val = jac ? A->val_cs : A->val;

    FV_HIP(hipEventRecord(w.t_begin, s));
    BiState* h0 = &w.hst[2];
    *h0 = BiState();
    h0->tol_abs = tol;
    h0->maxit = maxit;
    h0->status = FVPCG_NOT_CONVERGED;
    FV_HIP(hipMemcpyAsync(st, h0, sizeof(BiState), hipMemcpyHostToDevice, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_init<kBsBi, W_, CI_>), dim3(g.grid), dim3(kBsBi), 0, s, cols_, A->val, A->d,
                                    n, g, b, x, w.r, w.rhat, w.p, st, part));
    FV_LAUNCHED();
    BiState h;
    if ((rc = bi_state_read(w, 0, &h, s))) return rc;
    FV_HIP(hipEventRecord(w.t_it0, s));
    if (h.zero_b) {
        FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    } else if (!h.done) {
        // Iterations are enqueued in growing chunks; after each chunk the
        // state is copied to pinned memory, and the previous chunk's copy is
        // inspected while the current one runs.  Kernels enqueued after the
        // exit return at once.
        int launched = 0, chunk = 2, pending = -1, slot = 0;
        while (launched < maxit) {
            const int cnt = chunk < maxit - launched ? chunk : maxit - launched;
            for (int i = 0; i < cnt; ++i) {
                FV_LAYOUT(m,
                          if (jac) {
                              hipLaunchKernelGGL((k_bi_pv<kBsBi, W_, CI_, true>), dim3(g.grid), dim3(kBsBi), 0, s,
                                                 cols_, val, A->d, n, g, w.p, w.rhat, w.v, st, part);
                              hipLaunchKernelGGL((k_bi_st<kBsBi, W_, CI_, true>), dim3(g.grid), dim3(kBsBi), 0, s,
                                                 cols_, val, A->d, n, g, w.r, w.v, w.rhat, w.t, st, part);
                          } else {
                              hipLaunchKernelGGL((k_bi_pv<kBsBi, W_, CI_, false>), dim3(g.grid), dim3(kBsBi), 0, s,
                                                 cols_, val, A->d, n, g, w.p, w.rhat, w.v, st, part);
                              hipLaunchKernelGGL((k_bi_st<kBsBi, W_, CI_, false>), dim3(g.grid), dim3(kBsBi), 0, s,
                                                 cols_, val, A->d, n, g, w.r, w.v, w.rhat, w.t, st, part);
                          });
                if (jac)
                    hipLaunchKernelGGL((k_bi_update<kBsBi, true>), dim3(g.grid), dim3(kBsBi), 0, s, x, w.r, w.p, w.v,
                                       w.t, A->d, n, g, st, part);
                else
                    hipLaunchKernelGGL((k_bi_update<kBsBi, false>), dim3(g.grid), dim3(kBsBi), 0, s, x, w.r, w.p, w.v,
                                       w.t, A->d, n, g, st, part);
            }
            FV_LAUNCHED();
            launched += cnt;
            FV_HIP(hipMemcpyAsync(&w.hst[slot], st, sizeof(BiState), hipMemcpyDeviceToHost, s));
            FV_HIP(hipEventRecord(w.ev[slot], s));
            if (pending >= 0) {
                FV_HIP(hipEventSynchronize(w.ev[pending]));
                if (w.hst[pending].done) break;
            }
            pending = slot;
            slot ^= 1;
            if (chunk < kMaxChunk) chunk *= 2;
        }
    }
    FV_HIP(hipEventRecord(w.t_it1, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_true<kBsBi, W_, CI_>), dim3(g.grid), dim3(kBsBi), 0, s, cols_, A->val, A->d,
                                    n, g, b, x, st, part));
    FV_LAUNCHED();
    FV_HIP(hipEventRecord(w.t_end, s));
    if ((rc = bi_state_read(w, 0, &h, s))) return rc;
    if (stats) {
        stats->iters = h.iter;
        stats->outer_iters = 0;
        stats->status = h.status;
        stats->b_norm = h.bnorm;
        stats->r0_norm = h.r0norm;
        stats->rel_res = h.bnorm > 0 ? sqrt(h.rr) / h.bnorm : 0.0;
        stats->true_rel_res = h.bnorm > 0 ? sqrt(h.true_rr) / h.bnorm : 0.0;
        stats->device_ms = bi_elapsed(w.t_begin, w.t_end);
        stats->iter_ms = bi_elapsed(w.t_it0, w.t_it1);
    }
    return h.status;
}

}  // namespace fvpcg
