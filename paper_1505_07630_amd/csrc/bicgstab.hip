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
//
// Several right-hand sides with the same matrix (the three velocity
// components of a momentum predictor) are solved together: the kernels are
// templated on the count NR, every vector is stored component after
// component (each component's streams stay unit-stride), each component
// keeps its own scalars and stopping test, and the matrix slots of a row are
// loaded once for all of them: (120 NR + 8) n + 48 F bytes per iteration.  A
// component that has stopped is left untouched while the others go on: its
// values are still loaded (every load of a row is issued before the
// arithmetic), but nothing is computed into its sums or stored for it.  So
// every component's iterates are those of its own single solve.
#include "handles.hpp"
#include "rows.hpp"

namespace fvpcg {

// Scalars of one component's recurrences, written by the last workgroup of
// each kernel.
struct alignas(128) BiState {
    double rho;      // (rhat, r) of the current iterate
    double rho_next; // (rhat, r') of the iterate being formed
    double alpha;    // alpha, omega, beta are 0 once the component has stopped
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
    uint32_t ticket; // reduction ticket (component 0's serves all)
    uint32_t pad;
};

constexpr int kBiMaxRhs = 4;

struct BiWork {
    int n = 0;
    int nr = 0;                  // components the vectors are sized for
    double* r = nullptr;         // [nr][n] each
    double* rhat = nullptr;
    double* p = nullptr;
    double* v = nullptr;
    double* t = nullptr;
    double* partials = nullptr;  // [5 kBiMaxRhs][kBiMaxGrid]
    BiState* st = nullptr;       // [kBiMaxRhs]
    BiState* hst = nullptr;      // pinned [3][kBiMaxRhs]: two chunk slots and the reset image
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
// With several components, s = r - alpha v is stored in r's place by its own
// streaming pass (k_bi_s) before t = A M^-1 s: the product then gathers one
// vector per component instead of two (three components: 766 us against 786
// us per iteration at 7.08M cells, the pass included).
#ifndef FVPCG_BICG_S_PASS
#define FVPCG_BICG_S_PASS 1
#endif
#ifndef FVPCG_GRID_BICG_S
#define FVPCG_GRID_BICG_S 8192
#endif
constexpr int kBsBi = FVPCG_BS_BICG;
constexpr int kBiMaxGrid = FVPCG_GRID_BICG;  // workgroups per launch at most
constexpr int kBiGridS = FVPCG_GRID_BICG_S;  // the s pass (no reduction; measured best of 256-8192)
constexpr bool kBiSPass = FVPCG_BICG_S_PASS != 0;

Geom bi_geom(int n, int cap = kBiMaxGrid) {
    if (n < 1) n = 1;
    int g = (n + kBsBi - 1) / kBsBi;
    if (g > cap) g = cap;
    return {g, kBsBi};
}

// s = r - alpha v with one rounding: the row that owns an entry and every
// row that gathers it compute the same bits.
__device__ __forceinline__ double bi_half(double r, double v, double alpha) { return fma(-alpha, v, r); }

// True while any component still iterates; act[k] for each.
template <int NR>
__device__ __forceinline__ bool bi_active(const BiState* st, bool (&act)[NR]) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        act[k] = !st[k].done;
        any |= act[k];
    }
    return any;
}

// The component's exit: status, and zero scalars so later launches leave it
// untouched.
__device__ __forceinline__ void bi_stop(BiState* st, int status) {
    st->done = 1;
    st->status = status;
    st->alpha = 0.0;
    st->omega = 0.0;
    st->beta = 0.0;
}

// acc[k] += sum_i m[i] * v[k][col_i] over the WT slots (j, m) of row c for
// the components still iterating (v component-major).  Every component's
// values are loaded before any is used, so all the row's gathers are in
// flight at once; the loads of a stopped component are made and discarded.
template <int WT, typename CI, int NR>
__device__ __forceinline__ void gather_v(const CI (&j)[WT], const double (&m)[WT], int n, int c,
                                         const double* __restrict__ v, const bool (&act)[NR], double (&acc)[NR]) {
    double g[NR][WT];
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int i = 0; i < WT; ++i) g[k][i] = v[(size_t)k * n + slot_abs(j[i], c)];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (!act[k]) continue;
#pragma unroll
        for (int i = 0; i < WT; ++i) acc[k] += m[i] * g[k][i];
    }
}

// Same with s = r - alpha v formed from the gathered r and v.
template <int WT, typename CI, int NR>
__device__ __forceinline__ void gather_s(const CI (&j)[WT], const double (&m)[WT], int n, int c,
                                         const double* __restrict__ r, const double* __restrict__ v,
                                         const double (&alpha)[NR], const bool (&act)[NR], double (&acc)[NR]) {
    double gr[NR][WT], gv[NR][WT];
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int i = 0; i < WT; ++i) {
            const int jc = slot_abs(j[i], c);
            gr[k][i] = r[(size_t)k * n + jc];
            gv[k][i] = v[(size_t)k * n + jc];
        }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (!act[k]) continue;
#pragma unroll
        for (int i = 0; i < WT; ++i) acc[k] += m[i] * bi_half(gr[k][i], gv[k][i], alpha[k]);
    }
}

// The row loop of the two products: with several components the slots of
// the next row are prefetched (rows_prefetched), else FV_ROWS with the row's
// slots loaded in place.
#define BI_ROWS(BODY)                                                               \
    if constexpr (NR > 1) {                                                         \
        rows_prefetched<BS, double, WT, CI>(col, val, n, g, BODY);                  \
    } else {                                                                        \
        FV_ROWS(blk_) {                                                             \
            CI j_[WT];                                                              \
            double m_[WT];                                                          \
            load_slots_raw<double, WT, CI>(col, val, n, c, j_, m_);                 \
            BODY(c, j_, m_);                                                        \
        }                                                                           \
    }

// r = b - A x, rhat = r, p = r; (r, r) and (b, b) -> the tolerance and
// rho_1 = (rhat, r) = (r, r).  b and x are component-major ([NR][n]).
template <int BS, int WT, typename CI, int NR>
__global__ __launch_bounds__(BS) void k_bi_init(const CI* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ d, int n, Geom g,
                                                const double* __restrict__ b, const double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ rhat,
                                                double* __restrict__ p, BiState* st, double* partials) {
    double acc[2 * NR];
#pragma unroll
    for (int k = 0; k < 2 * NR; ++k) acc[k] = 0.0;
    FV_ROWS(blk) {
        const double dc = d[c];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double* xk = x + (size_t)k * n;
            const double bc = b[(size_t)k * n + c];
            const double rc = bc - row_gather<double, WT, CI>(col, val, n, c, xk, dc * xk[c]);
            const size_t e = (size_t)k * n + c;
            r[e] = rc;
            st_once(rhat + e, rc);
            p[e] = rc;
            acc[2 * k] += rc * rc;
            acc[2 * k + 1] += bc * bc;
        }
    }
    double t[2 * NR];
    if (device_reduce<BS, 2 * NR>(acc, partials, &st[0].ticket, blk, g.grid, t) && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            BiState* sk = &st[k];
            const double rr = t[2 * k], bb = t[2 * k + 1];
            sk->iter = 0;
            sk->bnorm = sqrt(bb);
            if (bb == 0.0) {
                sk->zero_b = 1;
                sk->rr = 0.0;
                bi_stop(sk, FVPCG_OK);
                continue;
            }
            sk->tol_abs *= sk->bnorm;
            sk->rr = rr;
            sk->rho = rr;
            sk->r0norm = sqrt(rr);
            if (sk->r0norm <= sk->tol_abs)
                bi_stop(sk, FVPCG_OK);
            else if (sk->maxit <= 0)
                bi_stop(sk, FVPCG_NOT_CONVERGED);
        }
    }
}

// v = A M^-1 p; alpha = rho / (rhat, v).
template <int BS, int WT, typename CI, bool JAC, int NR>
__global__ __launch_bounds__(BS) void k_bi_pv(const CI* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ d, int n, Geom g,
                                              const double* __restrict__ p, const double* __restrict__ rhat,
                                              double* __restrict__ v, BiState* st, double* partials) {
    bool act[NR];
    if (!bi_active<NR>(st, act)) return;
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    auto row = [&](int c, const CI (&j)[WT], const double (&m)[WT]) {
        double vc[NR];
        const double dc = JAC ? 1.0 : ld_once(d + c);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double pc = p[(size_t)k * n + c];
            vc[k] = JAC ? pc : dc * pc;
        }
        gather_v<WT, CI, NR>(j, m, n, c, p, act, vc);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            const size_t e = (size_t)k * n + c;
            v[e] = vc[k];
            acc[k] += ld_once(rhat + e) * vc[k];
        }
    };
    BI_ROWS(row);
    const int blk = (int)blockIdx.x;
    double t[NR];
    if (device_reduce<BS, NR>(acc, partials, &st[0].ticket, blk, g.grid, t) && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            const double rv = t[k];
            const double alpha = st[k].rho / rv;
            if (rv == 0.0 || !isfinite(alpha)) {
                bi_stop(&st[k], FVPCG_BREAKDOWN);
                continue;
            }
            st[k].alpha = alpha;
        }
    }
}

// s = r - alpha v stored in r's place for the components still iterating
// (the same rounding as forming it on the fly), so that the product after it
// gathers one vector per component instead of r and v.
template <int BS, int NR>
__global__ __launch_bounds__(BS) void k_bi_s(double* __restrict__ r, const double* __restrict__ v, int n, Geom g,
                                             const BiState* st) {
    bool act[NR];
    if (!bi_active<NR>(st, act)) return;
    double alpha[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) alpha[k] = st[k].alpha;
    FV_ROWS(blk) {
        double rc[NR], vc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const size_t e = (size_t)k * n + c;
            rc[k] = ld_once(r + e);
            vc[k] = ld_once(v + e);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (act[k]) st_once(r + (size_t)k * n + c, bi_half(rc[k], vc[k], alpha[k]));
    }
}

// t = A M^-1 s with s = r - alpha v; omega = (t, s) / (t, t), or omega = 0
// and the half-step exit when ||s|| meets the tolerance; rho' and beta.
// With SP, s has been stored in r's place (k_bi_s) and is gathered as is.
template <int BS, int WT, typename CI, bool JAC, int NR, bool SP>
__global__ __launch_bounds__(BS) void k_bi_st(const CI* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ d, int n, Geom g,
                                              const double* __restrict__ r, const double* __restrict__ v,
                                              const double* __restrict__ rhat, double* __restrict__ t, BiState* st,
                                              double* partials) {
    bool act[NR];
    if (!bi_active<NR>(st, act)) return;
    double alpha[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) alpha[k] = st[k].alpha;
    double acc[5 * NR];
#pragma unroll
    for (int k = 0; k < 5 * NR; ++k) acc[k] = 0.0;
    auto row = [&](int c, const CI (&j)[WT], const double (&m)[WT]) {
        double sc[NR], tc[NR];
        const double dc = JAC ? 1.0 : ld_once(d + c);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const size_t e = (size_t)k * n + c;
            sc[k] = SP ? r[e] : bi_half(r[e], v[e], alpha[k]);
            tc[k] = JAC ? sc[k] : dc * sc[k];
        }
        if constexpr (SP)
            gather_v<WT, CI, NR>(j, m, n, c, r, act, tc);
        else
            gather_s<WT, CI, NR>(j, m, n, c, r, v, alpha, act, tc);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            const size_t e = (size_t)k * n + c;
            const double hc = ld_once(rhat + e);
            st_once(t + e, tc[k]);
            acc[5 * k] += tc[k] * sc[k];
            acc[5 * k + 1] += tc[k] * tc[k];
            acc[5 * k + 2] += sc[k] * sc[k];
            acc[5 * k + 3] += hc * sc[k];
            acc[5 * k + 4] += hc * tc[k];
        }
    };
    BI_ROWS(row);
    const int blk = (int)blockIdx.x;
    double tot[5 * NR];
    if (device_reduce<BS, 5 * NR>(acc, partials, &st[0].ticket, blk, g.grid, tot) && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            BiState* sk = &st[k];
            const double* q = tot + 5 * k;
            if (sqrt(q[2]) <= sk->tol_abs) {
                sk->omega = 0.0;
                sk->beta = 0.0;
                sk->half = 1;
                continue;
            }
            const double omega = q[0] / q[1];
            if (q[1] == 0.0 || omega == 0.0 || !isfinite(omega)) {
                sk->iter = sk->iter + 1;
                bi_stop(sk, FVPCG_BREAKDOWN);
                continue;
            }
            const double rho_next = q[3] - omega * q[4];
            sk->omega = omega;
            sk->rho_next = rho_next;
            sk->beta = (rho_next / sk->rho) * (alpha[k] / omega);
        }
    }
}

// x += M^-1 (alpha p + omega s), r' = s - omega t, p' = r' + beta (p - omega v)
// for the components still iterating (x is component-major); (r', r'):
// stopping test; breakdown if rho' is zero or a scalar not finite.
template <int BS, bool JAC, int NR, bool SP>
__global__ __launch_bounds__(BS) void k_bi_update(double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ p, const double* __restrict__ v,
                                                  const double* __restrict__ t, const double* __restrict__ d, int n,
                                                  Geom g, BiState* st, double* partials) {
    bool act[NR];
    if (!bi_active<NR>(st, act)) return;
    double alpha[NR], omega[NR], beta[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        alpha[k] = st[k].alpha;
        omega[k] = st[k].omega;
        beta[k] = st[k].beta;
    }
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    FV_ROWS(blk) {
        const double dc = JAC ? ld_once(d + c) : 1.0;
        double rc[NR], vc[NR], pc[NR], tc[NR], xc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const size_t e = (size_t)k * n + c;
            rc[k] = ld_once(r + e);
            vc[k] = ld_once(v + e);
            pc[k] = ld_once(p + e);
            tc[k] = ld_once(t + e);
            xc[k] = ld_once(x + e);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            const size_t e = (size_t)k * n + c;
            const double sc = SP ? rc[k] : bi_half(rc[k], vc[k], alpha[k]);
            const double dx = alpha[k] * pc[k] + omega[k] * sc;
            st_once(x + e, xc[k] + (JAC ? dx / dc : dx));
            const double rn = sc - omega[k] * tc[k];
            r[e] = rn;
            p[e] = rn + beta[k] * (pc[k] - omega[k] * vc[k]);
            acc[k] += rn * rn;
        }
    }
    double tot[NR];
    if (device_reduce<BS, NR>(acc, partials, &st[0].ticket, blk, g.grid, tot) && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!act[k]) continue;
            BiState* sk = &st[k];
            const int it = sk->iter + 1;
            sk->iter = it;
            sk->rr = tot[k];
            if (sk->half || sqrt(tot[k]) <= sk->tol_abs) {
                bi_stop(sk, FVPCG_OK);
                continue;
            }
            if (it >= sk->maxit) {
                bi_stop(sk, FVPCG_NOT_CONVERGED);
                continue;
            }
            const double rho = sk->rho_next;
            if (rho == 0.0 || !isfinite(rho) || !isfinite(beta[k])) {
                bi_stop(sk, FVPCG_BREAKDOWN);
                continue;
            }
            sk->rho = rho;
        }
    }
}

// ||b_k - A x_k||^2 at exit (b and x component-major).
template <int BS, int WT, typename CI, int NR>
__global__ __launch_bounds__(BS) void k_bi_true(const CI* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ d, int n, Geom g,
                                                const double* __restrict__ b, const double* __restrict__ x,
                                                BiState* st, double* partials) {
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = 0.0;
    FV_ROWS(blk) {
        const double dc = d[c];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double* xk = x + (size_t)k * n;
            const double rc = b[(size_t)k * n + c] - row_gather<double, WT, CI>(col, val, n, c, xk, dc * xk[c]);
            acc[k] += rc * rc;
        }
    }
    double tot[NR];
    if (device_reduce<BS, NR>(acc, partials, &st[0].ticket, blk, g.grid, tot) && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) st[k].true_rr = tot[k];
    }
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

int bi_alloc(BiWork* w, int n, int nr) {
    w->n = n;
    w->nr = nr;
    int rc;
    const size_t m = (size_t)n * nr;
    if ((rc = dev_alloc(&w->r, m, "BiCGSTAB r")) || (rc = dev_alloc(&w->rhat, m, "BiCGSTAB rhat")) ||
        (rc = dev_alloc(&w->p, m, "BiCGSTAB p")) || (rc = dev_alloc(&w->v, m, "BiCGSTAB v")) ||
        (rc = dev_alloc(&w->t, m, "BiCGSTAB t")) ||
        (rc = dev_alloc(&w->partials, (size_t)5 * kBiMaxRhs * kBiMaxGrid, "BiCGSTAB partials")) ||
        (rc = dev_alloc(&w->st, kBiMaxRhs, "BiCGSTAB state")))
        return rc;
    FV_HIP(hipMemset(w->st, 0, sizeof(BiState) * kBiMaxRhs));
    hipError_t e = hipHostMalloc((void**)&w->hst, 3 * kBiMaxRhs * sizeof(BiState), hipHostMallocDefault);
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

// The matrix's BiCGSTAB workspace for nr components, allocated on first use
// and again when more components are asked for (all or nothing).
int bi_work(BiWork*& w, int n, int nr) {
    if (w && w->nr >= nr) return FVPCG_OK;
    BiWork* nw = new BiWork();
    const int rc = bi_alloc(nw, n, nr);
    if (rc) {
        bi_release(nw);
        return rc;
    }
    bi_release(w);
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

// The nr states into pinned slot `slot`, waited for.
int bi_state_read(BiWork& w, int slot, int nr, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(&w.hst[slot * kBiMaxRhs], w.st, nr * sizeof(BiState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

bool bi_all_done(const BiState* h, int nr) {
    for (int k = 0; k < nr; ++k)
        if (!h[k].done) return false;
    return true;
}

// The next chunk from the components still running: the largest of their
// own estimates (next_chunk), 0 if every one is expected to stop within the
// iterations in flight.
int bi_next_chunk(const BiState* h, int nr, int chunk, int launched) {
    int c = 0;
    for (int k = 0; k < nr; ++k)
        if (!h[k].done)
            c = std::max(c, next_chunk(chunk, kMaxChunk, std::sqrt(h[k].rr), h[k].r0norm, h[k].tol_abs, h[k].iter,
                                       launched - h[k].iter));
    return c;
}

// One iteration: v = A M^-1 p and alpha; (several components, with the
// s pass) s = r - alpha v in r's place; t = A M^-1 s and omega, rho', beta;
// the update of x, r, p and the stopping test.
template <bool JAC, int NR>
void bi_enqueue_iter(const fvpcg_matrix* A, BiWork& w, const double* val, double* x, Geom g, hipStream_t s) {
    constexpr bool SP = kBiSPass && NR > 1;
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    BiState* st = w.st;
    double* part = w.partials;
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_pv<kBsBi, W_, CI_, JAC, NR>), dim3(g.grid), dim3(kBsBi), 0, s, cols_, val,
                                    A->d, n, g, w.p, w.rhat, w.v, st, part));
    if constexpr (SP) {
        const Geom gs = bi_geom(n, kBiGridS);
        hipLaunchKernelGGL((k_bi_s<kBsBi, NR>), dim3(gs.grid), dim3(kBsBi), 0, s, w.r, w.v, n, gs, st);
    }
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_st<kBsBi, W_, CI_, JAC, NR, SP>), dim3(g.grid), dim3(kBsBi), 0, s, cols_,
                                    val, A->d, n, g, w.r, w.v, w.rhat, w.t, st, part));
    hipLaunchKernelGGL((k_bi_update<kBsBi, JAC, NR, SP>), dim3(g.grid), dim3(kBsBi), 0, s, x, w.r, w.p, w.v, w.t,
                       A->d, n, g, st, part);
}

template <int NR>
int bi_solve(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, bool jac, hipStream_t s,
             fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    BiWork& w = *A->bi;
    const Geom g = bi_geom(n);
    BiState* st = w.st;
    double* part = w.partials;
    const double* val = jac ? A->val_cs : A->val;

    FV_HIP(hipEventRecord(w.t_begin, s));
    BiState* h0 = &w.hst[2 * kBiMaxRhs];
    for (int k = 0; k < NR; ++k) {
        h0[k] = BiState();
        h0[k].tol_abs = tol;
        h0[k].maxit = maxit;
        h0[k].status = FVPCG_NOT_CONVERGED;
    }
    FV_HIP(hipMemcpyAsync(st, h0, NR * sizeof(BiState), hipMemcpyHostToDevice, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_init<kBsBi, W_, CI_, NR>), dim3(g.grid), dim3(kBsBi), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, w.r, w.rhat, w.p, st, part));
    FV_LAUNCHED();
    int rc;
    if ((rc = bi_state_read(w, 0, NR, s))) return rc;
    const BiState* h = &w.hst[0];
    for (int k = 0; k < NR; ++k)
        if (h[k].zero_b) FV_HIP(hipMemsetAsync(x + (size_t)k * n, 0, sizeof(double) * (size_t)n, s));
    FV_HIP(hipEventRecord(w.t_it0, s));
    if (!bi_all_done(h, NR)) {
        // Iterations are enqueued in growing chunks; after each chunk the
        // states are copied to pinned memory, and the previous chunk's copy
        // is inspected while the current one runs.  Kernels enqueued after
        // every component has stopped return at once.
        int launched = 0, chunk = 2, pending = -1, slot = 0;
        while (launched < maxit) {
            const int cnt = chunk < maxit - launched ? chunk : maxit - launched;
            for (int i = 0; i < cnt; ++i) {
                if (jac)
                    bi_enqueue_iter<true, NR>(A, w, val, x, g, s);
                else
                    bi_enqueue_iter<false, NR>(A, w, val, x, g, s);
            }
            FV_LAUNCHED();
            launched += cnt;
            FV_HIP(hipMemcpyAsync(&w.hst[slot * kBiMaxRhs], st, NR * sizeof(BiState), hipMemcpyDeviceToHost, s));
            FV_HIP(hipEventRecord(w.ev[slot], s));
            if (pending < 0) {  // nothing to inspect yet
                if (launched == cnt) chunk = chunk * 2 < kMaxChunk ? chunk * 2 : kMaxChunk;
                pending = slot;
                slot ^= 1;
                continue;
            }
            FV_HIP(hipEventSynchronize(w.ev[pending]));
            if (bi_all_done(&w.hst[pending * kBiMaxRhs], NR)) break;
            const int c = bi_next_chunk(&w.hst[pending * kBiMaxRhs], NR, chunk, launched);
            if (c > 0) {
                chunk = c;
                pending = slot;
                slot ^= 1;
                continue;
            }
            // the chunk in flight should stop every component: wait for it
            FV_HIP(hipEventSynchronize(w.ev[slot]));
            if (bi_all_done(&w.hst[slot * kBiMaxRhs], NR)) break;
            chunk = std::max(bi_next_chunk(&w.hst[slot * kBiMaxRhs], NR, chunk, launched), 1);
            pending = -1;
        }
    }
    FV_HIP(hipEventRecord(w.t_it1, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_bi_true<kBsBi, W_, CI_, NR>), dim3(g.grid), dim3(kBsBi), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, st, part));
    FV_LAUNCHED();
    FV_HIP(hipEventRecord(w.t_end, s));
    if ((rc = bi_state_read(w, 0, NR, s))) return rc;
    h = &w.hst[0];
    const float dev_ms = bi_elapsed(w.t_begin, w.t_end), it_ms = bi_elapsed(w.t_it0, w.t_it1);
    int worst = FVPCG_OK;
    for (int k = 0; k < NR; ++k) {
        if (stats) {
            fvpcg_stats* sk = &stats[k];
            sk->iters = h[k].iter;
            sk->outer_iters = 0;
            sk->status = h[k].status;
            sk->b_norm = h[k].bnorm;
            sk->r0_norm = h[k].r0norm;
            sk->rel_res = h[k].bnorm > 0 ? sqrt(h[k].rr) / h[k].bnorm : 0.0;
            sk->true_rel_res = h[k].bnorm > 0 ? sqrt(h[k].true_rr) / h[k].bnorm : 0.0;
            sk->device_ms = dev_ms;
            sk->iter_ms = it_ms;
        }
        if (h[k].status == FVPCG_BREAKDOWN)
            worst = FVPCG_BREAKDOWN;
        else if (h[k].status == FVPCG_NOT_CONVERGED && worst == FVPCG_OK)
            worst = FVPCG_NOT_CONVERGED;
    }
    return worst;
}

}  // namespace

void bicgstab_free(fvpcg_matrix* A) {
    bi_release(A->bi);
    A->bi = nullptr;
}

int solve_bicgstab_multi(const fvpcg_matrix* A, int nrhs, const double* b, double* x, double tol, int maxit,
                         int precond, hipStream_t s, fvpcg_stats* stats) {
    int rc;
    if ((rc = bi_work(A->bi, A->mesh->n, nrhs))) return rc;
    const bool jac = precond == FVPCG_PRECOND_JACOBI;
    switch (nrhs) {
        case 1: return bi_solve<1>(A, b, x, tol, maxit, jac, s, stats);
        case 2: return bi_solve<2>(A, b, x, tol, maxit, jac, s, stats);
        case 3: return bi_solve<3>(A, b, x, tol, maxit, jac, s, stats);
        default: return bi_solve<4>(A, b, x, tol, maxit, jac, s, stats);
    }
}

int solve_bicgstab(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int precond,
                   hipStream_t s, fvpcg_stats* stats) {
    return solve_bicgstab_multi(A, 1, b, x, tol, maxit, precond, s, stats);
}

}  // namespace fvpcg
