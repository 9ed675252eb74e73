// icoFoam's PISO time step on the device (Section 2 names icoFoam and its
// solvers: BiCGSTAB for the momentum equation, CG for the pressure
// equation; Section 4.1: the application calls the solver repeatedly).
// Finite volumes on the LDU addressing of a box of cubes of side h
// (V = h^3, face area h^2, w = area / centre distance = h):
//   momentum (implicit Euler, upwind convection of the face flux phi_f,
//   owner -> neighbour), one matrix for the three velocity components:
//     upper_f = -nu w - max(-phi_f, 0),   lower_f = -nu w - max(phi_f, 0),
//     diag_c  = V/dt + bwall_c + sum over c's faces of (nu w + its outflow, if > 0),
//     bH_kc   = (V/dt) U_kc + blid_c [k = x];
//   pressure gradient (Gauss, linear face values, zero gradient at walls):
//     (grad p)_kc = (1/h) (bgrad_kc p_c + sum over c's faces along k of n_cf (p_o + p_n)/2),
//     n_cf the outward normal component: face_sgn for the owner, -face_sgn for the neighbour;
//   predictor: A U_k = bH_k - V (grad p)_k, the three components together
//   (BiCGSTAB with Jacobi, from the old U);
//   each corrector: rAU = V / diag, HbyA_k = (bH_k - offdiag(A) U_k) / diag,
//     phiHbyA_f = face_sgn h^2 (HbyA_{d,o} + HbyA_{d,n}) / 2 (d = the face's axis),
//     c_f = w (rAU_o + rAU_n) / 2, pressure system sum_f c_f (p_c - p_other) =
//     -div(phiHbyA)_c with cell 0 pinned (its couplings zero in both
//     triangles, b_0 = 0), solved by CG (Jacobi, or the AMG preconditioner)
//     from the previous p;
//     phi_f = phiHbyA_f - c_f (p_n - p_o),   U_k = HbyA_k - rAU (grad p)_k.
// Cell sums (diagonals, divergences, gradients, the H operator) are gathers
// through the mesh's slot -> face map, one thread per cell in column order:
// no atomics, a fixed order.  The momentum matrix's device layout is
// refreshed every step, the pressure matrix's once per step (its
// coefficients change with rAU only).
#include <algorithm>
#include <climits>

#include "handles.hpp"
#include "rows.hpp"

struct fvpcg_piso {
    const fvpcg_mesh* mesh = nullptr;
    double h = 0.0, nu = 0.0;
    int psolver = FVPCG_CG;  // FVPCG_CG (Jacobi-PCG) or FVPCG_PSOLVER_AMG
    int8_t *fdir = nullptr, *fsgn = nullptr;  // [F]
    double *bwall = nullptr, *blid = nullptr, *bgrad = nullptr;  // [n], [n], [3][n]
    double *mdiag = nullptr, *mupper = nullptr, *mlower = nullptr;  // momentum coefficients
    double *bH = nullptr, *rhs = nullptr, *HbyA = nullptr;  // [3][n]
    double *rAU = nullptr, *pdiag = nullptr, *prhs = nullptr;  // [n]
    double *phiH = nullptr, *cf = nullptr, *pupper = nullptr;  // [F]
    fvpcg_matrix* mom = nullptr;   // momentum matrix (lower != upper)
    fvpcg_matrix* pres = nullptr;  // pressure matrix (symmetric)
    fvpcg_amg* amg = nullptr;      // its AMG hierarchy (AMG pressure solver), kept across steps and calls
};

namespace fvpcg {

int matrix_create(const fvpcg_mesh* m, const double* diag, const double* upper, const double* lower, uint32_t flags,
                  hipStream_t s, fvpcg_matrix** out);
int matrix_update(fvpcg_matrix* A, const double* diag, const double* upper, const double* lower, hipStream_t s);
int matrix_destroy(fvpcg_matrix* A);
int solve(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
          hipStream_t s, fvpcg_stats* stats);
int solve_bicgstab_multi(const fvpcg_matrix* A, int nrhs, const double* b, double* x, double tol, int maxit,
                         int precond, hipStream_t s, fvpcg_stats* stats);
int amg_create(const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, uint64_t seed, hipStream_t s,
               fvpcg_amg** out);
void amg_free(fvpcg_amg* h);
int amg_update(fvpcg_amg* h, hipStream_t s);
int solve_amg(const fvpcg_amg* h, const double* b, double* x, double tol, int maxit, int method, hipStream_t s,
              fvpcg_stats* stats);

namespace {

constexpr int kPisoBs = 256;
// AMG for the pressure correctors: the library's default strength threshold,
// the other parameters the typical ones of fvpcg_amg_create
constexpr double kPisoAmgTheta = 0.02;

int pgrid(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + kPisoBs - 1) / kPisoBs, 65536)); }

#define FV_PISO_LOOP(i, n) for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

// (grad p)_kc for the three axes by a gather over the cell's faces
__device__ __forceinline__ void cell_gradp(const int* __restrict__ ref, const int* __restrict__ owner,
                                           const int* __restrict__ nb, const int8_t* __restrict__ fdir,
                                           const int8_t* __restrict__ fsgn, const double* __restrict__ bgrad,
                                           const double* __restrict__ p, int n, int W, int c, double inv_h,
                                           double (&g)[3]) {
    const double pc = p[c];
    for (int k = 0; k < 3; ++k) g[k] = bgrad[(size_t)k * n + c] * pc;
    for (int q = 0; q < W; ++q) {
        const int e = ref[(size_t)q * n + c];
        if (e < 0) continue;
        const int f = e >> 1;
        const double pf = 0.5 * (p[owner[f]] + p[nb[f]]);
        const double sgn = (e & 1) ? -(double)fsgn[f] : (double)fsgn[f];
        g[fdir[f]] += sgn * pf;
    }
    for (int k = 0; k < 3; ++k) g[k] *= inv_h;
}

// momentum: face coefficients from phi
__global__ __launch_bounds__(kPisoBs) void k_mom_faces(const double* __restrict__ phi, int F, double D,
                                                      double* __restrict__ upper, double* __restrict__ lower) {
    FV_PISO_LOOP(f, F) {
        const double ph = phi[f];
        upper[f] = -D - fmax(-ph, 0.0);
        lower[f] = -D - fmax(ph, 0.0);
    }
}

// momentum: diagonal, H source and the predictor's right-hand side
__global__ __launch_bounds__(kPisoBs) void k_mom_cells(const int* __restrict__ ref, const int* __restrict__ owner,
                                                      const int* __restrict__ nb, const int8_t* __restrict__ fdir,
                                                      const int8_t* __restrict__ fsgn, const double* __restrict__ phi,
                                                      const double* __restrict__ bwall,
                                                      const double* __restrict__ blid,
                                                      const double* __restrict__ bgrad, const double* __restrict__ U,
                                                      const double* __restrict__ p, int n, int W, double h, double D,
                                                      double dt, double* __restrict__ diag, double* __restrict__ bH,
                                                      double* __restrict__ rhs) {
    const double V = h * h * h, vdt = V / dt;
    FV_PISO_LOOP(c, n) {
        double d = vdt + bwall[c];
        for (int q = 0; q < W; ++q) {
            const int e = ref[(size_t)q * n + c];
            if (e < 0) continue;
            const double ph = phi[e >> 1];
            d += D + ((e & 1) ? fmax(-ph, 0.0) : fmax(ph, 0.0));
        }
        diag[c] = d;
        double g[3];
        cell_gradp(ref, owner, nb, fdir, fsgn, bgrad, p, n, W, c, 1.0 / h, g);
        for (int k = 0; k < 3; ++k) {
            const double b = vdt * U[(size_t)k * n + c] + (k == 0 ? blid[c] : 0.0);
            bH[(size_t)k * n + c] = b;
            rhs[(size_t)k * n + c] = b - V * g[k];
        }
    }
}

// HbyA_k = (bH_k - sum over the row's slots of a_cj U_kj) / diag, rAU = V / diag,
// from the momentum matrix's slot layout
__global__ __launch_bounds__(kPisoBs) void k_hbya(const int* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ diag, const double* __restrict__ bH,
                                                 const double* __restrict__ U, int n, int W, double V,
                                                 double* __restrict__ HbyA, double* __restrict__ rAU) {
    FV_PISO_LOOP(c, n) {
        const double d = diag[c];
        for (int k = 0; k < 3; ++k) {
            double s = bH[(size_t)k * n + c];
            const double* Uk = U + (size_t)k * n;
            for (int q = 0; q < W; ++q) s -= val[(size_t)q * n + c] * Uk[col[(size_t)q * n + c]];
            HbyA[(size_t)k * n + c] = s / d;
        }
        rAU[c] = V / d;
    }
}

// phiHbyA, c_f and the pinned pressure couplings
__global__ __launch_bounds__(kPisoBs) void k_pres_faces(const int* __restrict__ owner, const int* __restrict__ nb,
                                                       const int8_t* __restrict__ fdir,
                                                       const int8_t* __restrict__ fsgn,
                                                       const double* __restrict__ HbyA, const double* __restrict__ rAU,
                                                       int n, int F, double h, double* __restrict__ phiH,
                                                       double* __restrict__ cf, double* __restrict__ pupper) {
    FV_PISO_LOOP(f, F) {
        const int o = owner[f], m = nb[f];
        const double* Hk = HbyA + (size_t)fdir[f] * n;
        phiH[f] = (double)fsgn[f] * h * h * (0.5 * (Hk[o] + Hk[m]));
        const double c = h * (0.5 * (rAU[o] + rAU[m]));
        cf[f] = c;
        pupper[f] = (o == 0 || m == 0) ? 0.0 : -c;
    }
}

// pressure diagonal (every face's c_f) and right-hand side -div(phiHbyA), b_0 = 0
__global__ __launch_bounds__(kPisoBs) void k_pres_cells(const int* __restrict__ ref, const double* __restrict__ phiH,
                                                       const double* __restrict__ cf, int n, int W,
                                                       double* __restrict__ pdiag, double* __restrict__ prhs) {
    FV_PISO_LOOP(c, n) {
        double d = 0.0, div = 0.0;
        for (int q = 0; q < W; ++q) {
            const int e = ref[(size_t)q * n + c];
            if (e < 0) continue;
            const int f = e >> 1;
            d += cf[f];
            div += (e & 1) ? -phiH[f] : phiH[f];
        }
        pdiag[c] = d;
        prhs[c] = c == 0 ? 0.0 : -div;
    }
}

// phi = phiHbyA - c_f (p_n - p_o)
__global__ __launch_bounds__(kPisoBs) void k_flux(const int* __restrict__ owner, const int* __restrict__ nb,
                                                 const double* __restrict__ phiH, const double* __restrict__ cf,
                                                 const double* __restrict__ p, int F, double* __restrict__ phi) {
    FV_PISO_LOOP(f, F) phi[f] = phiH[f] - cf[f] * (p[nb[f]] - p[owner[f]]);
}

// U_k = HbyA_k - rAU (grad p)_k
__global__ __launch_bounds__(kPisoBs) void k_ucorr(const int* __restrict__ ref, const int* __restrict__ owner,
                                                  const int* __restrict__ nb, const int8_t* __restrict__ fdir,
                                                  const int8_t* __restrict__ fsgn, const double* __restrict__ bgrad,
                                                  const double* __restrict__ p, const double* __restrict__ HbyA,
                                                  const double* __restrict__ rAU, int n, int W, double h,
                                                  double* __restrict__ U) {
    FV_PISO_LOOP(c, n) {
        double g[3];
        cell_gradp(ref, owner, nb, fdir, fsgn, bgrad, p, n, W, c, 1.0 / h, g);
        const double r = rAU[c];
        for (int k = 0; k < 3; ++k) U[(size_t)k * n + c] = HbyA[(size_t)k * n + c] - r * g[k];
    }
}

// bad = 1 if a face axis is outside {0, 1, 2} or an orientation outside {-1, +1}
__global__ __launch_bounds__(kPisoBs) void k_check_geom(const int8_t* __restrict__ fdir,
                                                       const int8_t* __restrict__ fsgn, int F, int* bad) {
    int b = 0;
    FV_PISO_LOOP(f, F) {
        const int d = fdir[f], g = fsgn[f];
        if (d < 0 || d > 2 || (g != 1 && g != -1)) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kPisoBs) void k_fill_unit(double* __restrict__ d, int n, double* __restrict__ a,
                                                      double* __restrict__ b, int F) {
    FV_PISO_LOOP(i, n) d[i] = 1.0;
    FV_PISO_LOOP(f, F) {
        a[f] = 0.0;
        if (b) b[f] = 0.0;
    }
}

}  // namespace

int piso_mesh_n(const fvpcg_piso* ps) { return ps->mesh->n; }
int piso_mesh_f(const fvpcg_piso* ps) { return ps->mesh->F; }

void piso_free(fvpcg_piso* ps) {
    if (!ps) return;
    amg_free(ps->amg);  // before the matrix it refers to
    if (ps->mom) matrix_destroy(ps->mom);
    if (ps->pres) matrix_destroy(ps->pres);
    int8_t* i8[] = {ps->fdir, ps->fsgn};
    for (int8_t* p : i8) dev_free(p);
    double* dv[] = {ps->bwall, ps->blid, ps->bgrad, ps->mdiag, ps->mupper, ps->mlower, ps->bH, ps->rhs,
                    ps->HbyA, ps->rAU, ps->pdiag, ps->prhs, ps->phiH, ps->cf, ps->pupper};
    for (double* p : dv) dev_free(p);
    delete ps;
}

int piso_create(const fvpcg_mesh* m, const int8_t* face_dir, const int8_t* face_sgn, const double* bwall,
                const double* blid, const double* bgrad, double h, double nu, int psolver, hipStream_t s,
                fvpcg_piso** out) {
    fvpcg_piso* ps = new (std::nothrow) fvpcg_piso();
    if (!ps) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    ps->mesh = m;
    ps->h = h;
    ps->nu = nu;
    ps->psolver = psolver;
    const size_t n = (size_t)std::max(m->n, 1), F = (size_t)std::max(m->F, 1);
    int rc;
    auto fail = [&](int code) {
        piso_free(ps);
        return code;
    };
    if ((rc = dev_alloc(&ps->fdir, F, "face axes")) || (rc = dev_alloc(&ps->fsgn, F, "face orientations")) ||
        (rc = dev_alloc(&ps->bwall, n, "wall coefficients")) || (rc = dev_alloc(&ps->blid, n, "lid sources")) ||
        (rc = dev_alloc(&ps->bgrad, 3 * n, "boundary normals")) || (rc = dev_alloc(&ps->mdiag, n, "momentum")) ||
        (rc = dev_alloc(&ps->mupper, F, "momentum")) || (rc = dev_alloc(&ps->mlower, F, "momentum")) ||
        (rc = dev_alloc(&ps->bH, 3 * n, "H source")) || (rc = dev_alloc(&ps->rhs, 3 * n, "momentum right-hand side")) ||
        (rc = dev_alloc(&ps->HbyA, 3 * n, "HbyA")) || (rc = dev_alloc(&ps->rAU, n, "rAU")) ||
        (rc = dev_alloc(&ps->pdiag, n, "pressure")) || (rc = dev_alloc(&ps->prhs, n, "pressure right-hand side")) ||
        (rc = dev_alloc(&ps->phiH, F, "phiHbyA")) || (rc = dev_alloc(&ps->cf, F, "pressure faces")) ||
        (rc = dev_alloc(&ps->pupper, F, "pressure faces")))
        return fail(rc);
    if (m->F > 0) {
        if (hipMemcpyAsync(ps->fdir, face_dir, (size_t)m->F, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(ps->fsgn, face_sgn, (size_t)m->F, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(hip_fail(hipGetLastError(), "copy of the face geometry", __FILE__, __LINE__));
    }
    if (m->F > 0) {  // the kernels index by face_dir: refuse anything else before the first step
        int* bad = nullptr;
        int hbad = 0;
        if ((rc = dev_alloc(&bad, 1, "geometry check"))) return fail(rc);
        bool ok = hipMemsetAsync(bad, 0, sizeof(int), s) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(k_check_geom, dim3(pgrid(m->F)), dim3(kPisoBs), 0, s, ps->fdir, ps->fsgn, m->F, bad);
            ok = hipGetLastError() == hipSuccess &&
                 hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
                 hipStreamSynchronize(s) == hipSuccess;
        }
        dev_free(bad);
        if (!ok) return fail(set_error(FVPCG_DEVICE_ERROR, "face geometry check failed"));
        if (hbad) return fail(set_error(FVPCG_INVALID_ARG, "face_dir must be 0, 1 or 2 and face_sgn +1 or -1"));
    }
    if (hipMemcpyAsync(ps->bwall, bwall, sizeof(double) * (size_t)m->n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ps->blid, blid, sizeof(double) * (size_t)m->n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ps->bgrad, bgrad, sizeof(double) * 3 * (size_t)m->n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(hip_fail(hipGetLastError(), "copy of the boundary terms", __FILE__, __LINE__));
    // both matrices start as the identity; every step assembles them
    hipLaunchKernelGGL(k_fill_unit, dim3(pgrid(std::max(m->n, m->F))), dim3(kPisoBs), 0, s, ps->mdiag, m->n,
                       ps->mupper, ps->mlower, m->F);
    hipLaunchKernelGGL(k_fill_unit, dim3(pgrid(std::max(m->n, m->F))), dim3(kPisoBs), 0, s, ps->pdiag, m->n,
                       ps->pupper, nullptr, m->F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(hip_fail(e, "kernel launch", __FILE__, __LINE__));
    if ((rc = matrix_create(m, ps->mdiag, ps->mupper, ps->mlower, 0, s, &ps->mom))) return fail(rc);
    if ((rc = matrix_create(m, ps->pdiag, ps->pupper, nullptr, 0, s, &ps->pres))) return fail(rc);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(hip_fail(hipGetLastError(), "sync", __FILE__, __LINE__));
    *out = ps;
    return FVPCG_OK;
}

// nsteps PISO steps; U [3][n], p [n], phi [F] in/out.  stats[0]: the
// momentum predictor (iters = BiCGSTAB iterations summed over components and
// steps, outer_iters = steps done, device_ms = the whole run); stats[1]: the
// pressure solves (iters summed, outer_iters = solves, true_rel_res of the
// last).  Returns the first non-OK solver status.
int piso_run(fvpcg_piso* ps, double dt, int nsteps, int n_corr, double* U, double* p, double* phi, double tol_u,
             double tol_p, int maxit, hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = ps->mesh;
    const int n = m->n, F = m->F, W = m->W;
    const double h = ps->h, D = ps->nu * h, V = h * h * h;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return set_error(FVPCG_DEVICE_ERROR, "event creation failed");
    }
    (void)hipEventRecord(e0, s);
    long long iu = 0, ip = 0;
    int rc = FVPCG_OK, step = 0, solves = 0;
    fvpcg_stats su{}, sp{};
    fvpcg_stats comp[3];
    const int gn = pgrid(n), gf = pgrid(F);
    for (step = 0; step < nsteps && rc == FVPCG_OK; ++step) {
        if (F > 0)
            hipLaunchKernelGGL(k_mom_faces, dim3(gf), dim3(kPisoBs), 0, s, phi, F, D, ps->mupper, ps->mlower);
        hipLaunchKernelGGL(k_mom_cells, dim3(gn), dim3(kPisoBs), 0, s, m->ref, m->owner, m->nb, ps->fdir, ps->fsgn,
                           phi, ps->bwall, ps->blid, ps->bgrad, U, p, n, W, h, D, dt, ps->mdiag, ps->bH, ps->rhs);
        FV_LAUNCHED();
        if ((rc = matrix_update(ps->mom, ps->mdiag, ps->mupper, ps->mlower, s))) break;
        rc = solve_bicgstab_multi(ps->mom, 3, ps->rhs, U, tol_u, maxit, FVPCG_PRECOND_JACOBI, s, comp);
        for (int k = 0; k < 3; ++k) iu += comp[k].iters;
        su = comp[0];
        if (rc != FVPCG_OK) break;
        for (int corr = 0; corr < n_corr && rc == FVPCG_OK; ++corr) {
            hipLaunchKernelGGL(k_hbya, dim3(gn), dim3(kPisoBs), 0, s, m->col, ps->mom->val, ps->mdiag, ps->bH, U, n,
                               W, V, ps->HbyA, ps->rAU);
            if (F > 0)
                hipLaunchKernelGGL(k_pres_faces, dim3(gf), dim3(kPisoBs), 0, s, m->owner, m->nb, ps->fdir, ps->fsgn,
                                   ps->HbyA, ps->rAU, n, F, h, ps->phiH, ps->cf, ps->pupper);
            hipLaunchKernelGGL(k_pres_cells, dim3(gn), dim3(kPisoBs), 0, s, m->ref, ps->phiH, ps->cf, n, W,
                               ps->pdiag, ps->prhs);
            FV_LAUNCHED();
            if (corr == 0) {  // rAU, and so the pressure matrix, is fixed within a step
                if ((rc = matrix_update(ps->pres, ps->pdiag, ps->pupper, nullptr, s))) break;
                // AMG: built on the first step, then refreshed numerically (the
                // pressure matrix keeps its pattern; its aggregates are kept)
                if (ps->psolver == FVPCG_PSOLVER_AMG) {
                    if (!ps->amg)
                        rc = amg_create(ps->pres, kPisoAmgTheta, 12, 64, 1, s, &ps->amg);
                    else
                        rc = amg_update(ps->amg, s);
                    if (rc) break;
                }
            }
            if (ps->psolver == FVPCG_PSOLVER_AMG)
                rc = solve_amg(ps->amg, ps->prhs, p, tol_p, maxit, FVPCG_CG, s, &sp);
            else
                rc = solve(ps->pres, ps->prhs, p, tol_p, maxit, FVPCG_CG, FVPCG_PRECOND_JACOBI, s, &sp);
            ip += sp.iters;
            ++solves;
            if (rc != FVPCG_OK) break;
            if (F > 0) hipLaunchKernelGGL(k_flux, dim3(gf), dim3(kPisoBs), 0, s, m->owner, m->nb, ps->phiH, ps->cf, p, F, phi);
            hipLaunchKernelGGL(k_ucorr, dim3(gn), dim3(kPisoBs), 0, s, m->ref, m->owner, m->nb, ps->fdir, ps->fsgn,
                               ps->bgrad, p, ps->HbyA, ps->rAU, n, W, h, U);
            FV_LAUNCHED();
        }
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        stats[0] = su;
        stats[0].iters = (int32_t)std::min<long long>(iu, INT32_MAX);
        stats[0].outer_iters = step;
        stats[0].device_ms = ms;
        stats[1] = sp;
        stats[1].iters = (int32_t)std::min<long long>(ip, INT32_MAX);
        stats[1].outer_iters = solves;
        stats[1].device_ms = ms;
        if (rc != FVPCG_OK) stats[0].status = rc;
    }
    return rc;
}

}  // namespace fvpcg
