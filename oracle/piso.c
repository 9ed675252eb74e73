/*
 * CPU oracle, icoFoam's PISO time step -- TEST INFRASTRUCTURE.
 *
 * Section 2 names icoFoam (incompressible laminar Navier-Stokes) among the
 * applications whose linear systems the solver is called for, and splits
 * its PISO step into a momentum predictor (BiCGSTAB), pressure solutions
 * (CG) and explicit velocity corrections; Section 4.1 adds that the
 * application invokes the solver repeatedly.  Written from the finite-volume
 * PISO algorithm on the LDU addressing of a box of cubes of side h
 * (V = h^3, face area h^2, centre distance h, w = area / distance = h):
 *
 * momentum (implicit Euler, first-order upwind convection of the face flux
 * phi_f, owner -> neighbour), one matrix for the three components:
 *   upper_f = -nu w - max(-phi_f, 0),   lower_f = -nu w - max(phi_f, 0),
 *   diag_c  = V/dt + sum over c's faces of (nu w + outflow_f, if > 0) + bwall_c,
 *   bH_kc   = (V/dt) U_kc + blid_c [k = x];
 * pressure gradient (Gauss, linear face values, zero-gradient walls):
 *   (grad p)_kc = (1/h) [ sum over c's faces along k of n_cf p_f + bgrad_kc p_c ],
 *   n_cf = the face's outward unit normal component (face_sgn for the owner,
 *   -face_sgn for the neighbour), p_f = (p_o + p_n) / 2;
 * predictor: solve A U_k = bH_k - V (grad p)_k, k = x, y, z (BiCGSTAB, Jacobi,
 * from the old U);
 * each of n_corr correctors:
 *   rAU_c = V / diag_c,  HbyA_kc = (bH_kc - sum_n a_cn U_kn) / diag_c,
 *   phiHbyA_f = face_sgn_f h^2 (HbyA_{d,o} + HbyA_{d,n}) / 2, d = face_dir_f,
 *   pressure: sum_f c_f (p_c - p_other) = -div(phiHbyA)_c, c_f = w (rAU_o +
 *   rAU_n) / 2, div(phi)_c = sum over owned faces of phi_f - sum over
 *   neighboured faces; the singular Neumann system made definite by pinning
 *   cell 0 (its couplings zeroed in both triangles, b_0 = 0, p_0 = 0); CG
 *   with Jacobi from the previous p;
 *   phi_f = phiHbyA_f - c_f (p_n - p_o),   U_kc = HbyA_kc - rAU_c (grad p)_kc.
 * After a corrector div(phi) vanishes up to the pressure tolerance.  Plain C,
 * FP64, single thread.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Momentum matrix of the step from phi and the H source from U_old. */
void or_piso_momentum(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const double* phi,
                      const double* bwall, const double* blid, double h, double nu, double dt, const double* U_old,
                      double* diag, double* upper, double* lower, double* bH)
{
    const double V = h * h * h, D = nu * h;
    for (int32_t c = 0; c < n; ++c) {
        diag[c] = V / dt + bwall[c];
        for (int32_t k = 0; k < 3; ++k) bH[(size_t)k * n + c] = V / dt * U_old[(size_t)k * n + c];
        bH[c] += blid[c];
    }
    for (int32_t f = 0; f < nf; ++f) {
        const double F = phi[f];
        upper[f] = -D - fmax(-F, 0.0);
        lower[f] = -D - fmax(F, 0.0);
        diag[owner[f]] += D + fmax(F, 0.0);
        diag[nb[f]] += D + fmax(-F, 0.0);
    }
}

/* (grad p)_k for every cell, [3][n]. */
void or_piso_gradp(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                   const int8_t* face_sgn, const double* bgrad, double h, const double* p, double* g)
{
    for (int32_t k = 0; k < 3; ++k)
        for (int32_t c = 0; c < n; ++c) g[(size_t)k * n + c] = bgrad[(size_t)k * n + c] * p[c];
    for (int32_t f = 0; f < nf; ++f) {
        const int32_t o = owner[f], m = nb[f], k = face_dir[f];
        const double pf = 0.5 * (p[o] + p[m]);
        g[(size_t)k * n + o] += face_sgn[f] * pf;
        g[(size_t)k * n + m] -= face_sgn[f] * pf;
    }
    for (size_t e = 0; e < (size_t)3 * n; ++e) g[e] /= h;
}

/* div(phi)_c: net outflow of every cell through its internal faces. */
void or_piso_div(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const double* phi, double* div)
{
    for (int32_t c = 0; c < n; ++c) div[c] = 0.0;
    for (int32_t f = 0; f < nf; ++f) {
        div[owner[f]] += phi[f];
        div[nb[f]] -= phi[f];
    }
}

/* One corrector's pressure system from the current U and the momentum
 * matrix: pdiag, pupper (pinned: cell 0's couplings zero), its right-hand
 * side, the unpinned face coefficients cf, HbyA [3][n], rAU and phiHbyA. */
void or_piso_pressure_system(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                             const int8_t* face_sgn, double h, const double* diag, const double* upper,
                             const double* lower, const double* bH, const double* U, double* HbyA, double* rAU,
                             double* phiHbyA, double* cf, double* pdiag, double* pupper, double* prhs)
{
    const double V = h * h * h;
    for (int32_t k = 0; k < 3; ++k) {
        double* Hk = HbyA + (size_t)k * n;
        const double* Uk = U + (size_t)k * n;
        memcpy(Hk, bH + (size_t)k * n, sizeof(double) * (size_t)n);
        for (int32_t f = 0; f < nf; ++f) {
            Hk[owner[f]] -= upper[f] * Uk[nb[f]];
            Hk[nb[f]] -= lower[f] * Uk[owner[f]];
        }
        for (int32_t c = 0; c < n; ++c) Hk[c] /= diag[c];
    }
    for (int32_t c = 0; c < n; ++c) {
        rAU[c] = V / diag[c];
        pdiag[c] = 0.0;
    }
    for (int32_t f = 0; f < nf; ++f) {
        const int32_t o = owner[f], m = nb[f], k = face_dir[f];
        phiHbyA[f] = face_sgn[f] * h * h * 0.5 * (HbyA[(size_t)k * n + o] + HbyA[(size_t)k * n + m]);
        cf[f] = h * 0.5 * (rAU[o] + rAU[m]);
        pdiag[o] += cf[f];
        pdiag[m] += cf[f];
        pupper[f] = (o == 0 || m == 0) ? 0.0 : -cf[f];
    }
    or_piso_div(n, nf, owner, nb, phiHbyA, prhs);
    for (int32_t c = 0; c < n; ++c) prhs[c] = -prhs[c];
    if (n > 0) prhs[0] = 0.0;
}

int32_t or_piso_run(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                    const int8_t* face_sgn, const double* bwall, const double* blid, const double* bgrad, double h,
                    double nu, double dt, int32_t nsteps, int32_t n_corr, double* U, double* p, double* phi,
                    double tol_u, double tol_p, int32_t maxit, int32_t* iters_u, int32_t* iters_p)
{
    const double V = h * h * h;
    const size_t nn = (size_t)(n > 0 ? n : 1), ff = (size_t)(nf > 0 ? nf : 1);
    double *diag = malloc(sizeof(double) * nn), *upper = malloc(sizeof(double) * ff);
    double *lower = malloc(sizeof(double) * ff), *bH = malloc(sizeof(double) * 3 * nn);
    double *rhs = malloc(sizeof(double) * nn), *g = malloc(sizeof(double) * 3 * nn);
    double *HbyA = malloc(sizeof(double) * 3 * nn), *rAU = malloc(sizeof(double) * nn);
    double *phiH = malloc(sizeof(double) * ff), *cf = malloc(sizeof(double) * ff);
    double *pdiag = malloc(sizeof(double) * nn), *pupper = malloc(sizeof(double) * ff);
    double* prhs = malloc(sizeof(double) * nn);
    int32_t status = OR_OK, iu = 0, ip = 0;
    for (int32_t s = 0; s < nsteps && status == OR_OK; ++s) {
        or_piso_momentum(n, nf, owner, nb, phi, bwall, blid, h, nu, dt, U, diag, upper, lower, bH);
        /* predictor with the old pressure gradient */
        or_piso_gradp(n, nf, owner, nb, face_dir, face_sgn, bgrad, h, p, g);
        for (int32_t k = 0; k < 3 && status == OR_OK; ++k) {
            for (int32_t c = 0; c < n; ++c) rhs[c] = bH[(size_t)k * n + c] - V * g[(size_t)k * n + c];
            or_stats st;
            status = or_bicgstab(n, nf, owner, nb, diag, upper, lower, rhs, U + (size_t)k * n, tol_u, maxit,
                                 OR_PRECOND_JACOBI, &st, NULL, NULL, NULL);
            iu += st.iters;
        }
        for (int32_t corr = 0; corr < n_corr && status == OR_OK; ++corr) {
            or_piso_pressure_system(n, nf, owner, nb, face_dir, face_sgn, h, diag, upper, lower, bH, U, HbyA, rAU,
                                    phiH, cf, pdiag, pupper, prhs);
            or_stats st;
            status = or_cg(n, nf, owner, nb, pdiag, pupper, pupper, prhs, p, tol_p, maxit, OR_PRECOND_JACOBI, &st,
                           NULL, NULL, NULL);
            ip += st.iters;
            for (int32_t f = 0; f < nf; ++f) phi[f] = phiH[f] - cf[f] * (p[nb[f]] - p[owner[f]]);
            or_piso_gradp(n, nf, owner, nb, face_dir, face_sgn, bgrad, h, p, g);
            for (int32_t k = 0; k < 3; ++k)
                for (int32_t c = 0; c < n; ++c)
                    U[(size_t)k * n + c] = HbyA[(size_t)k * n + c] - rAU[c] * g[(size_t)k * n + c];
        }
    }
    if (iters_u) *iters_u = iu;
    if (iters_p) *iters_p = ip;
    free(diag); free(upper); free(lower); free(bH); free(rhs); free(g); free(HbyA); free(rAU);
    free(phiH); free(cf); free(pdiag); free(pupper); free(prhs);
    return status;
}
