/*
 * CPU oracle, transient diffusion (laplacianFoam) -- TEST INFRASTRUCTURE.
 *
 * Section 2 names laplacianFoam's heat equation dT/dt = div(k grad T) as a
 * workload whose linear systems the solver is called for every time step.
 * Finite volumes on the LDU addressing with implicit Euler:
 *   (V_c / dt) (T'_c - T_c) = sum over faces f of c of k_f w_f (T'_other - T'_c)
 *                            - bdiag_c T'_c + bsrc_c,
 * w_f = |S_f| / |d_f|, bdiag and bsrc the Dirichlet (and source) terms.  As
 * an LDU system A T' = b:
 *   upper_f = lower_f = -k_f w_f,
 *   diag_c  = V_c / dt + sum_{f of c} k_f w_f + bdiag_c,
 *   b_c     = (V_c / dt) T_c + bsrc_c.
 * Each step is solved by the oracle's Jacobi-PCG from the previous field.
 */
#include "oracle.h"

#include <stdlib.h>

void or_assemble_transient(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                           const double* k, const double* w, const double* vol, const double* bdiag,
                           const double* bsrc, double dt, const double* T_old,
                           double* diag, double* upper, double* b)
{
    for (int32_t c = 0; c < n; ++c) {
        diag[c] = vol[c] / dt + bdiag[c];
        b[c] = vol[c] / dt * T_old[c] + bsrc[c];
    }
    for (int32_t f = 0; f < nf; ++f) {
        const double a = k[f] * w[f];
        upper[f] = -a;
        diag[owner[f]] += a;
        diag[nb[f]] += a;
    }
}

int32_t or_transient_run(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                         const double* k, const double* w, const double* vol, const double* bdiag,
                         const double* bsrc, double dt, int32_t nsteps, double* T, double tol, int32_t maxit,
                         int32_t* total_iters)
{
    double* diag = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* upper = malloc(sizeof(double) * (size_t)(nf > 0 ? nf : 1));
    double* b = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t status = OR_OK, its = 0;
    for (int32_t s = 0; s < nsteps; ++s) {
        or_assemble_transient(n, nf, owner, nb, k, w, vol, bdiag, bsrc, dt, T, diag, upper, b);
        or_stats st;
        status = or_cg(n, nf, owner, nb, diag, upper, upper, b, T, tol, maxit, OR_PRECOND_JACOBI, &st,
                       NULL, NULL, NULL);
        its += st.iters;
        if (status != OR_OK) break;
    }
    if (total_iters) *total_iters = its;
    free(diag); free(upper); free(b);
    return status;
}
