/*
 * CPU oracle, BiCGSTAB for non-symmetric LDU matrices -- TEST INFRASTRUCTURE.
 *
 * Section 2 names the second workload's solvers: icoFoam's PISO loop solves
 * the momentum equation with BiCGSTAB and the pressure equation with CG.
 * The momentum matrix carries convection, so lower != upper.  The paper does
 * not print the algorithm; this is van der Vorst's Bi-CGSTAB (SIAM J. Sci.
 * Stat. Comput. 13, 1992) in its preconditioned form with the preconditioner
 * applied to the search directions (right preconditioning, so r stays the
 * residual of A x = b):
 *
 *   r0 = b - A x0,  rhat = r0,  rho_0 = alpha = omega = 1
 *   for i = 1, 2, ...
 *     rho_i = (rhat, r)                      breakdown if 0
 *     p = r                                  (i = 1)
 *     p = r + (rho_i/rho_{i-1})(alpha/omega) (p - omega v)   (i > 1)
 *     phat = M^-1 p;  v = A phat;  alpha = rho_i / (rhat, v)  (breakdown if (rhat,v) = 0)
 *     s = r - alpha v
 *     if ||s|| <= tol ||b||: x += alpha phat, stop (half step)
 *     shat = M^-1 s;  t = A shat;  omega = (t, s) / (t, t)  (breakdown if 0)
 *     x += alpha phat + omega shat
 *     r = s - omega t;  stop if ||r|| <= tol ||b||
 *
 * M = I or the diagonal (Jacobi).  Every step is written out with the
 * oracle's plain LDU product and sequential dot product.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>

static void apply_m(int32_t n, int32_t precond, const double* diag, const double* in, double* out)
{
    for (int32_t c = 0; c < n; ++c) out[c] = precond == OR_PRECOND_JACOBI ? in[c] / diag[c] : in[c];
}

int32_t or_bicgstab(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                    const double* diag, const double* upper, const double* lower,
                    const double* b, double* x, double tol, int32_t maxit, int32_t precond,
                    or_stats* st, double* alpha_hist, double* omega_hist, double* res_hist)
{
    double* r = malloc(sizeof(double) * (size_t)n * 8 + 8);
    double* rhat = r + n;
    double* p = rhat + n;
    double* v = p + n;
    double* s = v + n;
    double* t = s + n;
    double* ph = t + n;
    double* sh = ph + n;
    const double bnorm = sqrt(or_dot(n, b, b));
    int32_t status = OR_NOT_CONVERGED, it = 0;
    double rnorm;

    or_spmv(n, nf, owner, nb, diag, upper, lower, x, r);
    for (int32_t c = 0; c < n; ++c) {
        r[c] = b[c] - r[c];
        rhat[c] = r[c];
        p[c] = 0.0;
        v[c] = 0.0;
    }
    rnorm = sqrt(or_dot(n, r, r));
    if (st) st->r0_norm = rnorm;
    if (res_hist) res_hist[0] = rnorm;
    const double tol_abs = tol * bnorm;
    if (bnorm == 0.0) {
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        rnorm = 0.0;
        status = OR_OK;
        goto done;
    }
    if (rnorm <= tol_abs) {
        status = OR_OK;
        goto done;
    }
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    while (it < maxit) {
        const double rho = or_dot(n, rhat, r);
        if (rho == 0.0 || !isfinite(rho)) {
            status = OR_BREAKDOWN;
            break;
        }
        if (it == 0) {
            for (int32_t c = 0; c < n; ++c) p[c] = r[c];
        } else {
            const double beta = (rho / rho_prev) * (alpha / omega);
            for (int32_t c = 0; c < n; ++c) p[c] = r[c] + beta * (p[c] - omega * v[c]);
        }
        apply_m(n, precond, diag, p, ph);
        or_spmv(n, nf, owner, nb, diag, upper, lower, ph, v);
        const double rv = or_dot(n, rhat, v);
        alpha = rho / rv;
        if (rv == 0.0 || !isfinite(alpha)) {
            status = OR_BREAKDOWN;
            break;
        }
        for (int32_t c = 0; c < n; ++c) s[c] = r[c] - alpha * v[c];
        const double snorm = sqrt(or_dot(n, s, s));
        ++it;
        if (alpha_hist) alpha_hist[it - 1] = alpha;
        if (snorm <= tol_abs) {
            for (int32_t c = 0; c < n; ++c) x[c] += alpha * ph[c];
            for (int32_t c = 0; c < n; ++c) r[c] = s[c];
            rnorm = snorm;
            if (omega_hist) omega_hist[it - 1] = 0.0;
            if (res_hist) res_hist[it] = rnorm;
            status = OR_OK;
            break;
        }
        apply_m(n, precond, diag, s, sh);
        or_spmv(n, nf, owner, nb, diag, upper, lower, sh, t);
        const double tt = or_dot(n, t, t);
        omega = or_dot(n, t, s) / tt;
        if (tt == 0.0 || omega == 0.0 || !isfinite(omega)) {
            status = OR_BREAKDOWN;
            break;
        }
        for (int32_t c = 0; c < n; ++c) x[c] += alpha * ph[c] + omega * sh[c];
        for (int32_t c = 0; c < n; ++c) r[c] = s[c] - omega * t[c];
        rnorm = sqrt(or_dot(n, r, r));
        if (omega_hist) omega_hist[it - 1] = omega;
        if (res_hist) res_hist[it] = rnorm;
        if (rnorm <= tol_abs) {
            status = OR_OK;
            break;
        }
        rho_prev = rho;
    }
done:
    if (st) {
        st->iters = it;
        st->outer_iters = 0;
        st->status = status;
        st->b_norm = bnorm;
        st->rel_res = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        or_spmv(n, nf, owner, nb, diag, upper, lower, x, t);
        for (int32_t c = 0; c < n; ++c) t[c] = b[c] - t[c];
        st->true_rel_res = bnorm > 0.0 ? sqrt(or_dot(n, t, t)) / bnorm : 0.0;
    }
    free(r);
    return status;
}
