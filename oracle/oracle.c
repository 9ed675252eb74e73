/*
 * CPU oracle for the finite-volume Laplacian CG solve -- TEST INFRASTRUCTURE.
 *
 * Written from the paper (AlOnazi, Keyes, Lastovetsky, Rychkov, arXiv
 * 1505.07630) and from the mathematics of the methods it names:
 *   - Section 2: A x = b with A square, symmetric positive (semi)definite;
 *     a CG iteration is a sparse matrix-vector product, an optional
 *     preconditioner, three global inner products and vector updates.
 *   - Section 4.1: the pipelined CG of Ghysels and Vanroose, one global
 *     reduction per iteration, overlapped with the matrix-vector product.
 *   - Section 5 / Table ai_cg: the kernels are memory bound; nothing here is
 *     blocked, fused or reordered beyond the definitions, except that inner
 *     products are summed pairwise (see or_dot).
 *
 * Plain FP64, single thread, built with -O2 -ffp-contract=off.  Used only by
 * tests, the smoke check and the benchmark's CPU-baseline leg.  A second
 * build with OpenMP (liboracle_omp.so) spreads or_cg's and or_pipecg's loops
 * over threads without changing a single rounding: see ldu_mv and dotp.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#define OR_PARFOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PARFOR
#endif

/* ---- LDU matrix-vector product (Section 4.2: nnz = n + 2F; Section 5:
 * OpenFOAM lduMatrix).  The plain definition: diagonal term, then each face
 * adds its upper coefficient to the owner row and its lower coefficient to
 * the neighbour row. */
void or_spmv(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
             const double* diag, const double* upper, const double* lower,
             const double* v, double* y)
{
    for (int32_t c = 0; c < n; ++c) y[c] = diag[c] * v[c];
    for (int32_t f = 0; f < nf; ++f) {
        y[owner[f]] += upper[f] * v[nb[f]];
        y[nb[f]] += lower[f] * v[owner[f]];
    }
}

/* Inner products are sums whose order the method does not fix; they are
 * evaluated by pairwise (cascade) summation, halving the range until at most
 * 8 terms remain, so the oracle's own rounding error grows like log2(n)
 * rather than sqrt(n) (the classical error analysis of recursive summation).
 * Comparisons then measure the device path, not the reference's summation
 * error. */
double or_dot(int32_t n, const double* a, const double* b)
{
    if (n <= 8) {
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    int32_t h = n / 2;
    return or_dot(h, a, b) + or_dot(n - h, a + h, b + h);
}

/* or_dot with the top six levels of its halving tree spread over threads
 * (OpenMP build): the 64 ranges of depth 6 are summed in parallel, each by
 * or_dot, and combined pairwise in the tree's own order, so the result is
 * bitwise or_dot's for any thread count. */
static double dotp(int32_t n, const double* a, const double* b)
{
#ifdef _OPENMP
    enum { DEPTH = 6, LEAVES = 1 << DEPTH };
    if (n >= 16 * LEAVES) {
        int32_t off[LEAVES], len[LEAVES];
        off[0] = 0;
        len[0] = n;
        for (int32_t d = 0, cnt = 1; d < DEPTH; ++d, cnt *= 2)
            for (int32_t k = cnt - 1; k >= 0; --k) {
                const int32_t o = off[k], l = len[k], h = l / 2;
                off[2 * k] = o;
                len[2 * k] = h;
                off[2 * k + 1] = o + h;
                len[2 * k + 1] = l - h;
            }
        double s[LEAVES];
        OR_PARFOR
        for (int32_t k = 0; k < LEAVES; ++k) s[k] = or_dot(len[k], a + off[k], b + off[k]);
        for (int32_t w = LEAVES; w > 1; w /= 2)
            for (int32_t k = 0; k < w / 2; ++k) s[k] = s[2 * k] + s[2 * k + 1];
        return s[0];
    }
#endif
    return or_dot(n, a, b);
}

int32_t or_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* The LDU product as or_cg and or_pipecg apply it: or_spmv's face loop.  In
 * the OpenMP build each row is evaluated on its own over its faces in
 * increasing face order (owner side: upper times the neighbour's value,
 * neighbour side: lower times the owner's), which is the sequence of
 * additions the face loop makes to that row: bitwise or_spmv's result. */
typedef struct {
    int32_t n, nf;
    const int32_t *owner, *nb;
    const double *diag, *upper, *lower;
    int32_t *fptr, *flist;  /* OpenMP build: row c's faces, 2f + side, at fptr[c] .. fptr[c+1] */
} ldu_t;

static void ldu_init(ldu_t* A, int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                     const double* diag, const double* upper, const double* lower)
{
    A->n = n; A->nf = nf; A->owner = owner; A->nb = nb;
    A->diag = diag; A->upper = upper; A->lower = lower;
    A->fptr = NULL; A->flist = NULL;
#ifdef _OPENMP
    A->fptr = calloc((size_t)n + 1, sizeof(int32_t));
    A->flist = malloc(sizeof(int32_t) * (size_t)(nf > 0 ? 2 * nf : 1));
    for (int32_t f = 0; f < nf; ++f) { A->fptr[owner[f] + 1]++; A->fptr[nb[f] + 1]++; }
    for (int32_t c = 0; c < n; ++c) A->fptr[c + 1] += A->fptr[c];
    int32_t* fill = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    memcpy(fill, A->fptr, sizeof(int32_t) * (size_t)n);
    for (int32_t f = 0; f < nf; ++f) {
        A->flist[fill[owner[f]]++] = 2 * f;
        A->flist[fill[nb[f]]++] = 2 * f + 1;
    }
    free(fill);
#endif
}

static void ldu_free(ldu_t* A)
{
    free(A->fptr);
    free(A->flist);
}

static void ldu_mv(const ldu_t* A, const double* v, double* y)
{
#ifdef _OPENMP
    OR_PARFOR
    for (int32_t c = 0; c < A->n; ++c) {
        double s = A->diag[c] * v[c];
        for (int32_t k = A->fptr[c]; k < A->fptr[c + 1]; ++k) {
            const int32_t f = A->flist[k] >> 1;
            if (A->flist[k] & 1) s += A->lower[f] * v[A->owner[f]];
            else s += A->upper[f] * v[A->nb[f]];
        }
        y[c] = s;
    }
#else
    or_spmv(A->n, A->nf, A->owner, A->nb, A->diag, A->upper, A->lower, v, y);
#endif
}

/* The same pairwise sum for FP32 vectors, accumulated in FP64. */
static double dot32(int32_t n, const float* a, const float* b)
{
    if (n <= 8) {
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += (double)a[i] * (double)b[i];
        return s;
    }
    int32_t h = n / 2;
    return dot32(h, a, b) + dot32(n - h, a + h, b + h);
}

static double* alloc_vec(int32_t n)
{
    return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
}

/* r = b - A x */
static void residual(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                     const double* diag, const double* upper, const double* lower,
                     const double* b, const double* x, double* r)
{
    or_spmv(n, nf, owner, nb, diag, upper, lower, x, r);
    for (int32_t c = 0; c < n; ++c) r[c] = b[c] - r[c];
}

/* z = M^-1 r for M = I or M = diag(A) (the "optional preconditioning" of
 * Section 2, taken as Jacobi). */
static void precond_apply(int32_t n, int32_t precond, const double* diag, const double* r, double* z)
{
    if (precond == OR_PRECOND_JACOBI) {
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) z[c] = r[c] / diag[c];
    } else {
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) z[c] = r[c];
    }
}

static int diag_positive(int32_t n, const double* diag)
{
    for (int32_t c = 0; c < n; ++c)
        if (!(diag[c] > 0.0) || !isfinite(diag[c])) return 0;
    return 1;
}

/* r = b - A x and the exit statistics through the context's product */
static void residual_ldu(const ldu_t* A, const double* b, const double* x, double* r)
{
    ldu_mv(A, x, r);
    OR_PARFOR
    for (int32_t c = 0; c < A->n; ++c) r[c] = b[c] - r[c];
}

static void finish_stats_ldu(const ldu_t* A, const double* b, const double* x, double bnorm, double rnorm,
                             or_stats* st)
{
    if (!st) return;
    double* r = alloc_vec(A->n);
    residual_ldu(A, b, x, r);
    const double tr = sqrt(dotp(A->n, r, r));
    free(r);
    st->b_norm = bnorm;
    st->rel_res = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    st->true_rel_res = bnorm > 0.0 ? tr / bnorm : 0.0;
}

/* ---- Standard preconditioned CG (Section 2).  The three inner products of
 * each iteration are delta = (p, A p), gamma = (r, z) and rho = (r, r); the
 * stopping test is ||r||_2 <= tol * ||b||_2 on the recursively updated,
 * unpreconditioned residual. */
int32_t or_cg(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
              const double* diag, const double* upper, const double* lower,
              const double* b, double* x, double tol, int32_t maxit, int32_t precond,
              or_stats* st, double* alpha_hist, double* beta_hist, double* res_hist)
{
    if (st) memset(st, 0, sizeof(*st));
    double bnorm = sqrt(dotp(n, b, b));
    if (bnorm == 0.0) {
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        if (st) { st->status = OR_OK; st->b_norm = 0.0; }
        if (res_hist) res_hist[0] = 0.0;
        return OR_OK;
    }
    if (precond == OR_PRECOND_JACOBI && !diag_positive(n, diag)) {
        if (st) { st->status = OR_BREAKDOWN; st->b_norm = bnorm; }
        return OR_BREAKDOWN;
    }
    double* r = alloc_vec(n);
    double* z = alloc_vec(n);
    double* p = alloc_vec(n);
    double* q = alloc_vec(n);
    ldu_t A;
    ldu_init(&A, n, nf, owner, nb, diag, upper, lower);

    residual_ldu(&A, b, x, r);
    precond_apply(n, precond, diag, r, z);
    memcpy(p, z, sizeof(double) * (size_t)n);
    double gamma = dotp(n, r, z);
    double rnorm = sqrt(dotp(n, r, r));
    if (st) st->r0_norm = rnorm;
    if (res_hist) res_hist[0] = rnorm;

    int32_t status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (rnorm <= tol * bnorm) {
        status = OR_OK;
    } else {
        for (k = 1; k <= maxit; ++k) {
            ldu_mv(&A, p, q);
            double delta = dotp(n, p, q);
            if (!(delta > 0.0) || !isfinite(delta) || !isfinite(gamma)) {
                status = OR_BREAKDOWN;
                k -= 1;
                break;
            }
            double alpha = gamma / delta;
            OR_PARFOR
            for (int32_t c = 0; c < n; ++c) x[c] += alpha * p[c];
            OR_PARFOR
            for (int32_t c = 0; c < n; ++c) r[c] -= alpha * q[c];
            precond_apply(n, precond, diag, r, z);
            double gamma_new = dotp(n, r, z);
            double rho = dotp(n, r, r);
            rnorm = sqrt(rho);
            if (alpha_hist) alpha_hist[k - 1] = alpha;
            if (res_hist) res_hist[k] = rnorm;
            if (rnorm <= tol * bnorm) {
                status = OR_OK;
                break;
            }
            double beta = gamma_new / gamma;
            if (beta_hist) beta_hist[k - 1] = beta;
            gamma = gamma_new;
            OR_PARFOR
            for (int32_t c = 0; c < n; ++c) p[c] = z[c] + beta * p[c];
        }
        if (k > maxit) k = maxit;
    }
    if (st) { st->iters = k; st->status = status; }
    finish_stats_ldu(&A, b, x, bnorm, rnorm, st);
    ldu_free(&A);
    free(r); free(z); free(p); free(q);
    return status;
}

/* ---- Pipelined preconditioned CG (Ghysels and Vanroose; Section 4.1).
 * Per iteration i: one reduction of gamma = (r,u), delta = (w,u) and
 * rho = (r,r); then m = M^-1 w and n = A m (the product the reduction would
 * overlap); the scalars come from the recurrences
 *   beta_i = gamma_i / gamma_{i-1},
 *   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
 * (beta_0 = 0, alpha_0 = gamma_0 / delta_0), and the vectors from
 *   z = n + beta z, q = m + beta q, s = w + beta s, p = u + beta p,
 *   x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z.
 * In the folded Jacobi form u = r/d, q = s/d and m = w/d are evaluated
 * instead of carried.  iters counts updates of x, as in or_cg. */
int32_t or_pipecg(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                  const double* diag, const double* upper, const double* lower,
                  const double* b, double* x, double tol, int32_t maxit, int32_t precond,
                  int32_t folded, or_stats* st, double* res_hist)
{
    if (st) memset(st, 0, sizeof(*st));
    if (folded && precond != OR_PRECOND_JACOBI) folded = 0;
    double bnorm = sqrt(dotp(n, b, b));
    if (bnorm == 0.0) {
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        if (st) st->status = OR_OK;
        if (res_hist) res_hist[0] = 0.0;
        return OR_OK;
    }
    if (precond == OR_PRECOND_JACOBI && !diag_positive(n, diag)) {
        if (st) { st->status = OR_BREAKDOWN; st->b_norm = bnorm; }
        return OR_BREAKDOWN;
    }
    double *r = alloc_vec(n), *u = alloc_vec(n), *w = alloc_vec(n), *m = alloc_vec(n);
    double *nv = alloc_vec(n), *z = alloc_vec(n), *q = alloc_vec(n), *s = alloc_vec(n);
    double *p = alloc_vec(n);
    ldu_t A;
    ldu_init(&A, n, nf, owner, nb, diag, upper, lower);

    residual_ldu(&A, b, x, r);
    precond_apply(n, precond, diag, r, u);
    ldu_mv(&A, u, w);

    double gamma_prev = 0.0, alpha_prev = 0.0, rnorm = 0.0;
    int32_t status = OR_NOT_CONVERGED;
    int32_t i;
    for (i = 0;; ++i) {
        if (folded) {
            OR_PARFOR
            for (int32_t c = 0; c < n; ++c) u[c] = r[c] / diag[c];
        }
        double gamma = dotp(n, r, u);
        double delta = dotp(n, w, u);
        double rho = dotp(n, r, r);
        rnorm = sqrt(rho);
        if (i == 0 && st) st->r0_norm = rnorm;
        if (res_hist) res_hist[i] = rnorm;
        if (rnorm <= tol * bnorm) { status = OR_OK; break; }
        if (i == maxit) { status = OR_NOT_CONVERGED; break; }

        precond_apply(n, precond, diag, w, m);
        ldu_mv(&A, m, nv);

        double alpha, beta, den;
        if (i == 0) {
            beta = 0.0;
            den = delta;
        } else {
            beta = gamma / gamma_prev;
            den = delta - beta * gamma / alpha_prev;
        }
        alpha = gamma / den;
        if (!(den > 0.0) || !isfinite(den) || !isfinite(alpha) || !isfinite(beta)) {
            status = OR_BREAKDOWN;
            break;
        }
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) {
            z[c] = nv[c] + beta * z[c];
            s[c] = w[c] + beta * s[c];
            p[c] = u[c] + beta * p[c];
            if (!folded) q[c] = m[c] + beta * q[c];
        }
        OR_PARFOR
        for (int32_t c = 0; c < n; ++c) {
            x[c] += alpha * p[c];
            r[c] -= alpha * s[c];
            if (!folded) u[c] -= alpha * q[c];
            w[c] -= alpha * z[c];
        }
        gamma_prev = gamma;
        alpha_prev = alpha;
    }
    if (st) { st->iters = i; st->status = status; }
    finish_stats_ldu(&A, b, x, bnorm, rnorm, st);
    ldu_free(&A);
    free(r); free(u); free(w); free(m); free(nv); free(z); free(q); free(s); free(p);
    return status;
}

/* ---- FP32 pieces for the refinement driver: the same LDU product and the
 * folded pipelined Jacobi-CG (O-3) in single precision, inner products
 * accumulated in double, stopped on its recursively updated residual. */

static void spmv32(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                   const float* diag, const float* upper, const float* lower,
                   const float* v, float* y)
{
    for (int32_t c = 0; c < n; ++c) y[c] = diag[c] * v[c];
    for (int32_t f = 0; f < nf; ++f) {
        y[owner[f]] += upper[f] * v[nb[f]];
        y[nb[f]] += lower[f] * v[owner[f]];
    }
}

/* y = A D^-1 v, with tmp as scratch */
static void spmv32_scaled(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                          const float* diag, const float* upper, const float* lower,
                          const float* v, float* tmp, float* y)
{
    for (int32_t c = 0; c < n; ++c) tmp[c] = v[c] / diag[c];
    spmv32(n, nf, owner, nb, diag, upper, lower, tmp, y);
}

static int32_t pipecg32_folded(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                               const float* diag, const float* upper, const float* lower,
                               const float* b, float* x, double tol, int32_t maxit, int32_t* iters)
{
    float *r = calloc((size_t)n, 4), *u = calloc((size_t)n, 4), *w = calloc((size_t)n, 4);
    float *m = calloc((size_t)n, 4), *nv = calloc((size_t)n, 4), *z = calloc((size_t)n, 4);
    float *s = calloc((size_t)n, 4), *p = calloc((size_t)n, 4);
    double bnorm = sqrt(dot32(n, b, b));
    spmv32(n, nf, owner, nb, diag, upper, lower, x, r);
    for (int32_t c = 0; c < n; ++c) r[c] = b[c] - r[c];
    spmv32_scaled(n, nf, owner, nb, diag, upper, lower, r, m, w);
    double gamma_prev = 0.0, alpha_prev = 0.0;
    int32_t status = OR_NOT_CONVERGED, i;
    for (i = 0;; ++i) {
        for (int32_t c = 0; c < n; ++c) u[c] = r[c] / diag[c];
        double gamma = dot32(n, r, u);
        double delta = dot32(n, w, u);
        double rho = dot32(n, r, r);
        if (sqrt(rho) <= tol * bnorm) { status = OR_OK; break; }
        if (i == maxit) break;
        for (int32_t c = 0; c < n; ++c) m[c] = w[c] / diag[c];
        spmv32(n, nf, owner, nb, diag, upper, lower, m, nv);
        double beta, den;
        if (i == 0) { beta = 0.0; den = delta; }
        else { beta = gamma / gamma_prev; den = delta - beta * gamma / alpha_prev; }
        double alpha = gamma / den;
        if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta)) { status = OR_BREAKDOWN; break; }
        float a32 = (float)alpha, b32 = (float)beta;
        for (int32_t c = 0; c < n; ++c) {
            z[c] = nv[c] + b32 * z[c];
            s[c] = w[c] + b32 * s[c];
            p[c] = u[c] + b32 * p[c];
            x[c] += a32 * p[c];
            r[c] -= a32 * s[c];
            w[c] -= a32 * z[c];
        }
        gamma_prev = gamma;
        alpha_prev = alpha;
    }
    *iters = i;
    free(r); free(u); free(w); free(m); free(nv); free(z); free(s); free(p);
    return status;
}

/* ---- Mixed-precision iterative refinement (an extension beside the
 * paper's FP64 solver, as the workload list states it).  Outer loop in FP64
 * with the FP64 matrix:
 *   r = b - A x; stop when ||r|| <= outer_tol ||b|| (OK), at max_outer
 *   (NOT_CONVERGED) or on a non-finite ||r|| (BREAKDOWN);
 *   solve A32 c = fp32(r / ||r||) by the FP32 folded pipelined Jacobi-CG to
 *   inner_tol (its recursive residual) or max_inner, from c = 0;
 *   x += ||r|| * c. */
int32_t or_refine(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                  const double* diag, const double* upper, const double* lower,
                  const double* b, double* x, double outer_tol, double inner_tol,
                  int32_t max_outer, int32_t max_inner, or_stats* st)
{
    if (st) memset(st, 0, sizeof(*st));
    double bnorm = sqrt(or_dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        return OR_OK;
    }
    if (!diag_positive(n, diag)) {
        if (st) st->status = OR_BREAKDOWN;
        return OR_BREAKDOWN;
    }
    float* d32 = malloc(sizeof(float) * (size_t)n);
    float* u32 = malloc(sizeof(float) * (size_t)(nf > 0 ? nf : 1));
    float* l32 = malloc(sizeof(float) * (size_t)(nf > 0 ? nf : 1));
    float* rhs = malloc(sizeof(float) * (size_t)n);
    float* cor = malloc(sizeof(float) * (size_t)n);
    double* r = alloc_vec(n);
    for (int32_t c = 0; c < n; ++c) d32[c] = (float)diag[c];
    for (int32_t f = 0; f < nf; ++f) { u32[f] = (float)upper[f]; l32[f] = (float)lower[f]; }

    int32_t status = OR_NOT_CONVERGED, j, total_inner = 0;
    double rnorm = 0.0;
    for (j = 0;; ++j) {
        residual(n, nf, owner, nb, diag, upper, lower, b, x, r);
        rnorm = sqrt(or_dot(n, r, r));
        if (j == 0 && st) st->r0_norm = rnorm;
        if (rnorm <= outer_tol * bnorm) { status = OR_OK; break; }
        if (!isfinite(rnorm)) { status = OR_BREAKDOWN; break; }
        if (j == max_outer) break;
        for (int32_t c = 0; c < n; ++c) { rhs[c] = (float)(r[c] / rnorm); cor[c] = 0.0f; }
        int32_t it = 0;
        int32_t s = pipecg32_folded(n, nf, owner, nb, d32, u32, l32, rhs, cor, inner_tol, max_inner, &it);
        total_inner += it;
        if (s == OR_BREAKDOWN && it == 0) { status = OR_BREAKDOWN; break; }
        for (int32_t c = 0; c < n; ++c) x[c] += rnorm * (double)cor[c];
    }
    if (st) {
        st->outer_iters = j;
        st->iters = total_inner;
        st->status = status;
        st->b_norm = bnorm;
        st->rel_res = rnorm / bnorm;
        st->true_rel_res = rnorm / bnorm;
    }
    free(d32); free(u32); free(l32); free(rhs); free(cor); free(r);
    return status;
}

/* ---- Mixed precision with reliable updates (an extension beside the
 * paper's FP64 solver; the residual-replacement idea of van der Vorst and
 * Ye, applied to the pipelined recurrences as by Cools et al.).  One FP32
 * folded pipelined Jacobi-CG iteration runs on the FP32-rounded matrix for
 * the scaled system A c = (b - A x0) / s, s = ||b - A x0||, with FP64
 * inner-product accumulation; its Krylov recurrences are never restarted.
 * Every `update_every` iterations (and at maxit) the FP64 side takes over:
 *   x += s * c, c = 0                         (solution accumulation, FP64)
 *   r64 = b - A x with the FP64 matrix        (outer residual, FP64)
 *   stop if ||r64|| <= tol ||b||, at maxit, or once ||r64|| has had no
 *   new minimum for max(OR_RU_STAGNATION, 10 update_every) iterations
 *   (NOT_CONVERGED; CG residual norms are not monotone, so the window is
 *   long);
 *   r = fp32(r64 / s), then s_ = A32 p, w = A32 D^-1 r, z = A32 D^-1 s_
 *   re-formed from their definitions (p is kept), and the next step's
 *   alpha, beta from the new dots and the previous gamma, alpha.
 * A breakdown of the FP32 recurrences (p'Ap <= 0 or a non-finite scalar)
 * also triggers an update, after which the recurrences restart from the
 * replaced residual (p = s = z = 0); a breakdown in the first iteration after
 * a restart ends the solve with BREAKDOWN.  st->iters counts FP32
 * iterations, st->outer_iters FP64 updates. */
enum { OR_RU_STAGNATION = 500 };

int32_t or_mixed_reliable(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                          const double* diag, const double* upper, const double* lower,
                          const double* b, double* x, double tol, int32_t update_every,
                          int32_t maxit, or_stats* st)
{
    if (st) memset(st, 0, sizeof(*st));
    double bnorm = sqrt(or_dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        return OR_OK;
    }
    if (!diag_positive(n, diag)) {
        if (st) st->status = OR_BREAKDOWN;
        return OR_BREAKDOWN;
    }
    if (update_every < 1) update_every = 1;
    double* r64 = alloc_vec(n);
    residual(n, nf, owner, nb, diag, upper, lower, b, x, r64);
    double rnorm = sqrt(or_dot(n, r64, r64));
    const double scale = rnorm;
    if (st) { st->r0_norm = rnorm; st->b_norm = bnorm; }
    int32_t status = OR_NOT_CONVERGED, it = 0, updates = 0;
    if (rnorm <= tol * bnorm) {
        free(r64);
        if (st) { st->status = OR_OK; st->rel_res = st->true_rel_res = rnorm / bnorm; }
        return OR_OK;
    }
    float* d32 = malloc(sizeof(float) * (size_t)n);
    float* u32 = malloc(sizeof(float) * (size_t)(nf > 0 ? nf : 1));
    float* l32 = malloc(sizeof(float) * (size_t)(nf > 0 ? nf : 1));
    for (int32_t c = 0; c < n; ++c) d32[c] = (float)diag[c];
    for (int32_t f = 0; f < nf; ++f) { u32[f] = (float)upper[f]; l32[f] = (float)lower[f]; }
    float *r = calloc((size_t)n, 4), *u = calloc((size_t)n, 4), *w = calloc((size_t)n, 4);
    float *m = calloc((size_t)n, 4), *nv = calloc((size_t)n, 4), *z = calloc((size_t)n, 4);
    float *s = calloc((size_t)n, 4), *p = calloc((size_t)n, 4), *cc = calloc((size_t)n, 4);

    for (int32_t c = 0; c < n; ++c) r[c] = (float)(r64[c] / scale);
    spmv32_scaled(n, nf, owner, nb, d32, u32, l32, r, m, w);
    double gamma_prev = 0.0, alpha_prev = 0.0, best = rnorm;
    int32_t first = 1, since = 0, it_best = 0;
    const int32_t window = OR_RU_STAGNATION > 10 * update_every ? OR_RU_STAGNATION : 10 * update_every;
    for (;;) {
        /* one FP32 pipelined iteration (Section 4.1 recurrences, folded Jacobi) */
        for (int32_t c = 0; c < n; ++c) u[c] = r[c] / d32[c];
        double gamma = dot32(n, r, u);
        double delta = dot32(n, w, u);
        double beta, den;
        if (first) { beta = 0.0; den = delta; }
        else { beta = gamma / gamma_prev; den = delta - beta * gamma / alpha_prev; }
        double alpha = gamma / den;
        int broke = !(den > 0.0) || !isfinite(alpha) || !isfinite(beta);
        if (broke && first) { status = OR_BREAKDOWN; break; }
        if (!broke) {
            for (int32_t c = 0; c < n; ++c) m[c] = w[c] / d32[c];
            spmv32(n, nf, owner, nb, d32, u32, l32, m, nv);
            float a32 = (float)alpha, b32 = (float)beta;
            for (int32_t c = 0; c < n; ++c) {
                z[c] = nv[c] + b32 * z[c];
                s[c] = w[c] + b32 * s[c];
                p[c] = u[c] + b32 * p[c];
                cc[c] += a32 * p[c];
                r[c] -= a32 * s[c];
                w[c] -= a32 * z[c];
            }
            gamma_prev = gamma;
            alpha_prev = alpha;
            first = 0;
            ++it;
            ++since;
        }
        if (!broke && since < update_every && it < maxit) continue;
        /* reliable update: FP64 accumulation and outer residual */
        since = 0;
        ++updates;
        for (int32_t c = 0; c < n; ++c) { x[c] += scale * (double)cc[c]; cc[c] = 0.0f; }
        residual(n, nf, owner, nb, diag, upper, lower, b, x, r64);
        rnorm = sqrt(or_dot(n, r64, r64));
        if (rnorm <= tol * bnorm) { status = OR_OK; break; }
        if (!isfinite(rnorm)) { status = OR_BREAKDOWN; break; }
        if (it >= maxit) break;
        if (rnorm < best) { best = rnorm; it_best = it; }
        else if (it - it_best >= window) break;
        for (int32_t c = 0; c < n; ++c) r[c] = (float)(r64[c] / scale);
        if (broke) {
            for (int32_t c = 0; c < n; ++c) { p[c] = 0.0f; s[c] = 0.0f; z[c] = 0.0f; }
            spmv32_scaled(n, nf, owner, nb, d32, u32, l32, r, m, w);
            first = 1;
        } else {
            spmv32(n, nf, owner, nb, d32, u32, l32, p, s);
            spmv32_scaled(n, nf, owner, nb, d32, u32, l32, r, m, w);
            spmv32_scaled(n, nf, owner, nb, d32, u32, l32, s, m, z);
        }
    }
    if (st) {
        st->iters = it;
        st->outer_iters = updates;
        st->status = status;
        st->rel_res = rnorm / bnorm;
        st->true_rel_res = rnorm / bnorm;
    }
    free(d32); free(u32); free(l32); free(r); free(u); free(w); free(m); free(nv); free(z); free(s); free(p);
    free(cc); free(r64);
    return status;
}

/* ---- Adjoint gradients on the sparsity pattern.  For L(x) with A x = b and
 * lambda = A^-T dL/dx: dL/db = lambda and dL/dA_ij = -lambda_i x_j, so the
 * diagonal gets -lambda_c x_c, upper[f] (row owner, column neighbour) gets
 * -lambda_owner x_neighbour and lower[f] gets -lambda_neighbour x_owner. */
void or_adjoint_grads(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                      const double* x, const double* lam,
                      double* g_diag, double* g_upper, double* g_lower)
{
    if (g_diag)
        for (int32_t c = 0; c < n; ++c) g_diag[c] = -lam[c] * x[c];
    for (int32_t f = 0; f < nf; ++f) {
        if (g_upper) g_upper[f] = -lam[owner[f]] * x[nb[f]];
        if (g_lower) g_lower[f] = -lam[nb[f]] * x[owner[f]];
    }
}
