/*
 * CPU oracle for the finite-volume Laplacian CG solve -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, single-threaded FP64 C written from the paper's description of
 * the method, used only by the tests, the benchmark's CPU-baseline leg and the
 * smoke check to judge the HIP path.  It shares no code, header, table or
 * helper with the HIP library and must never be called by the product path.
 *
 * Matrix convention: OpenFOAM lduMatrix (diag[n], upper[F], lower[F],
 * owner[F] < neighbour[F]); row owner[f] holds upper[f] in column
 * neighbour[f], row neighbour[f] holds lower[f] in column owner[f]
 * (nnz = n + 2F, Section 4.2).
 */
#ifndef FV_ORACLE_H
#define FV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_BREAKDOWN = -3 };
enum { OR_PRECOND_NONE = 0, OR_PRECOND_JACOBI = 1 };

typedef struct or_stats {
    int32_t iters;
    int32_t outer_iters;
    int32_t status;
    int32_t reserved;
    double rel_res;       /* recursive residual norm / ||b|| at exit */
    double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit */
    double r0_norm;
    double b_norm;
} or_stats;

/* y = A v by the LDU definition: diagonal term, then a scatter over faces. */
void or_spmv(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
             const double* diag, const double* upper, const double* lower,
             const double* v, double* y);

/* Sum of a[i]*b[i], pairwise (halves summed recursively, blocks of <= 8
 * sequentially). */
double or_dot(int32_t n, const double* a, const double* b);

/* Preconditioned CG, standard form (three inner products per iteration,
 * Section 2).  x holds x0 on entry.  Optional histories (length >= maxit+1,
 * may be NULL): alpha[k], beta[k] of iteration k and the recursive residual
 * norm after k updates (res_hist[0] = ||r0||). */
int32_t or_cg(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
              const double* diag, const double* upper, const double* lower,
              const double* b, double* x, double tol, int32_t maxit, int32_t precond,
              or_stats* st, double* alpha_hist, double* beta_hist, double* res_hist);

/* Pipelined preconditioned CG of Ghysels and Vanroose, the variant the paper
 * implements (Section 4.1): one fused reduction per iteration.
 * folded = 0: literal recurrences for u, q (and m = M^-1 w).
 * folded = 1 (Jacobi only): u = r/d, q = s/d, m = w/d evaluated directly. */
int32_t or_pipecg(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                  const double* diag, const double* upper, const double* lower,
                  const double* b, double* x, double tol, int32_t maxit, int32_t precond,
                  int32_t folded, or_stats* st, double* res_hist);

/* Mixed-precision iterative refinement: FP64 outer residual with the FP64
 * matrix, FP32 inner folded pipelined Jacobi-CG on the FP32-rounded matrix
 * with FP64 inner-product accumulation, FP64 correction. */
int32_t or_refine(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                  const double* diag, const double* upper, const double* lower,
                  const double* b, double* x, double outer_tol, double inner_tol,
                  int32_t max_outer, int32_t max_inner, or_stats* st);

/* Mixed precision with reliable updates: FP32 folded pipelined Jacobi-CG
 * whose recurrences are never restarted, with the FP64 solution
 * accumulation, FP64 outer residual and residual replacement every
 * update_every iterations. */
int32_t or_mixed_reliable(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                          const double* diag, const double* upper, const double* lower,
                          const double* b, double* x, double tol, int32_t update_every,
                          int32_t maxit, or_stats* st);

/* ---- Smoothed-aggregation AMG preconditioner (amg.c; the method is stated
 * at the top of that file).  seed selects the aggregation priorities. */
enum { OR_AMG_MAX_LEVELS = 16, OR_AMG_MAX_COARSE = 2048 };
typedef struct or_amg or_amg;

/* NULL if the last level has more than OR_AMG_MAX_COARSE unknowns or is not
 * positive definite. */
or_amg* or_amg_setup(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                     const double* diag, const double* upper, const double* lower,
                     double theta, int32_t max_levels, int32_t coarse_size, uint64_t seed);
/* Distance-2 maximal-independent-set aggregation of one CSR level (columns
 * sorted in each row); key == NULL takes the priorities from (seed, level).
 * Returns the aggregate count (-1: an unknown left out). */
int32_t or_amg_aggregate(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double theta,
                         const uint64_t* key, uint64_t seed, int32_t level, int32_t* agg);
uint64_t or_splitmix64(uint64_t seed, uint64_t k);
uint64_t or_amg_priority(uint64_t seed, int32_t level, int32_t i);
/* New coefficients of the same mesh, the aggregates kept (0, or -1). */
int32_t or_amg_refresh(or_amg* h, int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                       const double* diag, const double* upper, const double* lower);
void or_amg_free(or_amg* h);
int32_t or_amg_levels(const or_amg* h);
void or_amg_level_info(const or_amg* h, int32_t l, int32_t* n, int32_t* nnz, int32_t* n_coarse, double* omega);
void or_amg_aggregates(const or_amg* h, int32_t l, int32_t* out);
/* Level l's A (which = 0) or P (which = 1) as CSR; returns nnz; NULL arrays
 * query the sizes only. */
int32_t or_amg_export(const or_amg* h, int32_t l, int32_t which, int32_t* rows, int32_t* cols, int32_t* ptr,
                      int32_t* col, double* val);
/* x = M^-1 b, one V(1,1) cycle. */
void or_amg_vcycle(const or_amg* h, const double* b, double* x);
/* Standard PCG with the V-cycle; x holds x0 on entry. */
int32_t or_amg_pcg(const or_amg* h, const double* b, double* x, double tol, int32_t maxit, or_stats* st);
/* Pipelined CG (literal recurrences) with the V-cycle; x holds x0 on entry. */
int32_t or_amg_pipecg(const or_amg* h, const double* b, double* x, double tol, int32_t maxit, or_stats* st);

/* ---- icoFoam's PISO step (piso.c; the method is stated at the top of that
 * file).  Fields: U [3][n] (x, y, z components), p [n], phi [F]. */
void or_piso_momentum(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const double* phi,
                      const double* bwall, const double* blid, double h, double nu, double dt, const double* U_old,
                      double* diag, double* upper, double* lower, double* bH);
void or_piso_gradp(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                   const int8_t* face_sgn, const double* bgrad, double h, const double* p, double* g);
void or_piso_div(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const double* phi, double* div);
void or_piso_pressure_system(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                             const int8_t* face_sgn, double h, const double* diag, const double* upper,
                             const double* lower, const double* bH, const double* U, double* HbyA, double* rAU,
                             double* phiHbyA, double* cf, double* pdiag, double* pupper, double* prhs);
/* nsteps PISO steps (momentum predictor by BiCGSTAB to tol_u, n_corr
 * pressure correctors by CG to tol_p), U, p and phi updated in place. */
int32_t or_piso_run(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb, const int8_t* face_dir,
                    const int8_t* face_sgn, const double* bwall, const double* blid, const double* bgrad, double h,
                    double nu, double dt, int32_t nsteps, int32_t n_corr, double* U, double* p, double* phi,
                    double tol_u, double tol_p, int32_t maxit, int32_t* iters_u, int32_t* iters_p);

/* ---- Transient diffusion (transient.c): implicit-Euler LDU assembly of
 * laplacianFoam's heat equation and a run of nsteps steps (each solved by
 * Jacobi-PCG from the previous field; T in/out). */
void or_assemble_transient(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                           const double* k, const double* w, const double* vol, const double* bdiag,
                           const double* bsrc, double dt, const double* T_old,
                           double* diag, double* upper, double* b);
int32_t or_transient_run(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                         const double* k, const double* w, const double* vol, const double* bdiag,
                         const double* bsrc, double dt, int32_t nsteps, double* T, double tol, int32_t maxit,
                         int32_t* total_iters);

/* ---- BiCGSTAB (bicgstab.c), van der Vorst's form with M = I or Jacobi
 * applied to the search directions, for matrices with lower != upper
 * (Section 2: icoFoam's momentum solve).  x holds x0 on entry.  Optional
 * histories (length >= maxit+1, may be NULL): alpha[k], omega[k] of
 * iteration k (omega = 0 for a half-step exit) and ||r|| after k iterations
 * (res_hist[0] = ||r0||). */
int32_t or_bicgstab(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                    const double* diag, const double* upper, const double* lower,
                    const double* b, double* x, double tol, int32_t maxit, int32_t precond,
                    or_stats* st, double* alpha_hist, double* omega_hist, double* res_hist);

/* Gradients of a scalar loss L(x) with A x = b on the LDU pattern, given x
 * and lambda = A^-T dL/dx:  dL/ddiag = -lambda*x, dL/dupper[f] =
 * -lambda[owner]*x[nb], dL/dlower[f] = -lambda[nb]*x[owner]. */
void or_adjoint_grads(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                      const double* x, const double* lam,
                      double* g_diag, double* g_upper, double* g_lower);

#ifdef __cplusplus
}
#endif
#endif
