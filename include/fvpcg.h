/*
 * fvpcg -- preconditioned conjugate-gradient solves of finite-volume
 * Laplacian systems in LDU form on one AMD Instinct MI355X (gfx950).
 *
 * The method is the one of AlOnazi, Keyes, Lastovetsky and Rychkov
 * (arXiv 1505.07630): conjugate gradients on A x = b with A the symmetric
 * positive (semi)definite matrix of an OpenFOAM finite-volume discretisation
 * (Section 2), in the standard form with three inner products per iteration
 * and in the pipelined form of Ghysels and Vanroose with a single reduction
 * per iteration (Section 4.1), preconditioned by Jacobi or not at all.
 *
 * MATRIX FORMAT.  OpenFOAM's lduMatrix (named in the Section 5 discussion of
 * the CUDA/OpenFOAM interface; nnz = n + 2F as in Section 4.2):
 *   n_cells cells, n_faces internal faces;
 *   owner[f] < neighbour[f], faces sorted strictly by (owner, neighbour);
 *   diag[c]  = A[c][c];
 *   upper[f] = A[owner[f]][neighbour[f]];
 *   lower[f] = A[neighbour[f]][owner[f]].
 * Boundary conditions are folded into diag and b by the caller.
 *
 * MEMORY.  Every array argument is a DEVICE pointer (hipMalloc'd or a
 * contiguous torch tensor on the same device), owned by the caller.  The
 * library never frees caller memory and keeps no pointer to it after a call
 * returns: mesh and matrix data are copied into buffers owned by the handles,
 * which *_destroy frees.  Arrays: int32 addressing, FP64 coefficients and
 * vectors, all contiguous.
 *
 * STREAMS.  `stream` is a hipStream_t (NULL = the null stream).  All device
 * work is enqueued on it.  Calls that return statistics block the host until
 * their work on that stream is complete; a solve reads its convergence flag
 * back at chunk boundaries.  One call in flight per handle; distinct handles
 * may be used concurrently on distinct streams.
 *
 * ERRORS.  Every entry point returns an fvpcg_status.  fvpcg_last_error()
 * returns a human-readable, thread-local description of the last failure.
 * No exception crosses the interface.
 */
#ifndef FVPCG_H
#define FVPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FVPCG_VERSION 10000 /* 1.0.0 */

#ifndef FVPCG_API
#define FVPCG_API __attribute__((visibility("default")))
#endif

typedef enum fvpcg_status {
    FVPCG_OK = 0,
    FVPCG_NOT_CONVERGED = 1,  /* maxit reached; x = last iterate; stats valid */
    FVPCG_INVALID_ARG = -1,   /* null pointer, n < 1, tol < 0, b aliases x, tol = maxit = 0, ... */
    FVPCG_INVALID_MESH = -2,  /* addressing out of range, not owner < neighbour, not strictly sorted */
    FVPCG_BREAKDOWN = -3,     /* p'Ap <= 0, a non-finite scalar, or diag <= 0 under Jacobi */
    FVPCG_DEVICE_ERROR = -4,  /* a HIP call failed; the HIP message is in fvpcg_last_error() */
    FVPCG_OUT_OF_MEMORY = -5, /* a device or pinned allocation failed */
    FVPCG_UNSUPPORTED = -6    /* row degree > FVPCG_MAX_ROW_DEGREE, sizes beyond int32 slots, ... */
} fvpcg_status;

/* Krylov variants (Section 2: standard CG; Section 4.1: pipelined CG). */
enum {
    FVPCG_CG = 0,             /* standard form: three inner products, two reductions per iteration */
    FVPCG_PIPECG = 1,         /* pipelined form, one fused kernel and one reduction per iteration;
                                 with Jacobi, u = r/d, q = s/d, m = w/d are evaluated, not carried */
    FVPCG_PIPECG_LITERAL = 2  /* pipelined form carrying the u and q recurrences */
};

/* Preconditioner M ("optional" in Section 2). */
enum { FVPCG_PRECOND_NONE = 0, FVPCG_PRECOND_JACOBI = 1 };
/* pressure solver of fvpcg_piso_create: Jacobi-PCG, or PCG with the
 * smoothed-aggregation AMG cycle (hierarchy built once per time step) */
enum { FVPCG_PSOLVER_JACOBI = 0, FVPCG_PSOLVER_AMG = 1 };

/* fvpcg_matrix_create flags */
#define FVPCG_FP32_COPY 1u /* also keep an FP32 copy for the mixed-precision solves */

#define FVPCG_MAX_ROW_DEGREE 32
/* Largest system fvpcg_solve_noalloc takes (its work space is fixed). */
#define FVPCG_NOALLOC_MAX_CELLS 1048576

typedef struct fvpcg_mesh fvpcg_mesh;
typedef struct fvpcg_matrix fvpcg_matrix;
typedef struct fvpcg_batch fvpcg_batch;
typedef struct fvpcg_amg fvpcg_amg;
typedef struct fvpcg_piso fvpcg_piso;

typedef struct fvpcg_stats {
    int32_t iters;        /* updates of x (inner iterations summed for the mixed solver) */
    int32_t outer_iters;  /* refinement steps (mixed solver), else 0 */
    int32_t status;       /* the fvpcg_status of the solve */
    int32_t reserved;
    double rel_res;       /* recursive residual norm / ||b||_2 at exit */
    double true_rel_res;  /* ||b - A x||_2 / ||b||_2 recomputed at exit */
    double r0_norm;       /* ||b - A x0||_2 */
    double b_norm;        /* ||b||_2 */
    double device_ms;     /* whole call, HIP events on `stream` */
    double iter_ms;       /* the iteration kernels only, HIP events on `stream` */
} fvpcg_stats;

FVPCG_API int fvpcg_version(void);
FVPCG_API const char* fvpcg_last_error(void);

/* ---- Mesh: validates the addressing (0 <= owner < neighbour < n, faces
 * strictly sorted by (owner, neighbour)) and builds the device layout used by
 * every kernel (a slot-major ELL pattern with one slot per off-diagonal
 * entry of a row, columns ascending).  owner/neighbour: int32[n_faces]
 * device arrays; copied.  n_faces may be 0. */
FVPCG_API int fvpcg_mesh_create(int32_t n_cells, int32_t n_faces, const int32_t* owner,
                      const int32_t* neighbour, void* stream, fvpcg_mesh** out);
FVPCG_API int fvpcg_mesh_destroy(fvpcg_mesh* mesh);
/* ell_width = largest number of off-diagonal entries in a row. */
FVPCG_API int fvpcg_mesh_info(const fvpcg_mesh* mesh, int32_t* n_cells, int32_t* n_faces, int32_t* ell_width);

/* ---- Matrix: coefficients on a mesh (the mesh must outlive the matrix).
 * diag: FP64[n_cells]; upper, lower: FP64[n_faces]; lower == NULL means
 * lower = upper (symmetric).  Values are copied into the handle.
 * flags: FVPCG_FP32_COPY keeps an FP32 copy for the mixed-precision solver.
 * fvpcg_matrix_update refreshes the coefficients on the same pattern (the
 * repeated-solve use of Section 4.1, where the application calls the solver
 * again every time step). */
FVPCG_API int fvpcg_matrix_create(const fvpcg_mesh* mesh, const double* diag, const double* upper,
                        const double* lower, uint32_t flags, void* stream, fvpcg_matrix** out);
FVPCG_API int fvpcg_matrix_update(fvpcg_matrix* mat, const double* diag, const double* upper,
                        const double* lower, void* stream);
FVPCG_API int fvpcg_matrix_destroy(fvpcg_matrix* mat);

/* ---- y = A v in LDU semantics (the sparse matrix-vector product of
 * Section 2 / Table ai_cg).  v, y: FP64[n_cells], must not alias.
 * Asynchronous on `stream`. */
FVPCG_API int fvpcg_spmv(const fvpcg_matrix* mat, const double* v, double* y, void* stream);

/* ---- Solve A x = b by preconditioned CG (Section 2) or pipelined CG
 * (Section 4.1).  x: FP64[n_cells], holds x0 on entry and the solution on
 * exit.  b: FP64[n_cells], must not alias x.
 * Stops when the recursively updated residual satisfies
 * ||r||_2 <= tol * ||b||_2, or after maxit updates of x (status
 * FVPCG_NOT_CONVERGED).  tol = 0 with maxit > 0 runs exactly maxit
 * iterations unless the residual vanishes.  b = 0 gives x = 0.
 * method: FVPCG_CG / FVPCG_PIPECG / FVPCG_PIPECG_LITERAL;
 * precond: FVPCG_PRECOND_NONE / FVPCG_PRECOND_JACOBI.
 * stats may be NULL.  On FVPCG_BREAKDOWN x holds the last finite iterate. */
FVPCG_API int fvpcg_solve(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit,
                int32_t method, int32_t precond, void* stream, fvpcg_stats* stats);

/* ---- BiCGSTAB for non-symmetric matrices (lower != upper), the solver of
 * icoFoam's momentum equation (Section 2; the paper does not print it):
 * van der Vorst's Bi-CGSTAB with the preconditioner (precond:
 * FVPCG_PRECOND_NONE / FVPCG_PRECOND_JACOBI) applied to the search
 * directions, so r is the residual of A x = b, and shadow residual
 * rhat = r0.  Stops when ||r|| <= tol ||b|| (OK; also when ||s|| does after
 * the first half of an iteration, with x += alpha M^-1 p), after maxit
 * iterations (NOT_CONVERGED), or when (rhat, r), (rhat, A M^-1 p) or omega
 * is zero or not finite (BREAKDOWN).  Works on matrices created with or
 * without lower.  x holds x0 on entry (FP64[n_cells], device); b likewise;
 * they must not overlap.  The first call on a matrix allocates its
 * workspace (5 vectors of n doubles), freed by fvpcg_matrix_destroy.
 * Stats: iters = iterations that formed alpha, rel_res = ||r||/||b||,
 * true_rel_res = ||b - A x||/||b||. */
FVPCG_API int fvpcg_solve_bicgstab(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit,
                                   int32_t precond, void* stream, fvpcg_stats* stats);

/* ---- BiCGSTAB for nrhs = 1..4 right-hand sides with the same matrix (the
 * velocity components of a momentum predictor, Section 2), solved together:
 * each iteration reads the matrix once for all of them.  b and x hold the
 * components one after another (FP64[nrhs][n_cells], device; x = x0 on
 * entry); stats, if not NULL, points to nrhs structs.  Each component has
 * its own scalars and stopping test, as in fvpcg_solve_bicgstab; one that
 * has stopped is left untouched while the others go on.  Returns FVPCG_OK if
 * every component converged, else FVPCG_BREAKDOWN if any broke down, else
 * FVPCG_NOT_CONVERGED; device_ms and iter_ms are those of the whole call.
 * The workspace grows to 5 nrhs vectors of n doubles. */
FVPCG_API int fvpcg_solve_bicgstab_multi(const fvpcg_matrix* mat, int32_t nrhs, const double* b, double* x,
                                         double tol, int32_t maxit, int32_t precond, void* stream,
                                         fvpcg_stats* stats);

/* ---- Mixed-precision iterative refinement (FP32 inner, FP64 outer).
 * Outer: r = b - A x in FP64 with the FP64 matrix, stop at
 * ||r|| <= outer_tol ||b|| or after max_outer corrections.  Inner: the
 * FP32 copy solves A c = r/||r|| by folded pipelined Jacobi-CG in FP32 with
 * FP64 inner-product accumulation to inner_tol (at most max_inner
 * iterations), from c = 0; then x += ||r|| c in FP64.  Needs a matrix
 * created with FVPCG_FP32_COPY (else FVPCG_UNSUPPORTED). */
FVPCG_API int fvpcg_solve_mixed(const fvpcg_matrix* mat, const double* b, double* x, double outer_tol,
                      double inner_tol, int32_t max_outer, int32_t max_inner, void* stream,
                      fvpcg_stats* stats);

/* ---- Mixed precision with reliable updates (needs FVPCG_FP32_COPY; Jacobi).
 * The FP32 folded pipelined Jacobi-CG recurrences (Section 4.1) run on the
 * FP32-rounded matrix for A c = (b - A x0)/s, s = ||b - A x0||, with FP64
 * inner-product accumulation, and are never restarted.  Every update_every
 * FP32 iterations the FP64 side accumulates x += s c (c = 0), recomputes
 * r = b - A x with the FP64 matrix and re-forms the FP32 r = r/s, s = A p,
 * w = A D^-1 r, z = A D^-1 s (residual replacement).  Stops when
 * ||b - A x|| <= tol ||b|| (OK), after maxit FP32 iterations or once the FP64
 * residual has not reached a new minimum for max(500, 10 update_every)
 * iterations (NOT_CONVERGED), or on a breakdown of the FP32 recurrences right
 * after a restart from the replaced residual (BREAKDOWN); any other FP32
 * breakdown restarts them.  x holds x0 on entry (FP64[n_cells]).  Stats:
 * iters = FP32 iterations, outer_iters = FP64 updates, true_rel_res = the
 * last FP64 residual.  update_every >= 1, maxit >= 1. */
FVPCG_API int fvpcg_solve_mixed_reliable(const fvpcg_matrix* mat, const double* b, double* x, double tol,
                                         int32_t update_every, int32_t maxit, void* stream, fvpcg_stats* stats);

/* ---- Adjoint of a solve, for a scalar loss L(x) with A x = b.  Given the
 * solution x and g = dL/dx, solves A^T lambda = g (A is symmetric for CG,
 * so this is one more solve with A, same method and precond) and writes
 *   grad_b[c]     = lambda[c]
 *   grad_diag[c]  = -lambda[c] * x[c]
 *   grad_upper[f] = -lambda[owner[f]] * x[neighbour[f]]
 *   grad_lower[f] = -lambda[neighbour[f]] * x[owner[f]].
 * Any grad pointer may be NULL to skip it.  If the matrix was created with
 * lower == NULL (one coefficient per face), grad_upper receives the sum of
 * the upper and lower gradients and grad_lower is not written.
 * x, g: FP64[n_cells]; grad_diag, grad_b: FP64[n_cells]; grad_upper,
 * grad_lower: FP64[n_faces]. */
FVPCG_API int fvpcg_solve_backward(const fvpcg_matrix* mat, const double* x, const double* g, double* grad_b,
                         double* grad_diag, double* grad_upper, double* grad_lower, double tol,
                         int32_t maxit, int32_t method, int32_t precond, void* stream,
                         fvpcg_stats* stats);

/* ---- Batched solves: nsys independent systems of uneven sizes in one
 * persistent launch.  cell_off_host, face_off_host: HOST int32[nsys+1]
 * prefix offsets into the concatenated device arrays; owner/neighbour hold
 * LOCAL cell indices of each system (LDU rules per system).  lower == NULL
 * means symmetric.  Data are copied into the handle. */
FVPCG_API int fvpcg_batch_create(int32_t nsys, const int32_t* cell_off_host, const int32_t* face_off_host,
                       const int32_t* owner, const int32_t* neighbour, const double* diag,
                       const double* upper, const double* lower, uint32_t flags, void* stream,
                       fvpcg_batch** out);
FVPCG_API int fvpcg_batch_destroy(fvpcg_batch* batch);
/* b, x: concatenated FP64[total cells]; stats: HOST array of nsys entries
 * (may be NULL).  Returns FVPCG_OK if every system converged, else the
 * first non-OK status in system order.  Systems far larger than a
 * workgroup's share of the batch may be solved by a team of workgroups that
 * synchronise through device memory.  A launch with teams uses exactly the
 * device's resident workgroup capacity, so kernels running at the same time
 * on other streams can delay members; each wait is bounded
 * (FVPCG_BATCH_BARRIER_TIMEOUT_MS, default 5000): on a timeout every
 * workgroup leaves, x and stats are invalid and FVPCG_DEVICE_ERROR is
 * returned.  The first call per batch shape times the launch candidates
 * (block size, workgroups per CU, teams on/off) and caches the choice in
 * $FVPCG_TUNE_CACHE (FVPCG_TUNE=0: fixed defaults; FVPCG_BATCH_TEAMS=0/1:
 * never/always form teams).  Calls on one batch handle must not overlap. */
FVPCG_API int fvpcg_solve_batched(const fvpcg_batch* batch, const double* b, double* x, double tol,
                        int32_t maxit, int32_t method, int32_t precond, void* stream,
                        fvpcg_stats* stats);
/* Adjoint of fvpcg_solve_batched, per system as fvpcg_solve_backward, on
 * the concatenated arrays (face-indexed gradients use the face offsets). */
FVPCG_API int fvpcg_solve_batched_backward(const fvpcg_batch* batch, const double* x, const double* g,
                                 double* grad_b, double* grad_diag, double* grad_upper,
                                 double* grad_lower, double tol, int32_t maxit, int32_t method,
                                 int32_t precond, void* stream, fvpcg_stats* stats);

/* ---- Transient diffusion, laplacianFoam's heat equation dT/dt = div(k grad T)
 * (Section 2: the linear solver is called every time step), implicit Euler
 * on the LDU addressing:
 *   upper[f] = -k_face[f] w_face[f]            (w = |S_f| / |d_f|)
 *   diag[c]  = vol[c] / dt + bdiag[c] + sum over the faces of c of k w
 *   b[c]     = vol[c] / dt * T_old[c] + bsrc[c]
 * (bdiag, bsrc: Dirichlet and source terms per cell).  All arrays are device
 * FP64: k_face, w_face, upper [n_faces]; vol, bdiag, bsrc, T_old, diag, b
 * [n_cells]; outputs must not overlap inputs. */
FVPCG_API int fvpcg_assemble_transient(const fvpcg_mesh* mesh, const double* k_face, const double* w_face,
                                       const double* vol, const double* bdiag, const double* bsrc, double dt,
                                       const double* T_old, double* diag, double* upper, double* b,
                                       void* stream);
/* nsteps time steps on mat's mesh (mat created with lower == NULL; its
 * coefficients are replaced every step): assemble, refresh the device layout
 * (as fvpcg_matrix_update), solve with Jacobi and `method` from the previous
 * field to tol.  T: the field, in/out.  Stats: iters = CG iterations over all
 * steps, outer_iters = steps done, device_ms = the whole run; returns the
 * status of the last solve (the run stops at the first non-OK one). */
FVPCG_API int fvpcg_transient_run(fvpcg_matrix* mat, const double* k_face, const double* w_face, const double* vol,
                                  const double* bdiag, const double* bsrc, double dt, int32_t nsteps, double* T,
                                  double tol, int32_t maxit, int32_t method, void* stream, fvpcg_stats* stats);

/* ---- icoFoam's PISO step (Section 2: icoFoam solves its momentum equation
 * with BiCGSTAB and its pressure equation with CG, then corrects the velocity
 * explicitly; Section 4.1: the application calls the solver every step), on
 * the mesh of a box of cubes of side h, all on the device:
 *   momentum, implicit Euler with upwind convection of the face flux phi
 *   (owner -> neighbour): upper_f = -nu h - max(-phi_f, 0), lower_f =
 *   -nu h - max(phi_f, 0), diag_c = h^3/dt + bwall_c + sum over c's faces of
 *   (nu h + outflow_f if > 0); H source bH = (h^3/dt) U + blid (x only);
 *   predictor A U_k = bH_k - h^3 (grad p)_k for the three components
 *   together (BiCGSTAB, Jacobi, from the old U to tol_u);
 *   n_corr correctors: rAU = h^3 / diag, HbyA_k = (bH_k - offdiag(A) U_k) / diag,
 *   phiHbyA_f = face_sgn h^2 (HbyA_o + HbyA_n)/2 along the face's axis,
 *   c_f = h (rAU_o + rAU_n) / 2, pressure sum_f c_f (p_c - p_other) =
 *   -div(phiHbyA)_c with cell 0 pinned at p = 0 (its couplings zero in both
 *   triangles), solved by CG from the previous p to tol_p;
 *   phi_f = phiHbyA_f - c_f (p_n - p_o); U_k = HbyA_k - rAU (grad p)_k.
 * (grad p)_kc = (1/h)(bgrad_kc p_c + sum over c's faces along k of the
 * outward normal sign times (p_o + p_n)/2) (zero-gradient walls).
 * Inputs (device, copied at creation): face_dir int8[F] (0/1/2: the face's
 * axis), face_sgn int8[F] (+1 if the neighbour lies on the + side of the
 * owner along that axis, else -1), bwall FP64[n] (2 nu h per no-slip face,
 * lid included), blid FP64[n] (2 nu h u_lid per lid face), bgrad FP64[3][n]
 * (sum of the outward normal signs of the cell's boundary faces per axis).
 * The mesh must outlive the handle; calls on one handle must not overlap. */
FVPCG_API int fvpcg_piso_create(const fvpcg_mesh* mesh, const int8_t* face_dir, const int8_t* face_sgn,
                                const double* bwall, const double* blid, const double* bgrad, double h, double nu,
                                int32_t pressure_solver, void* stream, fvpcg_piso** out);
FVPCG_API int fvpcg_piso_destroy(fvpcg_piso* piso);
/* nsteps steps of size dt; U FP64[3][n] (x, y, z), p FP64[n] and phi FP64[F]
 * are device arrays updated in place (p[0] must be 0).  stats[0]: momentum
 * (iters = BiCGSTAB iterations over all components and steps, outer_iters =
 * steps done, device_ms = the whole run), stats[1]: pressure (iters summed,
 * outer_iters = pressure solves); stats may be NULL.  Returns the first
 * non-OK solver status (NOT_CONVERGED, BREAKDOWN) or an error code. */
FVPCG_API int fvpcg_piso_run(fvpcg_piso* piso, double dt, int32_t nsteps, int32_t n_corr, double* U, double* p,
                             double* phi, double tol_u, double tol_p, int32_t maxit, void* stream,
                             fvpcg_stats* stats);

/* ---- For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): fvpcg_solve with the same arguments,
 * kernels and results, whose work buffers (solver vectors, reduction
 * partials, device state) live in a fixed array in device memory that each
 * GPU holds from the library's load to the end of the process (64 MiB, for
 * at most FVPCG_NOALLOC_MAX_CELLS cells; larger systems: FVPCG_INVALID_ARG).
 * It calls no hipMalloc, hipFree, pinned-memory or event routine: the
 * convergence state is read into host stack memory and waited for after each
 * chunk of iterations, and stats->device_ms / iter_ms come from the host
 * clock.  The matrix (created beforehand) must live on the current device.
 * Every call on one GPU shares that array and keeps the last call's contents:
 * calls that overlap on one GPU (other threads, other streams) race. */
FVPCG_API int fvpcg_solve_noalloc(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit,
                                  int32_t method, int32_t precond, void* stream, fvpcg_stats* stats);

/* ---- Smoothed-aggregation AMG preconditioner (Section 5, discussion of
 * Fig. pcgs1 and Table pcgs2: a V-cycle of aggregation-based AMG whose
 * aggregates come from the parallel distance-2 maximal-independent-set
 * method, weighted Jacobi with omega = 4/3 as smoother).  The method:
 * strength j ~ i iff a_ij != 0 and |a_ij| >= theta_l sqrt(|a_ii a_jj|),
 * theta_l = theta / 2^l (theta = 0: every coupling); roots = a distance-2
 * maximal independent set of the strength graph in the order of SplitMix64
 * priorities drawn from (seed, level, unknown); each root's neighbours join
 * its aggregate, the rest the aggregate of their strongest such neighbour;
 * P = (I - omega D^-1 A) P_t, omega = (4/3) / (Gershgorin bound of D^-1 A);
 * A_c = P^T A P; levels until n <= coarse_size, max_levels, or an
 * aggregation keeping > 60% of the unknowns; the last level (at most 2048
 * unknowns) solved exactly.  Cycle V(1,1) with damped Jacobi (the same
 * omega).  The whole hierarchy is built on the device from the matrix's
 * current coefficients (sync on `stream` at exit).  The matrix must outlive
 * the handle and be symmetric (FVPCG_UNSUPPORTED otherwise); once the
 * matrix is updated, the handle's solves return FVPCG_INVALID_ARG until
 * fvpcg_amg_refresh (or a new handle).  Calls on one handle must not overlap.  Typical: theta = 0.02
 * (measured best on the lognormal cube and the graded cavity; 0 takes 1.4x
 * and 3.2x their iterations), max_levels = 12, coarse_size = 64, seed = 1.  Errors: FVPCG_UNSUPPORTED if
 * the last level exceeds 2048 unknowns, FVPCG_BREAKDOWN if it is not
 * positive definite, FVPCG_OUT_OF_MEMORY. */
FVPCG_API int fvpcg_amg_create(const fvpcg_matrix* mat, double theta, int32_t max_levels, int32_t coarse_size,
                               uint64_t seed, void* stream, fvpcg_amg** out);
/* Repeated solves (Section 4.1: the application calls the solver every time
 * step with new coefficients on the same mesh): the hierarchy for the
 * matrix's current coefficients after fvpcg_matrix_update, keeping the
 * aggregates, the level count and every sparsity pattern of the setup and
 * recomputing the rest as fvpcg_amg_create does (diagonals, omega, P, R,
 * the coarse operators, the last level's inverse), with the product kernels
 * the setup chose and no independent-set rounds.  The result equals a fresh
 * setup whenever the aggregates would not change (for instance all
 * coefficients scaled by a power of two, which scales every level exactly);
 * otherwise it is the same method on the kept aggregates.  Sync on `stream` at exit.  The matrix must still be
 * symmetric (FVPCG_UNSUPPORTED); FVPCG_BREAKDOWN if a diagonal is not
 * positive or the last level is not positive definite, after which the
 * handle's solves return FVPCG_INVALID_ARG until a refresh succeeds. */
FVPCG_API int fvpcg_amg_refresh(fvpcg_amg* amg, void* stream);
FVPCG_API int fvpcg_amg_destroy(fvpcg_amg* amg);
/* Number of levels; rows and stored entries of `level` (n, nnz may be NULL). */
FVPCG_API int fvpcg_amg_info(const fvpcg_amg* amg, int32_t level, int32_t* levels, int32_t* n, int64_t* nnz);
/* Aggregate index of every row of `level` (a level with a coarser one) into a
 * HOST int32 array of that level's row count. */
FVPCG_API int fvpcg_amg_aggregates(const fvpcg_amg* amg, int32_t level, int32_t* host_out);
/* Level `level`'s operator (which = 0; levels >= 1: level 0's operator is
 * the matrix), prolongator P (1) or restriction R = P^T (2; levels with a
 * coarser one) as CSR copied into HOST arrays: host_ptr int32[rows + 1],
 * host_col int32[nnz], host_val FP64[nnz], columns ascending in each row.
 * Pass NULL arrays to get rows, cols and nnz only. */
FVPCG_API int fvpcg_amg_export(const fvpcg_amg* amg, int32_t level, int32_t which, int32_t* rows, int32_t* cols,
                               int64_t* nnz, int32_t* host_ptr, int32_t* host_col, double* host_val);
/* z = M^-1 r, one cycle; r, z: FP64[n_cells] device arrays, not overlapping. */
FVPCG_API int fvpcg_amg_apply(const fvpcg_amg* amg, const double* r, double* z, void* stream);
/* Preconditioned CG with M^-1 = one cycle: method FVPCG_CG (standard form,
 * Section 2) or FVPCG_PIPECG (pipelined form of Section 4.1 with the literal
 * recurrences u = M^-1 r, m = M^-1 w, q = M^-1 s; one cycle per iteration
 * applied to w).  Stopping and stats as fvpcg_solve (x holds x0). */
FVPCG_API int fvpcg_solve_amg(const fvpcg_amg* amg, const double* b, double* x, double tol, int32_t maxit,
                              int32_t method, void* stream, fvpcg_stats* stats);

/* ---- STREAM-style copy and triad over device arrays of `bytes_per_array`
 * bytes each (three arrays; 0 = 1 GiB), as the paper measures attainable
 * bandwidth for its roofline (Section 1).  Results in GB/s (1e9 B/s);
 * copy moves 2, triad 3 arrays per pass. */
FVPCG_API int fvpcg_stream_calibrate(void* stream, uint64_t bytes_per_array, double* copy_gbs, double* triad_gbs);
/* Attainable rate of a kernel that streams n_read device arrays in and
 * n_write out (1..16 and 0..8, each of `bytes_per_array` bytes; 0 = 256 MiB):
 * the roofline line for a kernel with that mix of reads and writes (Section
 * 1 draws the paper's from STREAM).  Best over two orders (every workgroup
 * over one contiguous chunk of each array; all workgroups sweeping the
 * arrays together in interleaved tiles, as the solver kernels read their
 * vectors and matrix slots) and five grid sizes, in GB/s of (n_read +
 * n_write) arrays per pass.  The arrays are allocated and freed inside the call.  INVALID_ARG
 * for counts out of range or arrays under 16 KiB. */
FVPCG_API int fvpcg_stream_mix(void* stream, uint64_t bytes_per_array, int32_t n_read, int32_t n_write, double* gbs);

#ifdef __cplusplus
}
#endif
#endif /* FVPCG_H */
