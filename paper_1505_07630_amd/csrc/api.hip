// The C ABI of libfvpcg.so (include/fvpcg.h): argument validation, error
// reporting and dispatch to the solvers.  No exception crosses it.
#include <cstring>
#include <new>

#include "handles.hpp"

namespace fvpcg {

// Implemented in setup.hip / solve.hip / batched.hip / calibrate.hip / amg.hip /
// transient.hip / bicgstab.hip.
int mesh_create(int32_t n, int32_t F, const int32_t* owner, const int32_t* nb, hipStream_t s, fvpcg_mesh** out);
int mesh_destroy(fvpcg_mesh* m);
int matrix_create(const fvpcg_mesh* m, const double* diag, const double* upper, const double* lower, uint32_t flags,
                  hipStream_t s, fvpcg_matrix** out);
int matrix_update(fvpcg_matrix* A, const double* diag, const double* upper, const double* lower, hipStream_t s);
int matrix_destroy(fvpcg_matrix* A);
int spmv(const fvpcg_matrix* A, const double* v, double* y, hipStream_t s);
int solve(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
          hipStream_t s, fvpcg_stats* stats);
int solve_mixed(const fvpcg_matrix* A, const double* b, double* x, double outer_tol, double inner_tol, int max_outer,
                int max_inner, hipStream_t s, fvpcg_stats* stats);
int solve_mixed_reliable(const fvpcg_matrix* A, const double* b, double* x, double tol, int update_every, int maxit,
                         hipStream_t s, fvpcg_stats* stats);
int solve_backward(const fvpcg_matrix* A, const double* x, const double* g, double* grad_b, double* grad_diag,
                   double* grad_upper, double* grad_lower, double tol, int maxit, int method, int precond,
                   hipStream_t s, fvpcg_stats* stats);
int batch_create(int32_t nsys, const int32_t* cell_off, const int32_t* face_off, const int32_t* owner,
                 const int32_t* nb, const double* diag, const double* upper, const double* lower, uint32_t flags,
                 hipStream_t s, fvpcg_batch** out);
int batch_destroy(fvpcg_batch* bt);
int batch_total_cells(const fvpcg_batch* bt);
int batch_total_faces(const fvpcg_batch* bt);
int batch_nsys(const fvpcg_batch* bt);
int solve_batched(const fvpcg_batch* bt, const double* b, double* x, double tol, int maxit, int method, int precond,
                  hipStream_t s, fvpcg_stats* stats);
int solve_batched_backward(const fvpcg_batch* bt, const double* x, const double* g, double* grad_b,
                           double* grad_diag, double* grad_upper, double* grad_lower, double tol, int maxit,
                           int method, int precond, hipStream_t s, fvpcg_stats* stats);
int stream_calibrate(hipStream_t s, uint64_t bytes, double* copy_gbs, double* triad_gbs);
int stream_mix(hipStream_t s, uint64_t bytes, int nr, int nw, double* gbs);
int solve_bicgstab(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int precond,
                   hipStream_t s, fvpcg_stats* stats);
int solve_bicgstab_multi(const fvpcg_matrix* A, int nrhs, const double* b, double* x, double tol, int maxit,
                         int precond, hipStream_t s, fvpcg_stats* stats);
void bicgstab_free(fvpcg_matrix* A);
int assemble_transient(const fvpcg_mesh* m, const double* k, const double* w, const double* vol, const double* bdiag,
                       const double* bsrc, double dt, const double* T_old, double* diag, double* upper, double* b,
                       hipStream_t s);
int transient_run(fvpcg_matrix* A, const double* k, const double* w, const double* vol, const double* bdiag,
                  const double* bsrc, double dt, int nsteps, double* T, double tol, int maxit, int method,
                  hipStream_t s, fvpcg_stats* stats);
bool batch_symmetric(const fvpcg_batch* bt);
int solve_noalloc(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
                  hipStream_t s, fvpcg_stats* stats);
int amg_create(const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, uint64_t seed, hipStream_t s,
               fvpcg_amg** out);
int piso_create(const fvpcg_mesh* m, const int8_t* face_dir, const int8_t* face_sgn, const double* bwall,
                const double* blid, const double* bgrad, double h, double nu, int psolver, hipStream_t s,
                fvpcg_piso** out);
void piso_free(fvpcg_piso* ps);
int piso_run(fvpcg_piso* ps, double dt, int nsteps, int n_corr, double* U, double* p, double* phi, double tol_u,
             double tol_p, int maxit, hipStream_t s, fvpcg_stats* stats);
int piso_mesh_n(const fvpcg_piso* ps);
int piso_mesh_f(const fvpcg_piso* ps);
void amg_free(fvpcg_amg* h);
int amg_update(fvpcg_amg* h, hipStream_t s);
int amg_levels(const fvpcg_amg* h);
int amg_level_n(const fvpcg_amg* h, int l);
long long amg_level_nnz(const fvpcg_amg* h, int l);
int amg_level_agg(const fvpcg_amg* h, int l, int* host_out, hipStream_t s);
int amg_export(const fvpcg_amg* h, int l, int which, int* rows, int* cols, long long* nnz, int* ptr, int* col,
               double* val, hipStream_t s);
int amg_apply(const fvpcg_amg* h, const double* r, double* z, hipStream_t s);
int solve_amg(const fvpcg_amg* h, const double* b, double* x, double tol, int maxit, int method, hipStream_t s,
              fvpcg_stats* stats);

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
    (void)hipGetLastError();
    const char* base = strrchr(file, '/');
    return set_error(e == hipErrorOutOfMemory ? FVPCG_OUT_OF_MEMORY : FVPCG_DEVICE_ERROR, "%s failed: %s (%s:%d)",
                     what, hipGetErrorString(e), base ? base + 1 : file, line);
}

// A caller array must be device-accessible memory covering `bytes` bytes.
int check_dev(const void* p, size_t bytes, const char* name) {
    if (!p) return set_error(FVPCG_INVALID_ARG, "%s is NULL", name);
    if (bytes == 0) return FVPCG_OK;
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FVPCG_INVALID_ARG, "%s is not a device pointer", name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return set_error(FVPCG_INVALID_ARG, "%s is not device memory", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e == hipSuccess && base) {
        const char* b = (const char*)base;
        const char* q = (const char*)p;
        if (q < b || (size_t)(q - b) + bytes > size)
            return set_error(FVPCG_INVALID_ARG, "%s: %zu bytes exceed its allocation", name, bytes);
    } else {
        (void)hipGetLastError();
    }
    return FVPCG_OK;
}

int check_opt(const void* p, size_t bytes, const char* name) { return p ? check_dev(p, bytes, name) : FVPCG_OK; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b) return false;
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

int check_solver_args(double tol, int maxit, int method, int precond) {
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(FVPCG_INVALID_ARG, "tol must be finite and >= 0");
    if (maxit < 0) return set_error(FVPCG_INVALID_ARG, "maxit must be >= 0");
    if (tol == 0.0 && maxit == 0) return set_error(FVPCG_INVALID_ARG, "tol = 0 and maxit = 0: nothing to do");
    if (method < FVPCG_CG || method > FVPCG_PIPECG_LITERAL) return set_error(FVPCG_INVALID_ARG, "unknown method %d", method);
    if (precond != FVPCG_PRECOND_NONE && precond != FVPCG_PRECOND_JACOBI)
        return set_error(FVPCG_INVALID_ARG, "unknown preconditioner %d", precond);
    return FVPCG_OK;
}

void stats_status(fvpcg_stats* st, int code) {
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->status = code;
    }
}

}  // namespace fvpcg

using namespace fvpcg;

template <typename F>
static int guard(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return set_error(FVPCG_DEVICE_ERROR, "unexpected internal exception");
    }
}

#define FV_TRY(expr)              \
    do {                          \
        int fv_rc_ = (expr);      \
        if (fv_rc_) return fv_rc_; \
    } while (0)

extern "C" {

int fvpcg_version(void) { return FVPCG_VERSION; }

const char* fvpcg_last_error(void) { return g_last_error.c_str(); }

int fvpcg_mesh_create(int32_t n_cells, int32_t n_faces, const int32_t* owner, const int32_t* neighbour, void* stream,
                      fvpcg_mesh** out) {
    return guard([&]() -> int {
        if (!out) return set_error(FVPCG_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (n_cells < 1) return set_error(FVPCG_INVALID_ARG, "n_cells must be >= 1");
        if (n_faces < 0 || n_faces >= (1 << 30)) return set_error(FVPCG_INVALID_ARG, "n_faces out of range");
        if (n_faces > 0) {
            FV_TRY(check_dev(owner, sizeof(int32_t) * (size_t)n_faces, "owner"));
            FV_TRY(check_dev(neighbour, sizeof(int32_t) * (size_t)n_faces, "neighbour"));
        }
        return mesh_create(n_cells, n_faces, owner, neighbour, (hipStream_t)stream, out);
    });
}

int fvpcg_mesh_destroy(fvpcg_mesh* mesh) {
    return guard([&]() -> int { return mesh ? mesh_destroy(mesh) : FVPCG_OK; });
}

int fvpcg_mesh_info(const fvpcg_mesh* mesh, int32_t* n_cells, int32_t* n_faces, int32_t* ell_width) {
    if (!mesh) return set_error(FVPCG_INVALID_ARG, "mesh is NULL");
    if (n_cells) *n_cells = mesh->n;
    if (n_faces) *n_faces = mesh->F;
    if (ell_width) *ell_width = mesh->maxdeg;
    return FVPCG_OK;
}

int fvpcg_matrix_create(const fvpcg_mesh* mesh, const double* diag, const double* upper, const double* lower,
                        uint32_t flags, void* stream, fvpcg_matrix** out) {
    return guard([&]() -> int {
        if (!out) return set_error(FVPCG_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!mesh) return set_error(FVPCG_INVALID_ARG, "mesh is NULL");
        if (flags & ~FVPCG_FP32_COPY) return set_error(FVPCG_INVALID_ARG, "unknown flags 0x%x", flags);
        FV_TRY(check_dev(diag, sizeof(double) * (size_t)mesh->n, "diag"));
        if (mesh->F > 0) {
            FV_TRY(check_dev(upper, sizeof(double) * (size_t)mesh->F, "upper"));
            FV_TRY(check_opt(lower, sizeof(double) * (size_t)mesh->F, "lower"));
        }
        return matrix_create(mesh, diag, upper, lower, flags, (hipStream_t)stream, out);
    });
}

int fvpcg_matrix_update(fvpcg_matrix* mat, const double* diag, const double* upper, const double* lower,
                        void* stream) {
    return guard([&]() -> int {
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        const fvpcg_mesh* m = mat->mesh;
        FV_TRY(check_dev(diag, sizeof(double) * (size_t)m->n, "diag"));
        if (m->F > 0) {
            FV_TRY(check_dev(upper, sizeof(double) * (size_t)m->F, "upper"));
            FV_TRY(check_opt(lower, sizeof(double) * (size_t)m->F, "lower"));
        }
        return matrix_update(mat, diag, upper, lower, (hipStream_t)stream);
    });
}

int fvpcg_matrix_destroy(fvpcg_matrix* mat) {
    return guard([&]() -> int {
        if (!mat) return FVPCG_OK;
        bicgstab_free(mat);
        return matrix_destroy(mat);
    });
}

int fvpcg_spmv(const fvpcg_matrix* mat, const double* v, double* y, void* stream) {
    return guard([&]() -> int {
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_dev(v, bytes, "v"));
        FV_TRY(check_dev(y, bytes, "y"));
        if (overlap(v, bytes, y, bytes)) return set_error(FVPCG_INVALID_ARG, "v and y overlap");
        return spmv(mat, v, y, (hipStream_t)stream);
    });
}

// CG, its pipelined form, the mixed solvers and the adjoint assume A = A^T;
// a matrix whose lower coefficients differ from its upper ones goes to
// BiCGSTAB instead.
static int require_symmetric(bool sym, fvpcg_stats* stats) {
    if (sym) return FVPCG_OK;
    stats_status(stats, FVPCG_UNSUPPORTED);
    return set_error(FVPCG_UNSUPPORTED,
                     "CG needs a symmetric matrix (lower == upper on every face); use BiCGSTAB for this one");
}

int fvpcg_solve(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit, int32_t method,
                int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_solver_args(tol, maxit, method, precond));
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        FV_TRY(require_symmetric(mat->vals_sym, stats));
        if (precond == FVPCG_PRECOND_JACOBI && !mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        int rc = solve(mat, b, x, tol, maxit, method, precond, (hipStream_t)stream, stats);
        if (rc == FVPCG_BREAKDOWN) set_error(rc, "breakdown: p'Ap <= 0 or a non-finite scalar");
        return rc;
    });
}

int fvpcg_solve_noalloc(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit,
                        int32_t method, int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_solver_args(tol, maxit, method, precond));
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        FV_TRY(require_symmetric(mat->vals_sym, stats));
        if (precond == FVPCG_PRECOND_JACOBI && !mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        int rc = solve_noalloc(mat, b, x, tol, maxit, method, precond, (hipStream_t)stream, stats);
        if (rc == FVPCG_BREAKDOWN) set_error(rc, "breakdown: p'Ap <= 0 or a non-finite scalar");
        return rc;
    });
}

int fvpcg_solve_bicgstab(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t maxit,
                         int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_solver_args(tol, maxit, FVPCG_CG, precond));
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        if (precond == FVPCG_PRECOND_JACOBI && !mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        int rc = solve_bicgstab(mat, b, x, tol, maxit, precond, (hipStream_t)stream, stats);
        if (rc == FVPCG_BREAKDOWN) set_error(rc, "breakdown: (rhat, r), (rhat, A p) or omega is zero or not finite");
        return rc;
    });
}

int fvpcg_solve_bicgstab_multi(const fvpcg_matrix* mat, int32_t nrhs, const double* b, double* x, double tol,
                               int32_t maxit, int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        if (stats && nrhs >= 1 && nrhs <= 4)
            for (int k = 0; k < nrhs; ++k) stats_status(&stats[k], FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        if (nrhs < 1 || nrhs > 4) return set_error(FVPCG_INVALID_ARG, "nrhs must be 1..4 (got %d)", nrhs);
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n * (size_t)nrhs;
        FV_TRY(check_solver_args(tol, maxit, FVPCG_CG, precond));
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        if (precond == FVPCG_PRECOND_JACOBI && !mat->diag_ok) {
            if (stats)
                for (int k = 0; k < nrhs; ++k) stats_status(&stats[k], FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        int rc = solve_bicgstab_multi(mat, nrhs, b, x, tol, maxit, precond, (hipStream_t)stream, stats);
        if (rc == FVPCG_BREAKDOWN)
            set_error(rc, "breakdown in a component: (rhat, r), (rhat, A p) or omega is zero or not finite");
        return rc;
    });
}

int fvpcg_solve_mixed(const fvpcg_matrix* mat, const double* b, double* x, double outer_tol, double inner_tol,
                      int32_t max_outer, int32_t max_inner, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        if (!mat->fp32) {
            stats_status(stats, FVPCG_UNSUPPORTED);
            return set_error(FVPCG_UNSUPPORTED, "matrix was created without FVPCG_FP32_COPY");
        }
        if (!(outer_tol >= 0.0) || !std::isfinite(outer_tol) || !(inner_tol > 0.0) || !(inner_tol < 1.0))
            return set_error(FVPCG_INVALID_ARG, "need outer_tol >= 0 and 0 < inner_tol < 1");
        if (max_outer < 0 || max_inner < 1) return set_error(FVPCG_INVALID_ARG, "need max_outer >= 0, max_inner >= 1");
        if (outer_tol == 0.0 && max_outer == 0) return set_error(FVPCG_INVALID_ARG, "outer_tol = max_outer = 0");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        FV_TRY(require_symmetric(mat->vals_sym, stats));
        if (!mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        return solve_mixed(mat, b, x, outer_tol, inner_tol, max_outer, max_inner, (hipStream_t)stream, stats);
    });
}

int fvpcg_solve_mixed_reliable(const fvpcg_matrix* mat, const double* b, double* x, double tol, int32_t update_every,
                               int32_t maxit, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        if (!mat->fp32) {
            stats_status(stats, FVPCG_UNSUPPORTED);
            return set_error(FVPCG_UNSUPPORTED, "matrix was created without FVPCG_FP32_COPY");
        }
        if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(FVPCG_INVALID_ARG, "need a finite tol >= 0");
        if (update_every < 1 || maxit < 1) return set_error(FVPCG_INVALID_ARG, "need update_every >= 1, maxit >= 1");
        size_t bytes = sizeof(double) * (size_t)mat->mesh->n;
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        FV_TRY(require_symmetric(mat->vals_sym, stats));
        if (!mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        return solve_mixed_reliable(mat, b, x, tol, update_every, maxit, (hipStream_t)stream, stats);
    });
}

int fvpcg_solve_backward(const fvpcg_matrix* mat, const double* x, const double* g, double* grad_b, double* grad_diag,
                         double* grad_upper, double* grad_lower, double tol, int32_t maxit, int32_t method,
                         int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        FV_TRY(check_solver_args(tol, maxit, method, precond));
        size_t nb = sizeof(double) * (size_t)mat->mesh->n;
        size_t fb = sizeof(double) * (size_t)mat->mesh->F;
        FV_TRY(check_dev(x, nb, "x"));
        FV_TRY(check_dev(g, nb, "g"));
        FV_TRY(check_opt(grad_b, nb, "grad_b"));
        FV_TRY(check_opt(grad_diag, nb, "grad_diag"));
        if (fb) {
            FV_TRY(check_opt(grad_upper, fb, "grad_upper"));
            FV_TRY(check_opt(grad_lower, fb, "grad_lower"));
        }
        const void* ins[] = {x, g};
        const size_t insz[] = {nb, nb};
        void* outs[] = {grad_b, grad_diag, grad_upper, grad_lower};
        const size_t outsz[] = {nb, nb, fb, fb};
        for (int i = 0; i < 4; ++i) {
            for (int k = 0; k < 2; ++k)
                if (overlap(outs[i], outsz[i], ins[k], insz[k]))
                    return set_error(FVPCG_INVALID_ARG, "gradient outputs must not overlap x or g");
            for (int k = i + 1; k < 4; ++k)
                if (overlap(outs[i], outsz[i], outs[k], outsz[k]))
                    return set_error(FVPCG_INVALID_ARG, "gradient outputs must not overlap each other");
        }
        FV_TRY(require_symmetric(mat->vals_sym, stats));
        if (precond == FVPCG_PRECOND_JACOBI && !mat->diag_ok) {
            stats_status(stats, FVPCG_BREAKDOWN);
            return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
        }
        return solve_backward(mat, x, g, grad_b, grad_diag, grad_upper, grad_lower, tol, maxit, method, precond,
                              (hipStream_t)stream, stats);
    });
}

int fvpcg_batch_create(int32_t nsys, const int32_t* cell_off_host, const int32_t* face_off_host, const int32_t* owner,
                       const int32_t* neighbour, const double* diag, const double* upper, const double* lower,
                       uint32_t flags, void* stream, fvpcg_batch** out) {
    return guard([&]() -> int {
        if (!out) return set_error(FVPCG_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (nsys < 1) return set_error(FVPCG_INVALID_ARG, "nsys must be >= 1");
        if (!cell_off_host || !face_off_host) return set_error(FVPCG_INVALID_ARG, "offsets are NULL");
        if (flags != 0) return set_error(FVPCG_INVALID_ARG, "unknown flags 0x%x", flags);
        if (cell_off_host[0] != 0 || face_off_host[0] != 0) return set_error(FVPCG_INVALID_ARG, "offsets must start at 0");
        for (int s = 0; s < nsys; ++s) {
            if (cell_off_host[s + 1] - cell_off_host[s] < 1)
                return set_error(FVPCG_INVALID_ARG, "system %d has no cells", s);
            if (face_off_host[s + 1] < face_off_host[s])
                return set_error(FVPCG_INVALID_ARG, "face offsets decrease at system %d", s);
        }
        size_t nc = (size_t)cell_off_host[nsys], nf = (size_t)face_off_host[nsys];
        FV_TRY(check_dev(diag, sizeof(double) * nc, "diag"));
        if (nf) {
            FV_TRY(check_dev(owner, sizeof(int32_t) * nf, "owner"));
            FV_TRY(check_dev(neighbour, sizeof(int32_t) * nf, "neighbour"));
            FV_TRY(check_dev(upper, sizeof(double) * nf, "upper"));
            FV_TRY(check_opt(lower, sizeof(double) * nf, "lower"));
        }
        return batch_create(nsys, cell_off_host, face_off_host, owner, neighbour, diag, upper, lower, flags,
                            (hipStream_t)stream, out);
    });
}

int fvpcg_batch_destroy(fvpcg_batch* batch) {
    return guard([&]() -> int { return batch ? batch_destroy(batch) : FVPCG_OK; });
}

int fvpcg_solve_batched(const fvpcg_batch* batch, const double* b, double* x, double tol, int32_t maxit,
                        int32_t method, int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        if (!batch) return set_error(FVPCG_INVALID_ARG, "batch is NULL");
        FV_TRY(check_solver_args(tol, maxit, method, precond));
        size_t bytes = sizeof(double) * (size_t)batch_total_cells(batch);
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        if (!batch_symmetric(batch))
            return set_error(FVPCG_UNSUPPORTED, "CG needs symmetric systems (lower == upper on every face)");
        return solve_batched(batch, b, x, tol, maxit, method, precond, (hipStream_t)stream, stats);
    });
}

int fvpcg_solve_batched_backward(const fvpcg_batch* batch, const double* x, const double* g, double* grad_b,
                                 double* grad_diag, double* grad_upper, double* grad_lower, double tol,
                                 int32_t maxit, int32_t method, int32_t precond, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        if (!batch) return set_error(FVPCG_INVALID_ARG, "batch is NULL");
        FV_TRY(check_solver_args(tol, maxit, method, precond));
        size_t nb = sizeof(double) * (size_t)batch_total_cells(batch);
        size_t fb = sizeof(double) * (size_t)batch_total_faces(batch);
        FV_TRY(check_dev(x, nb, "x"));
        FV_TRY(check_dev(g, nb, "g"));
        FV_TRY(check_opt(grad_b, nb, "grad_b"));
        FV_TRY(check_opt(grad_diag, nb, "grad_diag"));
        if (fb) {
            FV_TRY(check_opt(grad_upper, fb, "grad_upper"));
            FV_TRY(check_opt(grad_lower, fb, "grad_lower"));
        }
        const void* ins[] = {x, g};
        void* outs[] = {grad_b, grad_diag, grad_upper, grad_lower};
        const size_t outsz[] = {nb, nb, fb, fb};
        for (int i = 0; i < 4; ++i) {
            for (int k = 0; k < 2; ++k)
                if (overlap(outs[i], outsz[i], ins[k], nb))
                    return set_error(FVPCG_INVALID_ARG, "gradient outputs must not overlap x or g");
            for (int k = i + 1; k < 4; ++k)
                if (overlap(outs[i], outsz[i], outs[k], outsz[k]))
                    return set_error(FVPCG_INVALID_ARG, "gradient outputs must not overlap each other");
        }
        if (!batch_symmetric(batch))
            return set_error(FVPCG_UNSUPPORTED, "CG needs symmetric systems (lower == upper on every face)");
        return solve_batched_backward(batch, x, g, grad_b, grad_diag, grad_upper, grad_lower, tol, maxit, method,
                                      precond, (hipStream_t)stream, stats);
    });
}

int fvpcg_piso_create(const fvpcg_mesh* mesh, const int8_t* face_dir, const int8_t* face_sgn, const double* bwall,
                      const double* blid, const double* bgrad, double h, double nu, int32_t pressure_solver,
                      void* stream, fvpcg_piso** out) {
    return guard([&]() -> int {
        if (!out) return set_error(FVPCG_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!mesh) return set_error(FVPCG_INVALID_ARG, "mesh is NULL");
        if (!(h > 0.0) || !std::isfinite(h) || !(nu > 0.0) || !std::isfinite(nu))
            return set_error(FVPCG_INVALID_ARG, "need finite h > 0 and nu > 0");
        if (pressure_solver != FVPCG_PSOLVER_JACOBI && pressure_solver != FVPCG_PSOLVER_AMG)
            return set_error(FVPCG_INVALID_ARG, "unknown pressure solver %d", pressure_solver);
        const size_t n = (size_t)mesh->n, F = (size_t)mesh->F;
        if (F) {
            FV_TRY(check_dev(face_dir, F, "face_dir"));
            FV_TRY(check_dev(face_sgn, F, "face_sgn"));
        }
        FV_TRY(check_dev(bwall, sizeof(double) * n, "bwall"));
        FV_TRY(check_dev(blid, sizeof(double) * n, "blid"));
        FV_TRY(check_dev(bgrad, sizeof(double) * 3 * n, "bgrad"));
        return piso_create(mesh, face_dir, face_sgn, bwall, blid, bgrad, h, nu,
                           pressure_solver == FVPCG_PSOLVER_AMG ? FVPCG_PSOLVER_AMG : FVPCG_CG, (hipStream_t)stream,
                           out);
    });
}

int fvpcg_piso_destroy(fvpcg_piso* piso) {
    return guard([&]() -> int {
        piso_free(piso);
        return FVPCG_OK;
    });
}

int fvpcg_piso_run(fvpcg_piso* piso, double dt, int32_t nsteps, int32_t n_corr, double* U, double* p, double* phi,
                   double tol_u, double tol_p, int32_t maxit, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        if (stats) {
            stats_status(&stats[0], FVPCG_INVALID_ARG);
            stats_status(&stats[1], FVPCG_INVALID_ARG);
        }
        if (!piso) return set_error(FVPCG_INVALID_ARG, "piso is NULL");
        if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0 || n_corr < 1 || maxit < 1)
            return set_error(FVPCG_INVALID_ARG, "need dt > 0, nsteps >= 0, n_corr >= 1, maxit >= 1");
        if (!(tol_u > 0.0) || !(tol_p > 0.0) || !std::isfinite(tol_u) || !std::isfinite(tol_p))
            return set_error(FVPCG_INVALID_ARG, "need finite tol_u > 0 and tol_p > 0");
        const size_t n = (size_t)piso_mesh_n(piso), F = (size_t)piso_mesh_f(piso);
        FV_TRY(check_dev(U, sizeof(double) * 3 * n, "U"));
        FV_TRY(check_dev(p, sizeof(double) * n, "p"));
        if (F) FV_TRY(check_dev(phi, sizeof(double) * F, "phi"));
        if (overlap(U, sizeof(double) * 3 * n, p, sizeof(double) * n) ||
            (F && (overlap(U, sizeof(double) * 3 * n, phi, sizeof(double) * F) ||
                   overlap(p, sizeof(double) * n, phi, sizeof(double) * F))))
            return set_error(FVPCG_INVALID_ARG, "U, p and phi must not overlap");
        return piso_run(piso, dt, nsteps, n_corr, U, p, phi, tol_u, tol_p, maxit, (hipStream_t)stream, stats);
    });
}

int fvpcg_amg_create(const fvpcg_matrix* mat, double theta, int32_t max_levels, int32_t coarse_size, uint64_t seed,
                     void* stream, fvpcg_amg** out) {
    return guard([&]() -> int {
        if (!out) return set_error(FVPCG_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        if (!(theta >= 0.0) || !std::isfinite(theta) || max_levels < 1 || coarse_size < 1)
            return set_error(FVPCG_INVALID_ARG, "need theta >= 0, max_levels >= 1, coarse_size >= 1");
        if (!mat->diag_ok) return set_error(FVPCG_BREAKDOWN, "AMG needs a finite positive diagonal");
        if (!mat->vals_sym)
            return set_error(FVPCG_UNSUPPORTED, "AMG needs a symmetric matrix (lower == upper on every face)");
        return amg_create(mat, theta, max_levels, coarse_size, seed, (hipStream_t)stream, out);
    });
}

int fvpcg_amg_refresh(fvpcg_amg* amg, void* stream) {
    return guard([&]() -> int {
        if (!amg) return set_error(FVPCG_INVALID_ARG, "amg is NULL");
        return amg_update(amg, (hipStream_t)stream);
    });
}

int fvpcg_amg_destroy(fvpcg_amg* amg) {
    return guard([&]() -> int {
        amg_free(amg);
        return FVPCG_OK;
    });
}

int fvpcg_amg_info(const fvpcg_amg* amg, int32_t level, int32_t* levels, int32_t* n, int64_t* nnz) {
    return guard([&]() -> int {
        if (!amg) return set_error(FVPCG_INVALID_ARG, "amg is NULL");
        if (levels) *levels = amg_levels(amg);
        if (level < 0 || level >= amg_levels(amg)) {
            if (n || nnz) return set_error(FVPCG_INVALID_ARG, "level %d outside [0, %d)", level, amg_levels(amg));
            return FVPCG_OK;
        }
        if (n) *n = amg_level_n(amg, level);
        if (nnz) *nnz = amg_level_nnz(amg, level);
        return FVPCG_OK;
    });
}

int fvpcg_amg_aggregates(const fvpcg_amg* amg, int32_t level, int32_t* host_out) {
    return guard([&]() -> int {
        if (!amg || !host_out) return set_error(FVPCG_INVALID_ARG, "amg or host_out is NULL");
        if (level < 0 || level + 1 >= amg_levels(amg))
            return set_error(FVPCG_INVALID_ARG, "level %d has no coarser level", level);
        return amg_level_agg(amg, level, host_out, nullptr);
    });
}

int fvpcg_amg_export(const fvpcg_amg* amg, int32_t level, int32_t which, int32_t* rows, int32_t* cols,
                     int64_t* nnz, int32_t* host_ptr, int32_t* host_col, double* host_val) {
    return guard([&]() -> int {
        if (!amg || !rows || !cols || !nnz) return set_error(FVPCG_INVALID_ARG, "amg, rows, cols or nnz is NULL");
        if (level < 0 || level >= amg_levels(amg))
            return set_error(FVPCG_INVALID_ARG, "level %d outside [0, %d)", level, amg_levels(amg));
        long long z = 0;
        int rc = amg_export(amg, level, which, rows, cols, &z, host_ptr, host_col, host_val, nullptr);
        *nnz = z;
        return rc;
    });
}

int fvpcg_amg_apply(const fvpcg_amg* amg, const double* r, double* z, void* stream) {
    return guard([&]() -> int {
        if (!amg) return set_error(FVPCG_INVALID_ARG, "amg is NULL");
        const size_t bytes = sizeof(double) * (size_t)amg_level_n(amg, 0);
        FV_TRY(check_dev(r, bytes, "r"));
        FV_TRY(check_dev(z, bytes, "z"));
        if (overlap(r, bytes, z, bytes)) return set_error(FVPCG_INVALID_ARG, "r and z overlap");
        return amg_apply(amg, r, z, (hipStream_t)stream);
    });
}

int fvpcg_solve_amg(const fvpcg_amg* amg, const double* b, double* x, double tol, int32_t maxit, int32_t method,
                    void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!amg) return set_error(FVPCG_INVALID_ARG, "amg is NULL");
        if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return set_error(FVPCG_INVALID_ARG, "need tol >= 0, maxit >= 0");
        if (tol == 0.0 && maxit == 0) return set_error(FVPCG_INVALID_ARG, "tol = maxit = 0");
        if (method != FVPCG_CG && method != FVPCG_PIPECG)
            return set_error(FVPCG_INVALID_ARG, "method must be FVPCG_CG or FVPCG_PIPECG");
        const size_t bytes = sizeof(double) * (size_t)amg_level_n(amg, 0);
        FV_TRY(check_dev(b, bytes, "b"));
        FV_TRY(check_dev(x, bytes, "x"));
        if (overlap(b, bytes, x, bytes)) return set_error(FVPCG_INVALID_ARG, "b and x overlap");
        return solve_amg(amg, b, x, tol, maxit, method, (hipStream_t)stream, stats);
    });
}

int fvpcg_assemble_transient(const fvpcg_mesh* mesh, const double* k_face, const double* w_face, const double* vol,
                             const double* bdiag, const double* bsrc, double dt, const double* T_old, double* diag,
                             double* upper, double* b, void* stream) {
    return guard([&]() -> int {
        if (!mesh) return set_error(FVPCG_INVALID_ARG, "mesh is NULL");
        if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(FVPCG_INVALID_ARG, "need a finite dt > 0");
        const size_t nb = sizeof(double) * (size_t)mesh->n, fb = sizeof(double) * (size_t)mesh->F;
        FV_TRY(check_dev(vol, nb, "vol"));
        FV_TRY(check_dev(bdiag, nb, "bdiag"));
        FV_TRY(check_dev(bsrc, nb, "bsrc"));
        FV_TRY(check_dev(T_old, nb, "T_old"));
        FV_TRY(check_dev(diag, nb, "diag"));
        FV_TRY(check_dev(b, nb, "b"));
        if (fb) {
            FV_TRY(check_dev(k_face, fb, "k_face"));
            FV_TRY(check_dev(w_face, fb, "w_face"));
            FV_TRY(check_dev(upper, fb, "upper"));
        }
        const void* outs[] = {diag, b};
        const size_t outsz[] = {nb, nb};
        const void* ins[] = {vol, bdiag, bsrc, T_old, k_face, w_face};
        const size_t insz[] = {nb, nb, nb, nb, fb, fb};
        for (int o = 0; o < 2; ++o)
            for (int i = 0; i < 6; ++i)
                if (insz[i] && overlap(outs[o], outsz[o], ins[i], insz[i]))
                    return set_error(FVPCG_INVALID_ARG, "an output overlaps an input");
        if (fb)
            for (int i = 0; i < 6; ++i)
                if (insz[i] && overlap(upper, fb, ins[i], insz[i]))
                    return set_error(FVPCG_INVALID_ARG, "an output overlaps an input");
        return assemble_transient(mesh, k_face, w_face, vol, bdiag, bsrc, dt, T_old, diag, upper, b,
                                  (hipStream_t)stream);
    });
}

int fvpcg_transient_run(fvpcg_matrix* mat, const double* k_face, const double* w_face, const double* vol,
                        const double* bdiag, const double* bsrc, double dt, int32_t nsteps, double* T, double tol,
                        int32_t maxit, int32_t method, void* stream, fvpcg_stats* stats) {
    return guard([&]() -> int {
        stats_status(stats, FVPCG_INVALID_ARG);
        if (!mat) return set_error(FVPCG_INVALID_ARG, "mat is NULL");
        if (!mat->sym) return set_error(FVPCG_INVALID_ARG, "the matrix must have been created with lower == NULL");
        if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0) return set_error(FVPCG_INVALID_ARG, "need dt > 0, nsteps >= 0");
        FV_TRY(check_solver_args(tol, maxit, method, FVPCG_PRECOND_JACOBI));
        const fvpcg_mesh* m = mat->mesh;
        const size_t nb = sizeof(double) * (size_t)m->n, fb = sizeof(double) * (size_t)m->F;
        FV_TRY(check_dev(vol, nb, "vol"));
        FV_TRY(check_dev(bdiag, nb, "bdiag"));
        FV_TRY(check_dev(bsrc, nb, "bsrc"));
        FV_TRY(check_dev(T, nb, "T"));
        if (fb) {
            FV_TRY(check_dev(k_face, fb, "k_face"));
            FV_TRY(check_dev(w_face, fb, "w_face"));
        }
        const void* ins[] = {vol, bdiag, bsrc, k_face, w_face};
        const size_t insz[] = {nb, nb, nb, fb, fb};
        for (int i = 0; i < 5; ++i)
            if (insz[i] && overlap(T, nb, ins[i], insz[i])) return set_error(FVPCG_INVALID_ARG, "T overlaps an input");
        return transient_run(mat, k_face, w_face, vol, bdiag, bsrc, dt, nsteps, T, tol, maxit, method,
                             (hipStream_t)stream, stats);
    });
}

int fvpcg_stream_calibrate(void* stream, uint64_t bytes_per_array, double* copy_gbs, double* triad_gbs) {
    return guard([&]() -> int {
        if (!copy_gbs || !triad_gbs) return set_error(FVPCG_INVALID_ARG, "result pointers are NULL");
        return stream_calibrate((hipStream_t)stream, bytes_per_array, copy_gbs, triad_gbs);
    });
}

int fvpcg_stream_mix(void* stream, uint64_t bytes_per_array, int32_t n_read, int32_t n_write, double* gbs) {
    return guard([&]() -> int {
        if (!gbs) return set_error(FVPCG_INVALID_ARG, "result pointer is NULL");
        return stream_mix((hipStream_t)stream, bytes_per_array, n_read, n_write, gbs);
    });
}

}  // extern "C"
