// Transient diffusion (laplacianFoam, Section 2: the solver is called every
// time step): implicit-Euler assembly of dT/dt = div(k grad T) on the LDU
// addressing, and a run of time steps that assembles, refreshes the
// matrix's device layout and solves from the previous field each step.
//   upper_f = lower_f = -k_f w_f
//   diag_c  = V_c / dt + bdiag_c + sum over the cell's faces of k_f w_f
//   b_c     = (V_c / dt) T_c + bsrc_c
// The cell sums are gathers through the mesh's slot -> face map (one thread
// per cell, the faces in column order), so no atomics and a fixed order.
#include <algorithm>
#include <climits>

#include "handles.hpp"
#include "rows.hpp"

namespace fvpcg {

int matrix_update(fvpcg_matrix* A, const double* diag, const double* upper, const double* lower, hipStream_t s);
int solve(const fvpcg_matrix* A, const double* b, double* x, double tol, int maxit, int method, int precond,
          hipStream_t s, fvpcg_stats* stats);

namespace {

__global__ void k_assemble_faces(const double* __restrict__ k, const double* __restrict__ w, int F,
                                 double* __restrict__ upper) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) upper[f] = -(k[f] * w[f]);
}

__global__ void k_assemble_cells(const int* __restrict__ ref, int n, int W, const double* __restrict__ k,
                                 const double* __restrict__ w, const double* __restrict__ vol,
                                 const double* __restrict__ bdiag, const double* __restrict__ bsrc, double dt,
                                 const double* __restrict__ T_old, double* __restrict__ diag, double* __restrict__ b) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double vd = vol[c] / dt;
        double s = vd + bdiag[c];
        for (int q = 0; q < W; ++q) {
            const int e = ref[(size_t)q * n + c];
            if (e >= 0) {
                const int f = e >> 1;
                s += k[f] * w[f];
            }
        }
        diag[c] = s;
        b[c] = vd * T_old[c] + bsrc[c];
    }
}

int grid_of(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 65536)); }

}  // namespace

int assemble_transient(const fvpcg_mesh* m, const double* k, const double* w, const double* vol, const double* bdiag,
                       const double* bsrc, double dt, const double* T_old, double* diag, double* upper, double* b,
                       hipStream_t s) {
    if (m->F > 0) hipLaunchKernelGGL(k_assemble_faces, dim3(grid_of(m->F)), dim3(256), 0, s, k, w, m->F, upper);
    hipLaunchKernelGGL(k_assemble_cells, dim3(grid_of(m->n)), dim3(256), 0, s, m->ref, m->n, m->W, k, w, vol, bdiag,
                       bsrc, dt, T_old, diag, b);
    FV_LAUNCHED();
    return FVPCG_OK;
}

// nsteps implicit-Euler steps on A's mesh; T holds the field (in/out).
// Stats: iters = CG iterations over all steps, outer_iters = steps done,
// device_ms = the whole run, status of the last solve.
int transient_run(fvpcg_matrix* A, const double* k, const double* w, const double* vol, const double* bdiag,
                  const double* bsrc, double dt, int nsteps, double* T, double tol, int maxit, int method,
                  hipStream_t s, fvpcg_stats* stats) {
    const fvpcg_mesh* m = A->mesh;
    double *diag = nullptr, *upper = nullptr, *b = nullptr;
    int rc;
    auto done = [&](int code) {
        dev_free(diag);
        dev_free(upper);
        dev_free(b);
        return code;
    };
    if ((rc = dev_alloc(&diag, (size_t)std::max(m->n, 1), "transient diagonal")) ||
        (rc = dev_alloc(&upper, (size_t)std::max(m->F, 1), "transient faces")) ||
        (rc = dev_alloc(&b, (size_t)std::max(m->n, 1), "transient right-hand side")))
        return done(rc);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return done(set_error(FVPCG_DEVICE_ERROR, "event creation failed"));
    }
    (void)hipEventRecord(e0, s);
    long long its = 0;
    int status = FVPCG_OK, step = 0;
    fvpcg_stats st{};
    for (step = 0; step < nsteps; ++step) {
        if ((rc = assemble_transient(m, k, w, vol, bdiag, bsrc, dt, T, diag, upper, b, s))) break;
        if ((rc = matrix_update(A, diag, upper, nullptr, s))) break;
        status = solve(A, b, T, tol, maxit, method, FVPCG_PRECOND_JACOBI, s, &st);
        its += st.iters;
        if (status != FVPCG_OK) {
            ++step;
            break;
        }
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        *stats = st;
        stats->iters = (int32_t)std::min<long long>(its, INT32_MAX);
        stats->outer_iters = step;
        stats->status = rc ? rc : status;
        stats->device_ms = ms;
    }
    if (rc) return done(rc);
    return done(status);
}

}  // namespace fvpcg
