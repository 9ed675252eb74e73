// Batched solves: many independent LDU systems of uneven sizes in one
// persistent launch, captured in a hipGraph.
//
// The systems are stored as one block-diagonal matrix (their addressing
// offset by each system's first cell), so the ELL layout, validation and
// coefficient handling are the single-system ones.  A system is solved from
// start to finish either by one workgroup (its rows, reductions and scalars
// stay inside the workgroup; no waiting on anyone) or, when it costs at least
// a workgroup's fair share of the batch, by a team of workgroups that
// split its row tiles and combine their reductions through device memory and
// a bounded team barrier.  Teams are assigned statically at launch; the other
// systems go to a device queue ordered by decreasing size (largest first, the
// list-scheduling rule that keeps the tail short), which team members join
// once their system is done.  Block size, workgroups per CU and teams on/off
// are chosen per batch by a small autotuner that times the candidates on the
// batch itself and caches the choice in a JSON file.
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <numeric>
#include <sstream>
#include <vector>

#include "handles.hpp"

namespace fvpcg {
int mesh_create(int32_t n, int32_t F, const int32_t* owner, const int32_t* nb, hipStream_t s, fvpcg_mesh** out);
int mesh_destroy(fvpcg_mesh* m);
int matrix_create(const fvpcg_mesh* m, const double* diag, const double* upper, const double* lower, uint32_t flags,
                  hipStream_t s, fvpcg_matrix** out);
int matrix_destroy(fvpcg_matrix* A);
int adjoint_grads(const fvpcg_matrix* A, const double* x, const double* lam, double* grad_b, double* grad_diag,
                  double* grad_upper, double* grad_lower, hipStream_t s);

struct BatchStat {
    int32_t iters;
    int32_t status;
    double bnorm;
    double r0norm;
    double rho;
    double true_rr;
};

struct BatchArgs {
    const void* col;  // int32 columns or int16 offsets (the kernel's CI)
    const double* val;     // plain values (residuals, standard CG, unpreconditioned)
    const double* val_cs;  // column-scaled values (Jacobi-folded pipelined)
    const double* d;
    const int* cell_off;
    const int* order;  // queued systems, largest first
    int nsys;          // queue length
    int n;  // total cells (slot stride)
    const double* b;
    double* x;
    double *r, *p, *q, *z, *s, *w0, *w1;
    double tol;
    int maxit;
    unsigned* queue;
    BatchStat* stats;
    // workgroup teams for systems larger than a workgroup's fair share
    const int4* tasks;            // [grid] (system, rank, team size, partials offset); system -1: none
    unsigned long long* arrive;   // [nsys] team barrier counters, zeroed per launch
    double* team_part;            // team partial sums, [2][size][3] per team system
    int* abort_flag;              // set when a team barrier times out; every workgroup then exits
    unsigned long long spin_ticks;  // team barrier timeout, wall-clock ticks
};

struct Tuning {
    int block = 256;
    int per_cu = 4;
    int teams = 0;
};

}  // namespace fvpcg

struct fvpcg_batch {
    int nsys = 0;
    int ncells = 0;
    int nfaces = 0;
    std::vector<int> cell_off, face_off;
    fvpcg_mesh* mesh = nullptr;
    fvpcg_matrix* mat = nullptr;
    int* d_cell_off = nullptr;
    int* d_order = nullptr;
    unsigned* d_queue = nullptr;
    fvpcg::BatchStat* d_stats = nullptr;
    fvpcg::BatchStat* h_stats = nullptr;  // pinned
    double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *s = nullptr, *w0 = nullptr, *w1 = nullptr;
    double* xscratch = nullptr;
    double* lam = nullptr;
    hipStream_t capture = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::map<std::string, fvpcg::Tuning> tuned;
    // teams: per-launch work table, barrier counters, partials, abort flag
    int pmax = 0;
    int4* d_tasks = nullptr;
    unsigned long long* d_arrive = nullptr;
    double* d_team_part = nullptr;
    int* d_abort = nullptr;
    int4* h_tasks = nullptr;   // pinned staging
    int* h_order = nullptr;    // pinned staging
    int* h_abort = nullptr;    // pinned
    unsigned long long spin_ticks = 0;
    // cached graph
    hipGraphExec_t gexec = nullptr;
    std::string gkey;
    // which work table the device holds now
    int plan_grid = -1, plan_block = 0, plan_teams = 0, plan_queue = 0;
};

namespace fvpcg {

namespace {

// Sum NV values over a workgroup of BS threads; every thread gets the totals.
template <int BS, int NV>
__device__ __forceinline__ void block_allreduce(double (&v)[NV]) {
    constexpr int NW = BS / 64;
    __shared__ double lds[NV][NW];
    __shared__ double out[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += lds[k][w];
            out[k] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = out[k];
    __syncthreads();
}

__device__ __forceinline__ int slot_col(const int* p, size_t o, int) { return p[o]; }
__device__ __forceinline__ int slot_col(const int16_t* p, size_t o, int c) { return c + (int)p[o]; }

template <int WT, typename CI>
__device__ __forceinline__ double gather(const void* colv, const double* __restrict__ val, int n, int c,
                                         const double* __restrict__ v, double acc) {
    const CI* __restrict__ col = (const CI*)colv;
    int j[WT];
    double a[WT];
#pragma unroll
    for (int k = 0; k < WT; ++k) {
        const size_t o = (size_t)k * n + c;
        j[k] = slot_col(col, o, c);
        a[k] = val[o];
    }
#pragma unroll
    for (int k = 0; k < WT; ++k) acc += a[k] * v[j[k]];
    return acc;
}

// A team: the workgroups that solve one system together (size 1 = one
// workgroup, no cross-workgroup synchronisation at all).
struct Team {
    int rank, size;
    unsigned long long* arrive;
    double* part;
    int* abort_flag;
    unsigned long long ticks;
    int nbar;  // barriers passed so far
    int par;   // which half of the double-buffered partials
};

// Barrier among the team's workgroups: a monotonic arrival counter (barrier k
// completes when it reaches k * size).  The workgroup's threads meet at a
// workgroup barrier; thread 0 then arrives with an agent-scope release,
// polls the counter with relaxed loads and ends with one agent-scope acquire
// fence before the closing workgroup barrier.  Under the HSA memory model
// (HRF-indirect, inclusive scopes) happens-before is transitive through the
// workgroup barriers and thread 0's agent-scope synchronisation, so every
// member sees the other members' vector writes; a fence per thread would
// only repeat the L2 write-back and invalidate once per wave.  The wait is
// bounded: past the timeout (or when another workgroup has timed out) the
// abort flag is set and false returned, and every workgroup leaves.
__device__ bool team_barrier(Team& t) {
    t.nbar += 1;
    if (t.size == 1) {
        __syncthreads();
        return true;
    }
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long target = (unsigned long long)t.nbar * (unsigned long long)t.size;
        __hip_atomic_fetch_add(t.arrive, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        const unsigned long long t0 = (unsigned long long)wall_clock64();
        while (__hip_atomic_load(t.arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(t.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            if ((unsigned long long)wall_clock64() - t0 > t.ticks) {
                __hip_atomic_store(t.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Sum NV values over the team: workgroup totals, then (size > 1) each member
// publishes its totals, waits at the barrier and adds all members' totals in
// rank order, so every member holds identical sums.
template <int BS, int NV>
__device__ bool team_allreduce(double (&v)[NV], Team& t) {
    block_allreduce<BS, NV>(v);
    if (t.size == 1) return true;
    double* mine = t.part + ((size_t)t.par * t.size + t.rank) * 3;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) mine[k] = v[k];
    }
    const bool ok = team_barrier(t);
    double tot[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    for (int r = 0; r < t.size; ++r) {
        const double* q = t.part + ((size_t)t.par * t.size + r) * 3;
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] += q[k];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = tot[k];
    t.par ^= 1;
    return ok;
}

// Rows of system [c0, c1) handled by this team member: tiles of BS rows,
// member r takes tiles r, r + size, ...  (size 1: every row, in order).
#define TEAM_ROWS(c)                                                             \
    for (int t_ = tm.rank; c0 + t_ * BS < c1; t_ += tm.size)                     \
        for (int c = c0 + t_ * BS + (int)threadIdx.x; c < c1 && c < c0 + (t_ + 1) * BS; c += BS)

// Scalar state of one system, identical in every thread of its workgroup.
struct Sys {
    double gamma = 0, alpha = 0, beta = 0, bnorm = 0, tol_abs = 0, r0norm = 0, rho = 0;
    int iter = 0, status = FVPCG_NOT_CONVERGED;
    bool done = false;
};

// The pipelined recurrences' scalar step (see the single-system solver).
__device__ __forceinline__ void pipe_step(Sys& y, double gamma, double delta, double rho, bool first, int maxit) {
    if (!first) y.iter += 1;
    y.rho = rho;
    if (sqrt(rho) <= y.tol_abs) {
        y.done = true;
        y.status = FVPCG_OK;
        return;
    }
    if (y.iter >= maxit) {
        y.done = true;
        y.status = FVPCG_NOT_CONVERGED;
        return;
    }
    double beta, den;
    if (first) {
        beta = 0.0;
        den = delta;
    } else {
        beta = gamma / y.gamma;
        den = delta - beta * gamma / y.alpha;
    }
    const double alpha = gamma / den;
    if (!(den > 0.0) || !isfinite(den) || !isfinite(alpha) || !isfinite(beta)) {
        y.done = true;
        y.status = FVPCG_BREAKDOWN;
        return;
    }
    y.gamma = gamma;
    y.alpha = alpha;
    y.beta = beta;
}

// r = b - A x over the member's rows and (b, b); returns false (x zeroed)
// when b = 0.
template <int BS, int WT, typename CI>
__device__ bool sys_begin(const BatchArgs& a, int c0, int c1, Sys& y, Team& tm, double* zero0, double* zero1,
                          double* zero2) {
    double acc[1] = {0.0};
    TEAM_ROWS(c) {
        const double bc = a.b[c];
        a.r[c] = bc - gather<WT, CI>(a.col, a.val, a.n, c, a.x, a.d[c] * a.x[c]);
        if (zero0) zero0[c] = 0.0;
        if (zero1) zero1[c] = 0.0;
        if (zero2) zero2[c] = 0.0;
        acc[0] += bc * bc;
    }
    if (!team_allreduce<BS, 1>(acc, tm)) {
        y.done = true;
        y.status = FVPCG_DEVICE_ERROR;
        return false;
    }
    y.bnorm = sqrt(acc[0]);
    y.tol_abs = a.tol * y.bnorm;
    if (acc[0] == 0.0) {
        TEAM_ROWS(c) { a.x[c] = 0.0; }
        y.done = true;
        y.status = FVPCG_OK;
        return false;
    }
    return true;
}

template <int BS, int WT, typename CI>
__device__ void sys_finish(const BatchArgs& a, int s, int c0, int c1, Sys& y, Team& tm) {
    double acc[1] = {0.0};
    // the last updates of x must be complete in every member before the gather
    if (!team_barrier(tm)) y.status = FVPCG_DEVICE_ERROR;
    TEAM_ROWS(c) {
        const double rc = a.b[c] - gather<WT, CI>(a.col, a.val, a.n, c, a.x, a.d[c] * a.x[c]);
        acc[0] += rc * rc;
    }
    if (!team_allreduce<BS, 1>(acc, tm)) y.status = FVPCG_DEVICE_ERROR;
    if (tm.rank == 0 && threadIdx.x == 0) {
        BatchStat st;
        st.iters = y.iter;
        st.status = y.status;
        st.bnorm = y.bnorm;
        st.r0norm = y.r0norm;
        st.rho = y.rho;
        st.true_rr = acc[0];
        a.stats[s] = st;
    }
}

template <int BS, int WT, typename CI, bool JAC>
__device__ void solve_pipe(const BatchArgs& a, int s, Team& tm) {
    const int c0 = a.cell_off[s], c1 = a.cell_off[s + 1];
    const double* val = JAC ? a.val_cs : a.val;
    Sys y;
    if (sys_begin<BS, WT, CI>(a, c0, c1, y, tm, a.z, a.s, a.p)) {
        double acc[3] = {0.0, 0.0, 0.0};
        TEAM_ROWS(c) {
            const double rc = a.r[c], dc = a.d[c];
            const double wc = gather<WT, CI>(a.col, val, a.n, c, a.r, JAC ? rc : dc * rc);
            a.w0[c] = wc;
            const double uc = JAC ? rc / dc : rc;
            acc[0] += rc * uc;
            acc[1] += wc * uc;
            acc[2] += rc * rc;
        }
        if (!team_allreduce<BS, 3>(acc, tm)) {
            y.done = true;
            y.status = FVPCG_DEVICE_ERROR;
        } else {
            y.r0norm = sqrt(acc[2]);
            pipe_step(y, acc[0], acc[1], acc[2], true, a.maxit);
        }
        int it = 0;
        while (!y.done) {
            const double* w_in = (it & 1) ? a.w1 : a.w0;
            double* w_out = (it & 1) ? a.w0 : a.w1;
            const double alpha = y.alpha, beta = y.beta;
            double t[3] = {0.0, 0.0, 0.0};
            TEAM_ROWS(c) {
                const double wc = w_in[c], dc = a.d[c];
                const double nv = gather<WT, CI>(a.col, val, a.n, c, w_in, JAC ? wc : dc * wc);
                const double zc = nv + beta * a.z[c];
                const double sc = wc + beta * a.s[c];
                double rc = a.r[c];
                const double uc = JAC ? rc / dc : rc;
                const double pc = uc + beta * a.p[c];
                a.p[c] = pc;
                a.x[c] += alpha * pc;
                rc -= alpha * sc;
                const double wn = wc - alpha * zc;
                a.z[c] = zc;
                a.s[c] = sc;
                a.r[c] = rc;
                w_out[c] = wn;
                const double un = JAC ? rc / dc : rc;
                t[0] += rc * un;
                t[1] += wn * un;
                t[2] += rc * rc;
            }
            if (!team_allreduce<BS, 3>(t, tm)) {
                y.done = true;
                y.status = FVPCG_DEVICE_ERROR;
                break;
            }
            pipe_step(y, t[0], t[1], t[2], false, a.maxit);
            ++it;
        }
    }
    sys_finish<BS, WT, CI>(a, s, c0, c1, y, tm);
}

template <int BS, int WT, typename CI, bool JAC>
__device__ void solve_cg(const BatchArgs& a, int s, Team& tm) {
    const int c0 = a.cell_off[s], c1 = a.cell_off[s + 1];
    Sys y;
    if (sys_begin<BS, WT, CI>(a, c0, c1, y, tm, nullptr, nullptr, nullptr)) {
        double acc[2] = {0.0, 0.0};
        TEAM_ROWS(c) {
            const double rc = a.r[c];
            const double zc = JAC ? rc / a.d[c] : rc;
            a.p[c] = zc;
            acc[0] += rc * zc;
            acc[1] += rc * rc;
        }
        if (!team_allreduce<BS, 2>(acc, tm)) {
            y.done = true;
            y.status = FVPCG_DEVICE_ERROR;
        } else {
            y.gamma = acc[0];
            y.rho = acc[1];
            y.r0norm = sqrt(acc[1]);
            if (y.r0norm <= y.tol_abs) {
                y.done = true;
                y.status = FVPCG_OK;
            } else if (a.maxit <= 0) {
                y.done = true;
            }
        }
        while (!y.done) {
            double t1[1] = {0.0};
            TEAM_ROWS(c) {
                const double pc = a.p[c];
                const double qc = gather<WT, CI>(a.col, a.val, a.n, c, a.p, a.d[c] * pc);
                a.q[c] = qc;
                t1[0] += pc * qc;
            }
            if (!team_allreduce<BS, 1>(t1, tm)) {
                y.done = true;
                y.status = FVPCG_DEVICE_ERROR;
                break;
            }
            const double delta = t1[0];
            if (!(delta > 0.0) || !isfinite(delta) || !isfinite(y.gamma)) {
                y.done = true;
                y.status = FVPCG_BREAKDOWN;
                break;
            }
            const double alpha = y.gamma / delta;
            double t2[2] = {0.0, 0.0};
            TEAM_ROWS(c) {
                a.x[c] += alpha * a.p[c];
                const double rc = a.r[c] - alpha * a.q[c];
                a.r[c] = rc;
                const double zc = JAC ? rc / a.d[c] : rc;
                t2[0] += rc * zc;
                t2[1] += rc * rc;
            }
            if (!team_allreduce<BS, 2>(t2, tm)) {
                y.done = true;
                y.status = FVPCG_DEVICE_ERROR;
                break;
            }
            y.iter += 1;
            y.rho = t2[1];
            if (sqrt(t2[1]) <= y.tol_abs) {
                y.done = true;
                y.status = FVPCG_OK;
                break;
            }
            if (y.iter >= a.maxit) {
                y.done = true;
                break;
            }
            const double beta = t2[0] / y.gamma;
            y.gamma = t2[0];
            TEAM_ROWS(c) {
                const double rc = a.r[c];
                const double zc = JAC ? rc / a.d[c] : rc;
                a.p[c] = zc + beta * a.p[c];
            }
            if (!team_barrier(tm)) {
                y.done = true;
                y.status = FVPCG_DEVICE_ERROR;
                break;
            }
        }
    }
    sys_finish<BS, WT, CI>(a, s, c0, c1, y, tm);
}

template <int BS, int WT, typename CI, bool JAC, int METHOD>
__device__ __forceinline__ void solve_one(const BatchArgs& a, int s, Team& tm) {
    if (METHOD == 1)
        solve_pipe<BS, WT, CI, JAC>(a, s, tm);
    else
        solve_cg<BS, WT, CI, JAC>(a, s, tm);
}

// method: 0 standard CG, 1 pipelined CG.  A workgroup first does its static
// team task (if any), then takes single-workgroup systems from the queue.
template <int BS, int WT, typename CI, bool JAC, int METHOD>
__global__ __launch_bounds__(BS) void k_batch(BatchArgs a) {
    __shared__ int s_next;
    const int4 task = a.tasks[blockIdx.x];
    if (task.x >= 0) {
        Team tm{task.y, task.z, a.arrive + task.x, a.team_part + task.w, a.abort_flag, a.spin_ticks, 0, 0};
        solve_one<BS, WT, CI, JAC, METHOD>(a, task.x, tm);
        __syncthreads();
    }
    for (;;) {
        if (threadIdx.x == 0) {
            int next = -1;
            if (!__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                const unsigned k = atomicAdd(a.queue, 1u);
                next = (k < (unsigned)a.nsys) ? a.order[k] : -1;
            }
            s_next = next;
        }
        __syncthreads();
        const int s = s_next;
        __syncthreads();
        if (s < 0) return;
        Team tm{0, 1, nullptr, nullptr, a.abort_flag, a.spin_ticks, 0, 0};
        solve_one<BS, WT, CI, JAC, METHOD>(a, s, tm);
        __syncthreads();
    }
}

// Per launch: queue head, team barrier counters and the abort flag to zero
// (a kernel, not a memset, so the captured graph replays it faithfully).
__global__ void k_queue_reset(unsigned* q, unsigned long long* arrive, int nsys, int* abort_flag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsys; i += gridDim.x * blockDim.x) arrive[i] = 0ull;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *q = 0u;
        *abort_flag = 0;
    }
}

__global__ void k_offset_faces(const int* __restrict__ owner, const int* __restrict__ nb, const int* __restrict__ face_off,
                               const int* __restrict__ cell_off, int nsys, int F, int* og, int* ng, unsigned* bad) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) {
        int lo = 0, hi = nsys - 1;  // system with face_off[s] <= f < face_off[s+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (face_off[mid] <= f) lo = mid;
            else hi = mid - 1;
        }
        const int c0 = cell_off[lo], ns = cell_off[lo + 1] - c0;
        const int o = owner[f], m = nb[f];
        if (o < 0 || m >= ns || o >= m) {
            atomicOr(bad, 1u);
            og[f] = 0;
            ng[f] = 1;
        } else {
            og[f] = o + c0;
            ng[f] = m + c0;
        }
    }
}

// ----------------------------------------------------------------- launching

typedef void (*BatchKernel)(BatchArgs);

template <int BS, typename CI, bool JAC, int METHOD>
BatchKernel pick_wt_kernel(int wt) {
    switch (wt) {
        case 4: return k_batch<BS, 4, CI, JAC, METHOD>;
        case 6: return k_batch<BS, 6, CI, JAC, METHOD>;
        case 8: return k_batch<BS, 8, CI, JAC, METHOD>;
        case 16: return k_batch<BS, 16, CI, JAC, METHOD>;
        default: return k_batch<BS, 32, CI, JAC, METHOD>;
    }
}

template <int BS, typename CI>
BatchKernel pick_kernel_ci(int wt, bool jac, int method) {
    if (method == 1) return jac ? pick_wt_kernel<BS, CI, true, 1>(wt) : pick_wt_kernel<BS, CI, false, 1>(wt);
    return jac ? pick_wt_kernel<BS, CI, true, 0>(wt) : pick_wt_kernel<BS, CI, false, 0>(wt);
}

template <int BS>
BatchKernel pick_kernel_bs(int wt, bool col16, bool jac, int method) {
    return col16 ? pick_kernel_ci<BS, int16_t>(wt, jac, method) : pick_kernel_ci<BS, int>(wt, jac, method);
}

BatchKernel pick_kernel(int bs, int wt, bool col16, bool jac, int method) {
    if (bs == 1024) return pick_kernel_bs<1024>(wt, col16, jac, method);
    if (bs == 512) return pick_kernel_bs<512>(wt, col16, jac, method);
    return pick_kernel_bs<256>(wt, col16, jac, method);
}

int device_cus(int* cus) {
    int dev = 0;
    FV_HIP(hipGetDevice(&dev));
    FV_HIP(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    return FVPCG_OK;
}

// Workgroups of one launch: all resident at once (occupancy-limited), which
// the team barriers rely on; without teams, no more than there are systems.
int grid_for(const fvpcg_batch* bt, const Tuning& t, BatchKernel k, int* grid) {
    int cus = 0, occ = 0;
    int rc;
    if ((rc = device_cus(&cus))) return rc;
    FV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, t.block, 0));
    const int per_cu = std::max(1, std::min(occ, t.per_cu));
    int g = cus * per_cu;
    if (!t.teams) g = std::min(g, bt->nsys);
    *grid = std::max(1, std::min(g, bt->pmax));
    return FVPCG_OK;
}

// Work table for a launch of P workgroups.  Cost of a system ~ n^(4/3)
// (cells times iterations, and CG iterations grow like the mesh edge for
// these Laplacians).  A system costing at least a workgroup's fair share C/P
// gets a team of about cost/share workgroups (at most one per tile), taken
// from one XCD's workgroups (b % 8) where they fit so the team shares an L2;
// the others go to the queue, largest first.  Returns the queue length.
int plan(fvpcg_batch* bt, int P, int bs, bool teams) {
    // measured on batch256 (pipelined / standard CG): threshold 4 share:
    // 419 / 476 ms, 2: 342 / 382 ms, 0.8 to 1.25: 330 / 355 ms; the team size
    // cap (32 to 128) and rounding up instead of to nearest change < 2%
    constexpr double kTeamThreshold = 1.0;
    constexpr int kTeamMax = 64;
    const int ns = bt->nsys;
    std::vector<double> cost(ns);
    double C = 0.0;
    for (int i = 0; i < ns; ++i) {
        cost[i] = std::pow((double)(bt->cell_off[i + 1] - bt->cell_off[i]), 4.0 / 3.0);
        C += cost[i];
    }
    const double share = C / P;
    std::vector<int> g(ns, 1);
    std::vector<int> team;
    if (teams) {
        for (int i = 0; i < ns; ++i) {
            const int tiles = (bt->cell_off[i + 1] - bt->cell_off[i] + bs - 1) / bs;
            if (cost[i] >= kTeamThreshold * share && tiles >= 2) {
                g[i] = std::max(2, std::min({(int)std::lround(cost[i] / share), tiles, kTeamMax}));
                team.push_back(i);
            }
        }
        std::sort(team.begin(), team.end(), [&](int x, int y) { return cost[x] > cost[y] || (cost[x] == cost[y] && x < y); });
        double small = 0.0;
        for (int i = 0; i < ns; ++i)
            if (g[i] == 1) small += cost[i];
        const int reserve = small > 0 ? std::max(1, (int)std::ceil(small / share)) : 0;
        auto used = [&]() { int u = 0; for (int i : team) u += g[i]; return u; };
        while (!team.empty() && used() + reserve > P) {
            int big = team[0];
            for (int i : team)
                if (g[i] > g[big]) big = i;
            if (g[big] > 2) {
                g[big] -= 1;
            } else {  // drop the cheapest team back to the queue
                g[team.back()] = 1;
                team.pop_back();
            }
        }
    }
    for (int b = 0; b < P; ++b) bt->h_tasks[b] = make_int4(-1, 0, 0, 0);
    std::vector<std::vector<int>> free_slots(8);
    for (int b = P - 1; b >= 0; --b) free_slots[b & 7].push_back(b);
    int part = 0;
    for (int i : team) {
        int rank = 0;
        while (rank < g[i]) {
            int x = 0;
            for (int k = 1; k < 8; ++k)
                if (free_slots[k].size() > free_slots[x].size()) x = k;
            if (free_slots[x].empty()) break;  // cannot happen: sum of team sizes <= P
            while (rank < g[i] && !free_slots[x].empty()) {
                const int b = free_slots[x].back();
                free_slots[x].pop_back();
                bt->h_tasks[b] = make_int4(i, rank++, g[i], part);
            }
        }
        part += 6 * g[i];
    }
    int nq = 0;
    std::vector<int> order;
    for (int i = 0; i < ns; ++i)
        if (g[i] == 1) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (bt->cell_off[x + 1] - bt->cell_off[x]) > (bt->cell_off[y + 1] - bt->cell_off[y]);
    });
    for (int i : order) bt->h_order[nq++] = i;
    return nq;
}

BatchArgs make_args(const fvpcg_batch* bt, const double* b, double* x, double tol, int maxit, int nqueue) {
    const fvpcg_matrix* A = bt->mat;
    BatchArgs a;
    a.col = bt->mesh->col16 ? (const void*)bt->mesh->col16 : (const void*)bt->mesh->col;
    a.val = A->val;
    a.val_cs = A->val_cs;
    a.d = A->d;
    a.cell_off = bt->d_cell_off;
    a.order = bt->d_order;
    a.nsys = nqueue;
    a.n = bt->ncells;
    a.b = b;
    a.x = x;
    a.r = bt->r;
    a.p = bt->p;
    a.q = bt->q;
    a.z = bt->z;
    a.s = bt->s;
    a.w0 = bt->w0;
    a.w1 = bt->w1;
    a.tol = tol;
    a.maxit = maxit;
    a.queue = bt->d_queue;
    a.stats = bt->d_stats;
    a.tasks = bt->d_tasks;
    a.arrive = bt->d_arrive;
    a.team_part = bt->d_team_part;
    a.abort_flag = bt->d_abort;
    a.spin_ticks = bt->spin_ticks;
    return a;
}

// Plan the launch and upload its tables on `s` (stream-ordered before the
// launch that uses them).
int prepare(fvpcg_batch* bt, const Tuning& t, bool jac, int method, hipStream_t s, int* grid, int* nqueue) {
    BatchKernel k = pick_kernel(t.block, bt->mesh->WT, bt->mesh->col16 != nullptr, jac, method);
    int rc;
    if ((rc = grid_for(bt, t, k, grid))) return rc;
    *nqueue = plan(bt, *grid, t.block, t.teams != 0);
    FV_HIP(hipMemcpyAsync(bt->d_tasks, bt->h_tasks, sizeof(int4) * (size_t)*grid, hipMemcpyHostToDevice, s));
    if (*nqueue > 0)
        FV_HIP(hipMemcpyAsync(bt->d_order, bt->h_order, sizeof(int) * (size_t)*nqueue, hipMemcpyHostToDevice, s));
    // the staging buffers are reused by the next plan: wait for the copies
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// Enqueue one batched solve (reset + persistent kernel) on `s`.
int launch_direct(const fvpcg_batch* bt, const Tuning& t, const BatchArgs& a, bool jac, int method, int grid,
                  hipStream_t s) {
    BatchKernel k = pick_kernel(t.block, bt->mesh->WT, bt->mesh->col16 != nullptr, jac, method);
    hipLaunchKernelGGL(k_queue_reset, dim3(std::max(1, std::min(64, (bt->nsys + 255) / 256))), dim3(256), 0, s,
                       bt->d_queue, bt->d_arrive, bt->nsys, bt->d_abort);
    hipLaunchKernelGGL(k, dim3(grid), dim3(t.block), 0, s, a);
    FV_LAUNCHED();
    return FVPCG_OK;
}

// FVPCG_BATCH_TEAMS: "0" never forms teams, "1" always offers them, unset
// lets the autotuner decide.
char teams_mode() {
    const char* e = getenv("FVPCG_BATCH_TEAMS");
    if (e && e[0] == '0') return '0';
    if (e && e[0] == '1') return '1';
    return 'a';
}

std::string tune_key(const fvpcg_batch* bt, bool jac, int method) {
    // gfx arch + sizes: the choice depends only on the shapes
    uint64_t h = 1469598103934665603ull;
    for (int v : bt->cell_off) {
        h ^= (uint64_t)v;
        h *= 1099511628211ull;
    }
    std::ostringstream os;
    os << "gfx950/nsys" << bt->nsys << "/cells" << bt->ncells << "/W" << bt->mesh->WT << "/m" << method << "/j"
       << (jac ? 1 : 0) << "/t" << teams_mode() << "/h" << std::hex << h;
    return os.str();
}

std::string cache_path() {
    const char* p = getenv("FVPCG_TUNE_CACHE");
    if (p && *p) return p;
    const char* home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/fvpcg_batched_tuning.json";
}

// The cache is a flat JSON object {"key": [block, per_cu, teams], ...}.
std::map<std::string, Tuning> load_cache() {
    std::map<std::string, Tuning> m;
    std::ifstream f(cache_path());
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t lb = s.find('[', j), rb = s.find(']', j);
        if (lb == std::string::npos || rb == std::string::npos) break;
        Tuning t;
        if (sscanf(s.c_str() + lb + 1, "%d , %d , %d", &t.block, &t.per_cu, &t.teams) == 3 &&
            (t.block == 256 || t.block == 512 || t.block == 1024) && t.per_cu >= 1 && t.per_cu <= 16 &&
            (t.teams == 0 || t.teams == 1))
            m[key] = t;
        i = rb + 1;
    }
    return m;
}

void store_cache(const std::string& key, const Tuning& t) {
    std::map<std::string, Tuning> m = load_cache();
    m[key] = t;
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        size_t pos = 1;  // create missing parent directories
        while ((pos = dir.find('/', pos)) != std::string::npos) {
            (void)mkdir(dir.substr(0, pos).c_str(), 0755);
            ++pos;
        }
        (void)mkdir(dir.c_str(), 0755);
    }
    const std::string tmp = path + ".tmp";
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (auto& kv : m)
        f << "  \"" << kv.first << "\": [" << kv.second.block << ", " << kv.second.per_cu << ", " << kv.second.teams
          << "]" << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    (void)rename(tmp.c_str(), path.c_str());
}

// Upload the work table for tuning t unless the device already holds it.
int ensure_plan(fvpcg_batch* bt, const Tuning& t, bool jac, int method, hipStream_t s, int* grid, int* nqueue) {
    BatchKernel k = pick_kernel(t.block, bt->mesh->WT, bt->mesh->col16 != nullptr, jac, method);
    int rc, g = 0;
    if ((rc = grid_for(bt, t, k, &g))) return rc;
    if (bt->plan_grid == g && bt->plan_block == t.block && bt->plan_teams == t.teams) {
        *grid = g;
        *nqueue = bt->plan_queue;
        return FVPCG_OK;
    }
    bt->plan_grid = -1;
    if ((rc = prepare(bt, t, jac, method, s, grid, nqueue))) return rc;
    bt->plan_grid = *grid;
    bt->plan_block = t.block;
    bt->plan_teams = t.teams;
    bt->plan_queue = *nqueue;
    return FVPCG_OK;
}

int check_abort(fvpcg_batch* bt, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(bt->h_abort, bt->d_abort, sizeof(int), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    if (*bt->h_abort)
        return set_error(FVPCG_DEVICE_ERROR, "batched solve: a workgroup team barrier timed out (results invalid)");
    return FVPCG_OK;
}

// Pick block size, workgroups per CU and teams on/off by timing each
// candidate on this batch (a copy of x0, the caller's tolerance), fastest
// wins.
int autotune(fvpcg_batch* bt, const double* b, const double* x0, double tol, int maxit, bool jac, int method,
             hipStream_t s, Tuning* out) {
    const std::string key = tune_key(bt, jac, method);
    auto it = bt->tuned.find(key);
    if (it != bt->tuned.end()) {
        *out = it->second;
        return FVPCG_OK;
    }
    const char mode = teams_mode();
    const char* env = getenv("FVPCG_TUNE");
    if (env && env[0] == '0') {
        *out = Tuning();
        out->teams = mode == '1' ? 1 : 0;
        bt->tuned[key] = *out;
        return FVPCG_OK;
    }
    std::map<std::string, Tuning> cache = load_cache();
    auto ct = cache.find(key);
    if (ct != cache.end()) {
        *out = ct->second;
        bt->tuned[key] = *out;
        return FVPCG_OK;
    }
    int rc;
    if (!bt->xscratch && (rc = dev_alloc(&bt->xscratch, (size_t)bt->ncells, "batched tuning x"))) return rc;
    std::vector<Tuning> cands;
    const int shapes[][2] = {{256, 4}, {256, 8}, {512, 2}, {512, 4}, {1024, 1}, {1024, 2}};
    for (int tm = 0; tm < 2; ++tm) {
        if ((mode == '0' && tm == 1) || (mode == '1' && tm == 0)) continue;
        for (auto& sh : shapes) {
            Tuning t;
            t.block = sh[0];
            t.per_cu = sh[1];
            t.teams = tm;
            cands.push_back(t);
        }
    }
    float best = 1e30f;
    Tuning pick = cands[0];
    for (const Tuning& t : cands) {
        int grid = 0, nq = 0;
        if ((rc = ensure_plan(bt, t, jac, method, s, &grid, &nq))) return rc;
        float ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            FV_HIP(hipMemcpyAsync(bt->xscratch, x0, sizeof(double) * (size_t)bt->ncells, hipMemcpyDeviceToDevice, s));
            FV_HIP(hipEventRecord(bt->e0, s));
            if ((rc = launch_direct(bt, t, make_args(bt, b, bt->xscratch, tol, maxit, nq), jac, method, grid, s)))
                return rc;
            FV_HIP(hipEventRecord(bt->e1, s));
            FV_HIP(hipEventSynchronize(bt->e1));
            FV_HIP(hipEventElapsedTime(&ms, bt->e0, bt->e1));
        }
        if ((rc = check_abort(bt, s))) return rc;
        if (ms < best) {
            best = ms;
            pick = t;
        }
    }
    bt->tuned[key] = pick;
    store_cache(key, pick);
    *out = pick;
    return FVPCG_OK;
}

void batch_free(fvpcg_batch* bt) {
    if (!bt) return;
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    if (bt->mat) matrix_destroy(bt->mat);
    if (bt->mesh) mesh_destroy(bt->mesh);
    dev_free(bt->d_cell_off);
    dev_free(bt->d_order);
    dev_free(bt->d_queue);
    dev_free(bt->d_stats);
    dev_free(bt->d_tasks);
    dev_free(bt->d_arrive);
    dev_free(bt->d_team_part);
    dev_free(bt->d_abort);
    double** vs[] = {&bt->r, &bt->p, &bt->q, &bt->z, &bt->s, &bt->w0, &bt->w1, &bt->xscratch, &bt->lam};
    for (double** v : vs) dev_free(*v);
    if (bt->h_stats) (void)hipHostFree(bt->h_stats);
    if (bt->h_tasks) (void)hipHostFree(bt->h_tasks);
    if (bt->h_order) (void)hipHostFree(bt->h_order);
    if (bt->h_abort) (void)hipHostFree(bt->h_abort);
    if (bt->capture) (void)hipStreamDestroy(bt->capture);
    if (bt->e0) (void)hipEventDestroy(bt->e0);
    if (bt->e1) (void)hipEventDestroy(bt->e1);
    delete bt;
}

}  // namespace

int batch_create(int32_t nsys, const int32_t* cell_off, const int32_t* face_off, const int32_t* owner, const int32_t* nb,
                 const double* diag, const double* upper, const double* lower, uint32_t, hipStream_t s,
                 fvpcg_batch** out) {
    fvpcg_batch* bt = new (std::nothrow) fvpcg_batch();
    if (!bt) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    bt->nsys = nsys;
    bt->ncells = cell_off[nsys];
    bt->nfaces = face_off[nsys];
    bt->cell_off.assign(cell_off, cell_off + nsys + 1);
    bt->face_off.assign(face_off, face_off + nsys + 1);
    int rc = FVPCG_OK;
    int *og = nullptr, *ng = nullptr, *dfo = nullptr;
    unsigned* bad = nullptr;
    auto fail = [&](int code) {
        dev_free(og);
        dev_free(ng);
        dev_free(dfo);
        dev_free(bad);
        batch_free(bt);
        return code;
    };
    const size_t n = (size_t)bt->ncells, F = (size_t)bt->nfaces;
    if ((rc = dev_alloc(&bt->d_cell_off, (size_t)nsys + 1, "cell offsets")) ||
        (rc = dev_alloc(&dfo, (size_t)nsys + 1, "face offsets")) || (rc = dev_alloc(&og, F, "owner")) ||
        (rc = dev_alloc(&ng, F, "neighbour")) || (rc = dev_alloc(&bad, 1, "flag")))
        return fail(rc);
#define CK(x)                                                                    \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) return fail(hip_fail(e_, #x, __FILE__, __LINE__)); \
    } while (0)
    CK(hipMemcpyAsync(bt->d_cell_off, cell_off, sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(dfo, face_off, sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
    CK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    if (F > 0) {
        int g = (int)std::min<size_t>((F + kBlock - 1) / kBlock, 65536);
        hipLaunchKernelGGL(k_offset_faces, dim3(g), dim3(kBlock), 0, s, owner, nb, dfo, bt->d_cell_off, nsys, (int)F,
                           og, ng, bad);
        CK(hipGetLastError());
    }
    unsigned hbad = 0;
    CK(hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (hbad) return fail(set_error(FVPCG_INVALID_MESH, "a face addresses a cell outside its system or owner >= neighbour"));
    if ((rc = mesh_create((int)n, (int)F, og, ng, s, &bt->mesh))) return fail(rc);
    dev_free(og);
    dev_free(ng);
    dev_free(dfo);
    dev_free(bad);
    if ((rc = matrix_create(bt->mesh, diag, upper, lower, 0, s, &bt->mat))) return fail(rc);
    // launch tables: at most 16 workgroups per CU are ever resident
    int cus = 0;
    if ((rc = device_cus(&cus))) return fail(rc);
    bt->pmax = 16 * cus;
    if ((rc = dev_alloc(&bt->d_order, (size_t)nsys, "system order")) || (rc = dev_alloc(&bt->d_queue, 1, "queue")) ||
        (rc = dev_alloc(&bt->d_stats, (size_t)nsys, "system stats")) ||
        (rc = dev_alloc(&bt->d_tasks, (size_t)bt->pmax, "team tasks")) ||
        (rc = dev_alloc(&bt->d_arrive, (size_t)nsys, "team barriers")) ||
        (rc = dev_alloc(&bt->d_team_part, (size_t)6 * bt->pmax, "team partials")) ||
        (rc = dev_alloc(&bt->d_abort, 1, "abort flag")))
        return fail(rc);
    double** vs[] = {&bt->r, &bt->p, &bt->q, &bt->z, &bt->s, &bt->w0, &bt->w1};
    for (double** v : vs)
        if ((rc = dev_alloc(v, n, "batched vector"))) return fail(rc);
    if (hipHostMalloc((void**)&bt->h_stats, sizeof(BatchStat) * nsys, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&bt->h_tasks, sizeof(int4) * bt->pmax, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&bt->h_order, sizeof(int) * nsys, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&bt->h_abort, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(set_error(FVPCG_OUT_OF_MEMORY, "pinned allocation failed"));
    *bt->h_abort = 0;
    // team barrier timeout (FVPCG_BATCH_BARRIER_TIMEOUT_MS, default 5 s) in
    // wall-clock ticks
    {
        int dev = 0, khz = 0;
        CK(hipGetDevice(&dev));
        CK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        const char* e = getenv("FVPCG_BATCH_BARRIER_TIMEOUT_MS");
        double ms = 5000.0;
        if (e && *e) ms = std::max(0.0, atof(e));
        bt->spin_ticks = (unsigned long long)((double)std::max(khz, 1) * ms);
    }
    CK(hipStreamCreateWithFlags(&bt->capture, hipStreamNonBlocking));
    CK(hipEventCreate(&bt->e0));
    CK(hipEventCreate(&bt->e1));
    CK(hipStreamSynchronize(s));
#undef CK
    *out = bt;
    return FVPCG_OK;
}

bool batch_symmetric(const fvpcg_batch* bt) { return bt->mat->vals_sym; }

int batch_destroy(fvpcg_batch* bt) {
    batch_free(bt);
    return FVPCG_OK;
}
int batch_total_cells(const fvpcg_batch* bt) { return bt->ncells; }
int batch_total_faces(const fvpcg_batch* bt) { return bt->nfaces; }
int batch_nsys(const fvpcg_batch* bt) { return bt->nsys; }

int solve_batched(const fvpcg_batch* cbt, const double* b, double* x, double tol, int maxit, int method, int precond,
                  hipStream_t s, fvpcg_stats* stats) {
    fvpcg_batch* bt = const_cast<fvpcg_batch*>(cbt);
    const bool jac = precond == FVPCG_PRECOND_JACOBI;
    if (jac && !bt->mat->diag_ok)
        return set_error(FVPCG_BREAKDOWN, "Jacobi preconditioner needs a finite positive diagonal");
    if (method == FVPCG_PIPECG_LITERAL) {
        if (jac) return set_error(FVPCG_UNSUPPORTED, "batched solver: literal pipelined form not built");
        method = FVPCG_PIPECG;
    }
    const int m = method == FVPCG_CG ? 0 : 1;
    int rc;
    Tuning t;
    if ((rc = autotune(bt, b, x, tol, maxit, jac, m, s, &t))) return rc;
    int grid = 0, nq = 0;
    if ((rc = ensure_plan(bt, t, jac, m, s, &grid, &nq))) return rc;
    // graph of (queue reset, persistent solve) for these arguments
    std::ostringstream os;
    os << (const void*)b << '/' << (const void*)x << '/' << tol << '/' << maxit << '/' << m << '/' << jac << '/'
       << t.block << '/' << t.per_cu << '/' << t.teams << '/' << grid << '/' << nq;
    if (!bt->gexec || bt->gkey != os.str()) {
        if (bt->gexec) {
            (void)hipGraphExecDestroy(bt->gexec);
            bt->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        FV_HIP(hipStreamBeginCapture(bt->capture, hipStreamCaptureModeThreadLocal));
        int lrc = launch_direct(bt, t, make_args(bt, b, x, tol, maxit, nq), jac, m, grid, bt->capture);
        hipError_t e = hipStreamEndCapture(bt->capture, &graph);
        if (lrc) {
            if (graph) (void)hipGraphDestroy(graph);
            return lrc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
        e = hipGraphInstantiate(&bt->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            bt->gexec = nullptr;
            return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__);
        }
        bt->gkey = os.str();
    }
    FV_HIP(hipEventRecord(bt->e0, s));
    FV_HIP(hipGraphLaunch(bt->gexec, s));
    FV_HIP(hipEventRecord(bt->e1, s));
    FV_HIP(hipMemcpyAsync(bt->h_stats, bt->d_stats, sizeof(BatchStat) * bt->nsys, hipMemcpyDeviceToHost, s));
    if ((rc = check_abort(bt, s))) return rc;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, bt->e0, bt->e1);
    int overall = FVPCG_OK;
    for (int i = 0; i < bt->nsys; ++i) {
        const BatchStat& h = bt->h_stats[i];
        if (stats) {
            fvpcg_stats& o = stats[i];
            o.iters = h.iters;
            o.outer_iters = 0;
            o.status = h.status;
            o.reserved = 0;
            o.b_norm = h.bnorm;
            o.r0_norm = h.r0norm;
            o.rel_res = h.bnorm > 0 ? sqrt(h.rho) / h.bnorm : 0.0;
            o.true_rel_res = h.bnorm > 0 ? sqrt(h.true_rr) / h.bnorm : 0.0;
            o.device_ms = ms;
            o.iter_ms = ms;
        }
        if (overall == FVPCG_OK && h.status != FVPCG_OK) overall = h.status;
    }
    if (overall == FVPCG_BREAKDOWN) set_error(overall, "breakdown in at least one system");
    return overall;
}

int solve_batched_backward(const fvpcg_batch* cbt, const double* x, const double* g, double* grad_b, double* grad_diag,
                           double* grad_upper, double* grad_lower, double tol, int maxit, int method, int precond,
                           hipStream_t s, fvpcg_stats* stats) {
    fvpcg_batch* bt = const_cast<fvpcg_batch*>(cbt);
    int rc;
    double* lam = grad_b;
    if (!lam) {
        if (!bt->lam && (rc = dev_alloc(&bt->lam, (size_t)bt->ncells, "adjoint solution"))) return rc;
        lam = bt->lam;
    }
    FV_HIP(hipMemsetAsync(lam, 0, sizeof(double) * (size_t)bt->ncells, s));
    const int st = solve_batched(bt, g, lam, tol, maxit, method, precond, s, stats);
    if (st < 0) return st;
    if ((rc = adjoint_grads(bt->mat, x, lam, nullptr, grad_diag, grad_upper, grad_lower, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    return st;
}

}  // namespace fvpcg
