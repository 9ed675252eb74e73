// Batched solves: many independent LDU systems of uneven sizes in one
// persistent launch, captured in a hipGraph.
//
// The systems are stored as one block-diagonal matrix (their addressing
// offset by each system's first cell), so the ELL layout, validation and
// coefficient handling are the single-system ones.  One workgroup solves one
// system from start to finish: its rows, its reductions (wave butterfly +
// LDS, fixed order) and its scalars stay inside the workgroup, so no
// workgroup ever waits for another.  Workgroups take systems from a device
// queue ordered by decreasing size (largest first, the list-scheduling rule
// that keeps the tail short); a launch uses min(nsys, resident capacity)
// workgroups.  Block size and workgroups per CU are chosen per batch by a
// small autotuner that times the candidates on the batch itself and caches
// the choice in a JSON file.
#include <sys/stat.h>

#include <algorithm>
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
    const int* order;  // systems, largest first
    int nsys;
    int n;  // total cells (slot stride)
    const double* b;
    double* x;
    double *r, *p, *q, *z, *s, *w0, *w1;
    double tol;
    int maxit;
    unsigned* queue;
    BatchStat* stats;
};

struct Tuning {
    int block = 256;
    int per_cu = 4;
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
    // cached graph
    hipGraphExec_t gexec = nullptr;
    std::string gkey;
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

// r = b - A x over [c0, c1) and (b, b); returns false (x zeroed) when b = 0.
template <int BS, int WT, typename CI>
__device__ bool sys_begin(const BatchArgs& a, int c0, int c1, Sys& y, double* zero0, double* zero1, double* zero2) {
    double acc[1] = {0.0};
    for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
        const double bc = a.b[c];
        a.r[c] = bc - gather<WT, CI>(a.col, a.val, a.n, c, a.x, a.d[c] * a.x[c]);
        if (zero0) zero0[c] = 0.0;
        if (zero1) zero1[c] = 0.0;
        if (zero2) zero2[c] = 0.0;
        acc[0] += bc * bc;
    }
    block_allreduce<BS, 1>(acc);
    y.bnorm = sqrt(acc[0]);
    y.tol_abs = a.tol * y.bnorm;
    if (acc[0] == 0.0) {
        for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) a.x[c] = 0.0;
        y.done = true;
        y.status = FVPCG_OK;
        return false;
    }
    return true;
}

template <int BS, int WT, typename CI>
__device__ void sys_finish(const BatchArgs& a, int s, int c0, int c1, const Sys& y) {
    __syncthreads();
    double acc[1] = {0.0};
    for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
        const double rc = a.b[c] - gather<WT, CI>(a.col, a.val, a.n, c, a.x, a.d[c] * a.x[c]);
        acc[0] += rc * rc;
    }
    block_allreduce<BS, 1>(acc);
    if (threadIdx.x == 0) {
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
__device__ void solve_pipe(const BatchArgs& a, int s) {
    const int c0 = a.cell_off[s], c1 = a.cell_off[s + 1];
    const double* val = JAC ? a.val_cs : a.val;
    Sys y;
    if (sys_begin<BS, WT, CI>(a, c0, c1, y, a.z, a.s, a.p)) {
        __syncthreads();
        double acc[3] = {0.0, 0.0, 0.0};
        for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
            const double rc = a.r[c], dc = a.d[c];
            const double wc = gather<WT, CI>(a.col, val, a.n, c, a.r, JAC ? rc : dc * rc);
            a.w0[c] = wc;
            const double uc = JAC ? rc / dc : rc;
            acc[0] += rc * uc;
            acc[1] += wc * uc;
            acc[2] += rc * rc;
        }
        block_allreduce<BS, 3>(acc);
        y.r0norm = sqrt(acc[2]);
        pipe_step(y, acc[0], acc[1], acc[2], true, a.maxit);
        int it = 0;
        while (!y.done) {
            const double* w_in = (it & 1) ? a.w1 : a.w0;
            double* w_out = (it & 1) ? a.w0 : a.w1;
            const double alpha = y.alpha, beta = y.beta;
            double t[3] = {0.0, 0.0, 0.0};
            for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
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
            block_allreduce<BS, 3>(t);
            pipe_step(y, t[0], t[1], t[2], false, a.maxit);
            ++it;
        }
    }
    sys_finish<BS, WT, CI>(a, s, c0, c1, y);
}

template <int BS, int WT, typename CI, bool JAC>
__device__ void solve_cg(const BatchArgs& a, int s) {
    const int c0 = a.cell_off[s], c1 = a.cell_off[s + 1];
    Sys y;
    if (sys_begin<BS, WT, CI>(a, c0, c1, y, nullptr, nullptr, nullptr)) {
        double acc[2] = {0.0, 0.0};
        for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
            const double rc = a.r[c];
            const double zc = JAC ? rc / a.d[c] : rc;
            a.p[c] = zc;
            acc[0] += rc * zc;
            acc[1] += rc * rc;
        }
        block_allreduce<BS, 2>(acc);
        y.gamma = acc[0];
        y.rho = acc[1];
        y.r0norm = sqrt(acc[1]);
        if (y.r0norm <= y.tol_abs) {
            y.done = true;
            y.status = FVPCG_OK;
        } else if (a.maxit <= 0) {
            y.done = true;
        }
        while (!y.done) {
            double t1[1] = {0.0};
            for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
                const double pc = a.p[c];
                const double qc = gather<WT, CI>(a.col, a.val, a.n, c, a.p, a.d[c] * pc);
                a.q[c] = qc;
                t1[0] += pc * qc;
            }
            block_allreduce<BS, 1>(t1);
            const double delta = t1[0];
            if (!(delta > 0.0) || !isfinite(delta) || !isfinite(y.gamma)) {
                y.done = true;
                y.status = FVPCG_BREAKDOWN;
                break;
            }
            const double alpha = y.gamma / delta;
            double t2[2] = {0.0, 0.0};
            for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
                a.x[c] += alpha * a.p[c];
                const double rc = a.r[c] - alpha * a.q[c];
                a.r[c] = rc;
                const double zc = JAC ? rc / a.d[c] : rc;
                t2[0] += rc * zc;
                t2[1] += rc * rc;
            }
            block_allreduce<BS, 2>(t2);
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
            for (int c = c0 + (int)threadIdx.x; c < c1; c += BS) {
                const double rc = a.r[c];
                const double zc = JAC ? rc / a.d[c] : rc;
                a.p[c] = zc + beta * a.p[c];
            }
            __syncthreads();
        }
    }
    sys_finish<BS, WT, CI>(a, s, c0, c1, y);
}

// method: 0 standard CG, 1 pipelined CG
template <int BS, int WT, typename CI, bool JAC, int METHOD>
__global__ __launch_bounds__(BS) void k_batch(BatchArgs a) {
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned k = atomicAdd(a.queue, 1u);
            s_next = (k < (unsigned)a.nsys) ? a.order[k] : -1;
        }
        __syncthreads();
        const int s = s_next;
        __syncthreads();
        if (s < 0) return;
        if (METHOD == 1)
            solve_pipe<BS, WT, CI, JAC>(a, s);
        else
            solve_cg<BS, WT, CI, JAC>(a, s);
        __syncthreads();
    }
}

__global__ void k_queue_reset(unsigned* q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0u;
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

int grid_for(const fvpcg_batch* bt, const Tuning& t, BatchKernel k, int* grid) {
    int cus = 0, occ = 0;
    int rc;
    if ((rc = device_cus(&cus))) return rc;
    FV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, t.block, 0));
    const int per_cu = std::max(1, std::min(occ, t.per_cu));
    *grid = std::max(1, std::min(bt->nsys, cus * per_cu));
    return FVPCG_OK;
}

BatchArgs make_args(const fvpcg_batch* bt, const double* b, double* x, double tol, int maxit) {
    const fvpcg_matrix* A = bt->mat;
    BatchArgs a;
    a.col = bt->mesh->col16 ? (const void*)bt->mesh->col16 : (const void*)bt->mesh->col;
    a.val = A->val;
    a.val_cs = A->val_cs;
    a.d = A->d;
    a.cell_off = bt->d_cell_off;
    a.order = bt->d_order;
    a.nsys = bt->nsys;
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
    return a;
}

// Enqueue one batched solve directly (used while tuning).
int launch_direct(const fvpcg_batch* bt, const Tuning& t, const BatchArgs& a, bool jac, int method, hipStream_t s) {
    BatchKernel k = pick_kernel(t.block, bt->mesh->WT, bt->mesh->col16 != nullptr, jac, method);
    int grid = 1, rc;
    if ((rc = grid_for(bt, t, k, &grid))) return rc;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, bt->d_queue);
    hipLaunchKernelGGL(k, dim3(grid), dim3(t.block), 0, s, a);
    FV_LAUNCHED();
    return FVPCG_OK;
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
       << (jac ? 1 : 0) << "/h" << std::hex << h;
    return os.str();
}

std::string cache_path() {
    const char* p = getenv("FVPCG_TUNE_CACHE");
    if (p && *p) return p;
    const char* home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/fvpcg_batched_tuning.json";
}

// The cache is a flat JSON object {"key": [block, per_cu], ...}.
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
        if (sscanf(s.c_str() + lb + 1, "%d , %d", &t.block, &t.per_cu) == 2 &&
            (t.block == 256 || t.block == 512 || t.block == 1024) && t.per_cu >= 1 && t.per_cu <= 32)
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
    for (auto& kv : m) f << "  \"" << kv.first << "\": [" << kv.second.block << ", " << kv.second.per_cu << "]"
                          << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    (void)rename(tmp.c_str(), path.c_str());
}

// Pick block size and workgroups per CU by timing each candidate on this
// batch (a copy of x0, the caller's tolerance), fastest wins.
int autotune(fvpcg_batch* bt, const double* b, const double* x0, double tol, int maxit, bool jac, int method,
             hipStream_t s, Tuning* out) {
    const std::string key = tune_key(bt, jac, method);
    auto it = bt->tuned.find(key);
    if (it != bt->tuned.end()) {
        *out = it->second;
        return FVPCG_OK;
    }
    const char* env = getenv("FVPCG_TUNE");
    if (env && env[0] == '0') {
        *out = Tuning();
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
    const Tuning cands[] = {{256, 4}, {256, 8}, {512, 2}, {512, 4}, {1024, 1}, {1024, 2}};
    float best = 1e30f;
    Tuning pick;
    for (const Tuning& t : cands) {
        float ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            FV_HIP(hipMemcpyAsync(bt->xscratch, x0, sizeof(double) * (size_t)bt->ncells, hipMemcpyDeviceToDevice, s));
            FV_HIP(hipEventRecord(bt->e0, s));
            if ((rc = launch_direct(bt, t, make_args(bt, b, bt->xscratch, tol, maxit), jac, method, s))) return rc;
            FV_HIP(hipEventRecord(bt->e1, s));
            FV_HIP(hipEventSynchronize(bt->e1));
            FV_HIP(hipEventElapsedTime(&ms, bt->e0, bt->e1));
        }
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
    double** vs[] = {&bt->r, &bt->p, &bt->q, &bt->z, &bt->s, &bt->w0, &bt->w1, &bt->xscratch, &bt->lam};
    for (double** v : vs) dev_free(*v);
    if (bt->h_stats) (void)hipHostFree(bt->h_stats);
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
    // largest systems first
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (cell_off[a + 1] - cell_off[a]) > (cell_off[b + 1] - cell_off[b]);
    });
    if ((rc = dev_alloc(&bt->d_order, (size_t)nsys, "system order")) || (rc = dev_alloc(&bt->d_queue, 1, "queue")) ||
        (rc = dev_alloc(&bt->d_stats, (size_t)nsys, "system stats")))
        return fail(rc);
    CK(hipMemcpyAsync(bt->d_order, order.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, s));
    double** vs[] = {&bt->r, &bt->p, &bt->q, &bt->z, &bt->s, &bt->w0, &bt->w1};
    for (double** v : vs)
        if ((rc = dev_alloc(v, n, "batched vector"))) return fail(rc);
    if (hipHostMalloc((void**)&bt->h_stats, sizeof(BatchStat) * nsys, hipHostMallocDefault) != hipSuccess) {
        bt->h_stats = nullptr;
        return fail(set_error(FVPCG_OUT_OF_MEMORY, "pinned allocation failed"));
    }
    CK(hipStreamCreateWithFlags(&bt->capture, hipStreamNonBlocking));
    CK(hipEventCreate(&bt->e0));
    CK(hipEventCreate(&bt->e1));
    CK(hipStreamSynchronize(s));
#undef CK
    *out = bt;
    return FVPCG_OK;
}

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
    // graph of (queue reset, persistent solve) for these arguments
    std::ostringstream os;
    os << (const void*)b << '/' << (const void*)x << '/' << tol << '/' << maxit << '/' << m << '/' << jac << '/'
       << t.block << '/' << t.per_cu;
    if (!bt->gexec || bt->gkey != os.str()) {
        if (bt->gexec) {
            (void)hipGraphExecDestroy(bt->gexec);
            bt->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        FV_HIP(hipStreamBeginCapture(bt->capture, hipStreamCaptureModeThreadLocal));
        int lrc = launch_direct(bt, t, make_args(bt, b, x, tol, maxit), jac, m, bt->capture);
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
    FV_HIP(hipStreamSynchronize(s));
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
