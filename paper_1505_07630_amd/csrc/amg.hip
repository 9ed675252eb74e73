// Smoothed-aggregation AMG preconditioner and AMG-preconditioned CG.
//
// The paper compares its Jacobi-preconditioned CG and pipelined CG with
// aggregation-AMG preconditioned versions (Section 5, Table pcgs2) without
// printing the AMG.  This is the classical smoothed-aggregation method of
// Vanek, Mandel and Brezina:
//   strength    j ~ i iff j != i and |a_ij| >= theta_l sqrt(a_ii a_jj),
//               theta_{l+1} = theta_l / 2;
//   aggregates  three greedy passes in index order: (1) i and all its strong
//               neighbours, when none of them is aggregated, form an
//               aggregate; (2) a remaining i joins the pass-1 aggregate of its
//               strongest strong neighbour (ties: lowest index); (3) what
//               remains forms aggregates of i and its still-free neighbours;
//   prolongator P = (I - omega D^-1 A) P_t, omega = 4 / (3 lambda), lambda
//               the Gershgorin bound max_i sum_j |a_ij| / a_ii;
//   coarse      A_c = P^T A P, R = P^T; stop at n <= coarse_size, at the
//               level limit, or when aggregation keeps more than 60% of the
//               unknowns; the last level is solved exactly (its inverse,
//               formed from a Cholesky factor at setup);
//   cycle       V(1,1): x = omega D^-1 b; r = b - A x; x += P V(R r);
//               y = x + omega D^-1 (b - A x).
// The hierarchy is built on the host at setup (sparse products with a dense
// accumulator per row); the cycle runs on the device: level 0 uses the
// matrix's ELL layout (the pre-smoothing and residual in one pass through
// the column-scaled values), coarser levels CSR, one row per thread.  The
// cycle is symmetric positive definite, so standard CG can use it as M^-1.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "handles.hpp"
#include "rows.hpp"

namespace fvpcg {

constexpr int kAmgMaxLevels = 16;
constexpr int kAmgMaxCoarse = 2048;  // largest exactly-solved last level
constexpr int kAmgBs = 512;          // level-0 and PCG kernels
constexpr int kAmgCsrBs = 256;       // CSR levels, one row per thread

struct AmgLevel {
    int n = 0, nc = 0;  // rows here and on the next level
    long long nnz = 0;
    double omega = 0.0;
    int *a_ptr = nullptr, *a_col = nullptr;  // levels >= 1
    double *a_val = nullptr, *d = nullptr;   // levels >= 1
    double* a_val_cs = nullptr;              // levels >= 1: a_ij / d_j
    int *p_ptr = nullptr, *p_col = nullptr;  // P: n x nc
    double* p_val = nullptr;
    int *r_ptr = nullptr, *r_col = nullptr;  // R = P^T: nc x n
    double* r_val = nullptr;
    double *b = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;  // work
    int ga = 1, gp = 1, gr = 1;  // lanes per row for A, P, R (1, 16 or 64)
    std::vector<int> agg;
};

}  // namespace fvpcg

struct fvpcg_amg {
    const fvpcg_matrix* mat = nullptr;
    int nlev = 0;
    fvpcg::AmgLevel lev[fvpcg::kAmgMaxLevels];
    double* cinv = nullptr;  // inverse of the last level, row-major
    int nlast = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // PCG vectors
    double *u = nullptr, *w = nullptr, *m = nullptr, *s = nullptr;  // pipelined CG, allocated on first use
    fvpcg::DevState* st = nullptr;
    fvpcg::DevState* hst = nullptr;  // pinned [2]
    double* partials = nullptr;
    hipEvent_t t_begin = nullptr, t_end = nullptr, t_it0 = nullptr, t_it1 = nullptr;
};

namespace fvpcg {

namespace {

// ---------------------------------------------------------------- host setup
// Products and sums are rounded one operation at a time (no fused
// multiply-add), in the orders stated, so the hierarchy does not depend on
// the compiler's contraction choices.
#pragma clang fp contract(off)

struct Csr {
    int n = 0, m = 0;
    std::vector<int> ptr, col;
    std::vector<double> val;
};

Csr transpose(const Csr& A) {
    Csr T;
    T.n = A.m;
    T.m = A.n;
    T.ptr.assign((size_t)T.n + 1, 0);
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    for (int c : A.col) T.ptr[(size_t)c + 1]++;
    for (int j = 0; j < T.n; ++j) T.ptr[(size_t)j + 1] += T.ptr[j];
    std::vector<int> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) {
            const int q = fill[A.col[k]]++;
            T.col[q] = i;
            T.val[q] = A.val[k];
        }
    return T;
}

// f(t, begin, end) on T contiguous parts of [0, n), one host thread each
// (up to 16).  Each output element is still computed by one thread in its
// sequential order, so results do not depend on T.  False if a part failed
// (an allocation inside it), which the caller reports.
template <typename F>
bool parallel_parts(int n, int min_part, F&& f) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = std::max(1, std::min({(int)std::min(hw, 16u), n / std::max(min_part, 1), n}));
    std::atomic<bool> ok{true};
    auto run = [&](int t) {
        const int b = (int)((long long)n * t / T), e = (int)((long long)n * (t + 1) / T);
        try {
            f(t, b, e);
        } catch (...) {
            ok = false;
        }
    };
    if (T == 1) {
        run(0);
        return ok;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)T - 1);
    try {
        for (int t = 1; t < T; ++t) th.emplace_back(run, t);
    } catch (...) {
        ok = false;
    }
    run(0);
    for (auto& x : th) x.join();
    return ok;
}

// C = X Y, row by row: products summed in the order of X's columns and then
// Y's columns into a dense accumulator; columns sorted.  Rows are split over
// host threads (each with its own accumulator) and concatenated in order.
// Throws std::bad_alloc if a part runs out of memory.
Csr multiply(const Csr& X, const Csr& Y) {
    Csr C;
    C.n = X.n;
    C.m = Y.m;
    C.ptr.assign((size_t)C.n + 1, 0);
    struct Part {
        std::vector<int> col;
        std::vector<double> val;
    };
    std::vector<Part> parts(16);
    std::vector<int> len((size_t)std::max(X.n, 1), 0);
    const bool ok = parallel_parts(X.n, 4096, [&](int t, int r0, int r1) {
        Part& out = parts[(size_t)t];
        std::vector<double> acc((size_t)std::max(Y.m, 1), 0.0);
        std::vector<int> mark((size_t)std::max(Y.m, 1), -1), touched;
        for (int i = r0; i < r1; ++i) {
            touched.clear();
            for (int a = X.ptr[i]; a < X.ptr[(size_t)i + 1]; ++a) {
                const int j = X.col[a];
                const double xv = X.val[a];
                for (int b = Y.ptr[j]; b < Y.ptr[(size_t)j + 1]; ++b) {
                    const int k = Y.col[b];
                    if (mark[k] != i) {
                        mark[k] = i;
                        acc[k] = 0.0;
                        touched.push_back(k);
                    }
                    acc[k] += xv * Y.val[b];
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int k : touched) {
                out.col.push_back(k);
                out.val.push_back(acc[k]);
            }
            len[(size_t)i] = (int)touched.size();
        }
    });
    if (!ok) throw std::bad_alloc();
    for (int i = 0; i < X.n; ++i) C.ptr[(size_t)i + 1] = C.ptr[i] + len[(size_t)i];
    C.col.reserve((size_t)C.ptr[C.n]);
    C.val.reserve((size_t)C.ptr[C.n]);
    for (const Part& q : parts) {
        C.col.insert(C.col.end(), q.col.begin(), q.col.end());
        C.val.insert(C.val.end(), q.val.begin(), q.val.end());
    }
    return C;
}

std::vector<double> diagonal(const Csr& A) {
    std::vector<double> d((size_t)A.n, 0.0);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
            if (A.col[k] == i) d[i] = A.val[k];
    return d;
}

int aggregate(const Csr& A, const std::vector<double>& d, double theta, std::vector<int>& agg) {
    const int n = A.n;
    agg.assign((size_t)n, -1);
    auto strong = [&](int i, int k) {
        const int j = A.col[k];
        return j != i && std::fabs(A.val[k]) >= theta * std::sqrt(std::fabs(d[i] * d[j]));
    };
    int na = 0;
    for (int i = 0; i < n; ++i) {  // pass 1
        if (agg[i] >= 0) continue;
        bool free_nbhd = true;
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1] && free_nbhd; ++k)
            if (strong(i, k) && agg[A.col[k]] >= 0) free_nbhd = false;
        if (!free_nbhd) continue;
        agg[i] = na;
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
            if (strong(i, k)) agg[A.col[k]] = na;
        ++na;
    }
    const std::vector<int> first(agg);
    for (int i = 0; i < n; ++i) {  // pass 2
        if (agg[i] >= 0) continue;
        int best = -1;
        double bw = -1.0;
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
            if (strong(i, k) && first[A.col[k]] >= 0 && std::fabs(A.val[k]) > bw) {
                bw = std::fabs(A.val[k]);
                best = A.col[k];
            }
        if (best >= 0) agg[i] = first[best];
    }
    for (int i = 0; i < n; ++i) {  // pass 3
        if (agg[i] >= 0) continue;
        agg[i] = na;
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
            if (strong(i, k) && agg[A.col[k]] < 0) agg[A.col[k]] = na;
        ++na;
    }
    return na;
}

double gershgorin(const Csr& A, const std::vector<double>& d) {
    double lam = 0.0;
    for (int i = 0; i < A.n; ++i) {
        double s = 0.0;
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) s += std::fabs(A.val[k]);
        lam = std::max(lam, s / d[i]);
    }
    return lam;
}

// P = (I - omega D^-1 A) P_t
Csr prolongator(const Csr& A, const std::vector<double>& d, const std::vector<int>& agg, int na, double omega) {
    Csr S = A;
    for (int i = 0; i < A.n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k)
            S.val[k] = (A.col[k] == i ? 1.0 : 0.0) - omega * A.val[k] / d[i];
    Csr Pt;
    Pt.n = A.n;
    Pt.m = na;
    Pt.ptr.resize((size_t)A.n + 1);
    for (int i = 0; i <= A.n; ++i) Pt.ptr[i] = i;
    Pt.col = agg;
    Pt.val.assign((size_t)A.n, 1.0);
    return multiply(S, Pt);
}

// inverse of a small SPD matrix through its Cholesky factor; false if not SPD
bool spd_inverse(const Csr& A, std::vector<double>& inv) {
    const int n = A.n;
    std::vector<double> L((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[(size_t)i + 1]; ++k) L[(size_t)i * n + A.col[k]] = A.val[k];
    for (int j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    // column c of A^-1: L L^T v = e_c; the columns are independent
    const bool ok = parallel_parts(n, 32, [&](int, int c0, int c1) {
        std::vector<double> e((size_t)n);
        for (int c = c0; c < c1; ++c) {
            for (int i = 0; i < n; ++i) {
                double s = i == c ? 1.0 : 0.0;
                for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * e[k];
                e[i] = s / L[(size_t)i * n + i];
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = e[i];
                for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * e[k];
                e[i] = s / L[(size_t)i * n + i];
            }
            for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = e[i];
        }
    });
    if (!ok) throw std::bad_alloc();
    return true;
}

// Level 0 as CSR from the device ELL layout: the diagonal plus every slot
// whose column is not the row itself (padding repeats the row), sorted.
int level0_from_device(const fvpcg_matrix* A, hipStream_t s, Csr& out) {
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n, W = m->W;
    std::vector<int> col((size_t)W * n);
    std::vector<double> val((size_t)W * n), d((size_t)n);
    FV_HIP(hipMemcpyAsync(col.data(), m->col, sizeof(int) * col.size(), hipMemcpyDeviceToHost, s));
    FV_HIP(hipMemcpyAsync(val.data(), A->val, sizeof(double) * val.size(), hipMemcpyDeviceToHost, s));
    FV_HIP(hipMemcpyAsync(d.data(), A->d, sizeof(double) * d.size(), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    out.n = out.m = n;
    out.ptr.assign((size_t)n + 1, 0);
    out.col.clear();
    out.val.clear();
    out.col.reserve((size_t)(W + 1) * n);
    out.val.reserve((size_t)(W + 1) * n);
    std::vector<std::pair<int, double>> row;
    for (int c = 0; c < n; ++c) {
        row.clear();
        row.emplace_back(c, d[c]);
        for (int k = 0; k < W; ++k) {
            const size_t o = (size_t)k * n + c;
            if (col[o] != c) row.emplace_back(col[o], val[o]);
        }
        std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        for (auto& e : row) {
            out.col.push_back(e.first);
            out.val.push_back(e.second);
        }
        out.ptr[(size_t)c + 1] = (int)out.col.size();
    }
    return FVPCG_OK;
}

bool symmetric(const Csr& A) {
    const Csr T = transpose(A);
    return T.ptr == A.ptr && T.col == A.col && T.val == A.val;
}

template <typename T>
int upload(T** dst, const std::vector<T>& src, const char* what, hipStream_t s) {
    int rc;
    if ((rc = dev_alloc(dst, std::max<size_t>(src.size(), 1), what))) return rc;
    if (!src.empty()) FV_HIP(hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
    return FVPCG_OK;
}

#pragma clang fp contract(on)

// ---------------------------------------------------------------- kernels

// Level 0, from x = 0: x = omega b / d and r = b - A x in one pass.  With
// x_j = omega b_j / d_j the product is omega (b_c + sum_j (a_cj / d_j) b_j),
// the column-scaled values' gather of b.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_amg_pre0(const CI* __restrict__ col, const double* __restrict__ val_cs,
                                                  const double* __restrict__ d, int n, Geom g, double w,
                                                  const double* __restrict__ b, double* __restrict__ x,
                                                  double* __restrict__ r, const DevState* st) {
    if (st->done) return;
    FV_ROWS(blk) {
        const double bc = b[c];
        const double t = row_gather<double, WT, CI>(col, val_cs, n, c, b, bc);
        x[c] = w * bc / d[c];
        r[c] = bc - w * t;
    }
}

// Level 0: y = x + omega (b - A x) / d; with DOT, also gamma' = (b, y) (b is
// the CG residual, y the preconditioned one): the first cycle sets gamma and
// beta = 0, later ones beta = gamma' / gamma.
template <int BS, int WT, typename CI, bool DOT>
__global__ __launch_bounds__(BS) void k_amg_post0(const CI* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ d, int n, Geom g, double w,
                                                   const double* __restrict__ b, const double* __restrict__ x,
                                                   double* __restrict__ y, int first, DevState* st,
                                                   double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double xc = x[c], dc = d[c], bc = b[c];
        const double ax = row_gather<double, WT, CI>(col, val, n, c, x, dc * xc);
        const double yc = xc + w * (bc - ax) / dc;
        y[c] = yc;
        if (DOT) acc[0] += bc * yc;
    }
    if (!DOT) return;
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        if (first) {
            st->beta = 0.0;
        } else {
            st->beta = t[0] / st->gamma;
        }
        st->gamma = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
        }
    }
}

// CSR levels, one row per thread.
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_pre(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val_cs, const double* __restrict__ d,
                                                      int n, double w, const double* __restrict__ b,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val_cs[k] * b[col[k]];
        const double bi = b[i];
        x[i] = w * bi / d[i];
        r[i] = bi - w * s;
    }
}

__global__ __launch_bounds__(kAmgCsrBs) void k_amg_post(const int* __restrict__ ptr, const int* __restrict__ col,
                                                       const double* __restrict__ val, const double* __restrict__ d,
                                                       int n, double w, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = x[i] + w * (b[i] - s) / d[i];
    }
}

// y = M v (restriction), or y += M v (prolongation, ADD)
template <bool ADD>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_csr_mv(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const double* __restrict__ val, int n,
                                                         const double* __restrict__ v, double* __restrict__ y,
                                                         const DevState* st) {
    if (st->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * v[col[k]];
        y[i] = ADD ? y[i] + s : s;
    }
}

// The same CSR operations with G lanes per row (G = 16: four rows per
// wavefront; G = 64: one), for operators whose rows are long (the coarse
// levels of smoothed aggregation hold tens to hundreds of entries per row):
// the lanes stride through the row, coalesced, and the row sum is an
// inclusive DPP scan within each 16-lane row of the wave (plus, for G = 64,
// the sum of the four row totals).  Rows are taken in wave-uniform blocks so
// every lane of a wave takes part in the scan.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    v += row_shr<1>(v);
    v += row_shr<2>(v);
    v += row_shr<4>(v);
    v += row_shr<8>(v);
    if (G == 64) return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
    return v;  // the group's sum in its last lane
}

#define AMG_GROUP_ROWS(G)                                                                  \
    const int lane_ = threadIdx.x & 63, sub_ = lane_ / (G), gl_ = lane_ % (G);              \
    const bool lead_ = (G) == 64 ? lane_ == 0 : gl_ == (G) - 1;                             \
    const int wave_ = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);                  \
    const int nwave_ = (int)((gridDim.x * blockDim.x) >> 6);                                \
    for (int base_ = wave_ * (64 / (G)); base_ < n; base_ += nwave_ * (64 / (G)))

// x = omega b / d; r = b - A x with A x = omega sum_j (a_ij / d_j) b_j
template <int G>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_pre_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                        const double* __restrict__ val_cs,
                                                        const double* __restrict__ d, int n, double w,
                                                        const double* __restrict__ b, double* __restrict__ x,
                                                        double* __restrict__ r, const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val_cs[k] * b[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) {
            const double bi = b[i];
            x[i] = w * bi / d[i];
            r[i] = bi - w * s;
        }
    }
}

template <int G>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_post_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                         const double* __restrict__ val, const double* __restrict__ d,
                                                         int n, double w, const double* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val[k] * x[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) y[i] = x[i] + w * (b[i] - s) / d[i];
    }
}

template <int G, bool ADD>
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_csr_mv_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                                           const double* __restrict__ val, int n,
                                                           const double* __restrict__ v, double* __restrict__ y,
                                                           const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(G) {
        const int i = base_ + sub_;
        double s = 0.0;
        if (i < n)
            for (int k = ptr[i] + gl_; k < ptr[i + 1]; k += G) s += val[k] * v[col[k]];
        s = group_sum<G>(s);
        if (i < n && lead_) y[i] = ADD ? y[i] + s : s;
    }
}

// last level: y = A^-1 b with the dense inverse, one wavefront per row
__global__ __launch_bounds__(kAmgCsrBs) void k_amg_coarse_w(const double* __restrict__ inv, int n,
                                                           const double* __restrict__ b, double* __restrict__ y,
                                                           const DevState* st) {
    if (st->done) return;
    AMG_GROUP_ROWS(64) {
        const int i = base_;
        double s = 0.0;
        for (int k = gl_; k < n; k += 64) s += inv[(size_t)i * n + k] * b[k];
        s = group_sum<64>(s);
        if (lead_) y[i] = s;
    }
}

// gamma' = (r, z) when the hierarchy has a single level (no post-smoothing)
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_dot(const double* __restrict__ r, const double* __restrict__ z, int n,
                                                 Geom g, int first, DevState* st, double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) { acc[0] += r[c] * z[c]; }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->beta = first ? 0.0 : t[0] / st->gamma;
        st->gamma = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
        }
    }
}

// r = b - A x; (b, b), (r, r); stopping test before the first iteration.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_init(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  double* __restrict__ r, DevState* st, double* partials) {
    double acc[2] = {0.0, 0.0};
    FV_ROWS(blk) {
        const double bc = b[c];
        const double rc = bc - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        r[c] = rc;
        acc[0] += bc * bc;
        acc[1] += rc * rc;
    }
    double t[2];
    if (device_reduce<BS, 2>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->iter = 0;
        st->bnorm = sqrt(t[0]);
        st->rho = t[1];
        st->r0norm = sqrt(t[1]);
        if (t[0] == 0.0) {
            st->zero_b = 1;
            st->done = 1;
            st->status = FVPCG_OK;
            return;
        }
        st->tol_abs *= st->bnorm;
        if (st->r0norm <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (st->maxit <= 0) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// p = z (first) or p = z + beta p
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_p(const double* __restrict__ z, double* __restrict__ p, int n, Geom g,
                                               int first, const DevState* st) {
    if (st->done) return;
    const double beta = st->beta;
    FV_ROWS(blk) { p[c] = first ? z[c] : z[c] + beta * p[c]; }
}

// q = A p; delta = (p, q); alpha = gamma / delta.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_spmv(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ p, double* __restrict__ q, DevState* st,
                                                  double* partials) {
    if (st->done) return;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double pc = p[c];
        const double qc = row_gather<double, WT, CI>(col, val, n, c, p, d[c] * pc);
        q[c] = qc;
        acc[0] += pc * qc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        st->delta = t[0];
        if (!(t[0] > 0.0) || !isfinite(t[0])) {
            st->done = 1;
            st->status = FVPCG_BREAKDOWN;
            return;
        }
        st->alpha = st->gamma / t[0];
    }
}

// x += alpha p; r -= alpha q; rho = (r, r); iteration count and stopping test.
template <int BS>
__global__ __launch_bounds__(BS) void k_apcg_xr(double* __restrict__ x, const double* __restrict__ p,
                                                double* __restrict__ r, const double* __restrict__ q, int n, Geom g,
                                                DevState* st, double* partials) {
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        x[c] += alpha * p[c];
        const double rc = r[c] - alpha * q[c];
        r[c] = rc;
        acc[0] += rc * rc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) {
        const int it = st->iter + 1;
        st->iter = it;
        st->rho = t[0];
        if (sqrt(t[0]) <= st->tol_abs) {
            st->done = 1;
            st->status = FVPCG_OK;
        } else if (it >= st->maxit) {
            st->done = 1;
            st->status = FVPCG_NOT_CONVERGED;
        }
    }
}

// Pipelined CG (Ghysels and Vanroose, Section 4.1) with the AMG cycle as
// M^-1, literal recurrences: w0 = A u0 and the first reduction.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apipe_init_w(const CI* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ d, int n, Geom g,
                                                     const double* __restrict__ r, const double* __restrict__ u,
                                                     double* __restrict__ w, DevState* st, double* partials) {
    if (st->done) return;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const double uc = u[c], rc = r[c];
        const double wc = row_gather<double, WT, CI>(col, val, n, c, u, d[c] * uc);
        w[c] = wc;
        acc[0] += rc * uc;
        acc[1] += wc * uc;
        acc[2] += rc * rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], true);
}

// One iteration, m = M^-1 w already formed by a cycle:
//   n = A m; z = n + beta z; q = m + beta q; s = w + beta s; p = u + beta p;
//   x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z;
// and the reduction (r, u), (w, u), (r, r) of the new iterate.
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apipe_iter(const CI* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ d, int n, Geom g,
                                                   const double* __restrict__ m, double* __restrict__ w,
                                                   double* __restrict__ z, double* __restrict__ q,
                                                   double* __restrict__ s, double* __restrict__ p,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ u, DevState* st, double* partials) {
    if (st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    double acc[3] = {0.0, 0.0, 0.0};
    FV_ROWS(blk) {
        const double mc = m[c];
        const double nv = row_gather<double, WT, CI>(col, val, n, c, m, d[c] * mc);
        const double zc = nv + beta * z[c];
        const double qc = mc + beta * q[c];
        const double wc = w[c];
        const double sc = wc + beta * s[c];
        double uc = u[c];
        const double pc = uc + beta * p[c];
        z[c] = zc;
        q[c] = qc;
        s[c] = sc;
        p[c] = pc;
        x[c] += alpha * pc;
        const double rc = r[c] - alpha * sc;
        r[c] = rc;
        uc -= alpha * qc;
        u[c] = uc;
        const double wn = wc - alpha * zc;
        w[c] = wn;
        acc[0] += rc * uc;
        acc[1] += wn * uc;
        acc[2] += rc * rc;
    }
    double t[3];
    if (device_reduce<BS, 3>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0)
        pipe_scalars(st, t[0], t[1], t[2], false);
}

// zero the pipelined recurrences z, q, s, p before the first iteration
template <int BS>
__global__ __launch_bounds__(BS) void k_apipe_clear(double* __restrict__ z, double* __restrict__ q,
                                                    double* __restrict__ s, double* __restrict__ p, int n, Geom g) {
    FV_ROWS(blk) {
        z[c] = 0.0;
        q[c] = 0.0;
        s[c] = 0.0;
        p[c] = 0.0;
    }
}

// ||b - A x||^2 at exit
template <int BS, int WT, typename CI>
__global__ __launch_bounds__(BS) void k_apcg_true(const CI* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ d, int n, Geom g,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  DevState* st, double* partials) {
    double acc[1] = {0.0};
    FV_ROWS(blk) {
        const double rc = b[c] - row_gather<double, WT, CI>(col, val, n, c, x, d[c] * x[c]);
        acc[0] += rc * rc;
    }
    double t[1];
    if (device_reduce<BS, 1>(acc, partials, &st->ticket, blk, g.grid, t) && threadIdx.x == 0) st->true_rr = t[0];
}

int csr_grid(int n) { return std::max(1, std::min((n + kAmgCsrBs - 1) / kAmgCsrBs, 4096)); }
// blocks for G lanes per row: 64 / G rows per wavefront, 4 wavefronts per block
int group_grid(int n, int G) {
    const int rows_per_block = (kAmgCsrBs / 64) * (64 / G);
    return std::max(1, std::min((n + rows_per_block - 1) / rows_per_block, 8192));
}
// lanes per row from the operator's mean row length (measured at 7M cells:
// 44-entry rows run fastest with 16 lanes, hundreds with 64)
int lanes_for(size_t nnz, int rows) {
    const double avg = (double)nnz / (double)std::max(rows, 1);
    return avg <= 6.0 ? 1 : (avg <= 48.0 ? 16 : 64);
}

void launch_pre(const AmgLevel& v, const double* b, const DevState* st, hipStream_t s) {
    if (v.ga == 1)
        hipLaunchKernelGGL(k_amg_pre, dim3(csr_grid(v.n)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col, v.a_val_cs, v.d,
                           v.n, v.omega, b, v.x, v.r, st);
    else if (v.ga == 16)
        hipLaunchKernelGGL((k_amg_pre_g<16>), dim3(group_grid(v.n, 16)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val_cs, v.d, v.n, v.omega, b, v.x, v.r, st);
    else
        hipLaunchKernelGGL((k_amg_pre_g<64>), dim3(group_grid(v.n, 64)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val_cs, v.d, v.n, v.omega, b, v.x, v.r, st);
}

void launch_post(const AmgLevel& v, const DevState* st, hipStream_t s) {
    if (v.ga == 1)
        hipLaunchKernelGGL(k_amg_post, dim3(csr_grid(v.n)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col, v.a_val, v.d,
                           v.n, v.omega, v.b, v.x, v.y, st);
    else if (v.ga == 16)
        hipLaunchKernelGGL((k_amg_post_g<16>), dim3(group_grid(v.n, 16)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val, v.d, v.n, v.omega, v.b, v.x, v.y, st);
    else
        hipLaunchKernelGGL((k_amg_post_g<64>), dim3(group_grid(v.n, 64)), dim3(kAmgCsrBs), 0, s, v.a_ptr, v.a_col,
                           v.a_val, v.d, v.n, v.omega, v.b, v.x, v.y, st);
}

template <bool ADD>
void launch_mv(const int* ptr, const int* col, const double* val, int rows, int G, const double* in, double* out,
               const DevState* st, hipStream_t s) {
    if (G == 1)
        hipLaunchKernelGGL((k_amg_csr_mv<ADD>), dim3(csr_grid(rows)), dim3(kAmgCsrBs), 0, s, ptr, col, val, rows, in,
                           out, st);
    else if (G == 16)
        hipLaunchKernelGGL((k_amg_csr_mv_g<16, ADD>), dim3(group_grid(rows, 16)), dim3(kAmgCsrBs), 0, s, ptr, col,
                           val, rows, in, out, st);
    else
        hipLaunchKernelGGL((k_amg_csr_mv_g<64, ADD>), dim3(group_grid(rows, 64)), dim3(kAmgCsrBs), 0, s, ptr, col,
                           val, rows, in, out, st);
}

// Enqueue one cycle y0 = M^-1 b0 on `s`; kernels skip once st->done.
int enqueue_cycle(const fvpcg_amg* h, const double* b0, double* y0, bool dot, bool first, DevState* st,
                  hipStream_t s) {
    const fvpcg_matrix* A = h->mat;
    const fvpcg_mesh* m = A->mesh;
    const int n0 = m->n;
    const Geom g0 = geom_for(n0, kAmgBs);
    const int L = h->nlev;
    if (L == 1) {
        hipLaunchKernelGGL(k_amg_coarse_w, dim3(group_grid(n0, 64)), dim3(kAmgCsrBs), 0, s, h->cinv, n0, b0, y0, st);
        if (dot)
            hipLaunchKernelGGL((k_apcg_dot<kAmgBs>), dim3(g0.grid), dim3(kAmgBs), 0, s, b0, y0, n0, g0, first ? 1 : 0,
                               st, h->partials);
        FV_LAUNCHED();
        return FVPCG_OK;
    }
    for (int l = 0; l + 1 < L; ++l) {
        const AmgLevel& v = h->lev[l];
        const double* b = l == 0 ? b0 : v.b;
        if (l == 0) {
            FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_pre0<kAmgBs, W_, CI_>), dim3(g0.grid), dim3(kAmgBs), 0, s, cols_,
                                            A->val_cs, A->d, n0, g0, v.omega, b, v.x, v.r, st));
        } else {
            launch_pre(v, b, st, s);
        }
        launch_mv<false>(v.r_ptr, v.r_col, v.r_val, v.nc, v.gr, v.r, h->lev[l + 1].b, st, s);
    }
    const AmgLevel& last = h->lev[L - 1];
    hipLaunchKernelGGL(k_amg_coarse_w, dim3(group_grid(last.n, 64)), dim3(kAmgCsrBs), 0, s, h->cinv, last.n, last.b,
                       last.y, st);
    for (int l = L - 2; l >= 0; --l) {
        const AmgLevel& v = h->lev[l];
        launch_mv<true>(v.p_ptr, v.p_col, v.p_val, v.n, v.gp, h->lev[l + 1].y, v.x, st, s);
        if (l == 0) {
            if (dot) {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_post0<kAmgBs, W_, CI_, true>), dim3(g0.grid), dim3(kAmgBs), 0,
                                                s, cols_, A->val, A->d, n0, g0, v.omega, b0, v.x, y0, first ? 1 : 0,
                                                st, h->partials));
            } else {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_amg_post0<kAmgBs, W_, CI_, false>), dim3(g0.grid), dim3(kAmgBs),
                                                0, s, cols_, A->val, A->d, n0, g0, v.omega, b0, v.x, y0, 0, st,
                                                h->partials));
            }
        } else {
            launch_post(v, st, s);
        }
    }
    FV_LAUNCHED();
    return FVPCG_OK;
}

int state_put(fvpcg_amg* h, double tol, int maxit, hipStream_t s) {
    DevState* hs = &h->hst[1];
    *hs = DevState();
    hs->tol_abs = tol;
    hs->maxit = maxit;
    hs->status = FVPCG_NOT_CONVERGED;
    FV_HIP(hipMemcpyAsync(h->st, hs, sizeof(DevState), hipMemcpyHostToDevice, s));
    return FVPCG_OK;
}

int state_get(fvpcg_amg* h, DevState* out, hipStream_t s) {
    FV_HIP(hipMemcpyAsync(&h->hst[0], h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    *out = h->hst[0];
    return FVPCG_OK;
}

}  // namespace

void amg_free(fvpcg_amg* h) {
    if (!h) return;
    for (AmgLevel& v : h->lev) {
        dev_free(v.a_ptr);
        dev_free(v.a_col);
        dev_free(v.a_val);
        dev_free(v.a_val_cs);
        dev_free(v.d);
        dev_free(v.p_ptr);
        dev_free(v.p_col);
        dev_free(v.p_val);
        dev_free(v.r_ptr);
        dev_free(v.r_col);
        dev_free(v.r_val);
        dev_free(v.b);
        dev_free(v.x);
        dev_free(v.r);
        dev_free(v.y);
    }
    dev_free(h->cinv);
    dev_free(h->r);
    dev_free(h->z);
    dev_free(h->p);
    dev_free(h->q);
    dev_free(h->u);
    dev_free(h->w);
    dev_free(h->m);
    dev_free(h->s);
    dev_free(h->st);
    dev_free(h->partials);
    if (h->hst) (void)hipHostFree(h->hst);
    hipEvent_t* evs[] = {&h->t_begin, &h->t_end, &h->t_it0, &h->t_it1};
    for (hipEvent_t* e : evs)
        if (*e) (void)hipEventDestroy(*e);
    delete h;
}

int amg_build(fvpcg_amg* h, const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, hipStream_t s);

int amg_create(const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, hipStream_t s,
               fvpcg_amg** out) {
    fvpcg_amg* h = new (std::nothrow) fvpcg_amg();
    if (!h) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    h->mat = A;
    int rc;
    try {
        rc = amg_build(h, A, theta, max_levels, coarse_size, s);
    } catch (const std::bad_alloc&) {
        rc = set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed during the AMG setup");
    }
    if (rc) {
        amg_free(h);
        return rc;
    }
    *out = h;
    return FVPCG_OK;
}

// The hierarchy into h (freed by the caller on failure).
int amg_build(fvpcg_amg* h, const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, hipStream_t s) {
    auto fail = [](int rc) { return rc; };
    int rc;
    Csr cur;
    if ((rc = level0_from_device(A, s, cur))) return fail(rc);
    if (!A->sym && !symmetric(cur))
        return fail(set_error(FVPCG_UNSUPPORTED, "AMG needs a symmetric matrix (lower == upper on every face)"));
    max_levels = std::max(1, std::min(max_levels, kAmgMaxLevels));
    double th = theta;
    int l = 0;
    for (;;) {
        AmgLevel& v = h->lev[l];
        const std::vector<double> d = diagonal(cur);
        v.n = cur.n;
        v.nnz = (long long)cur.col.size();
        v.omega = 4.0 / (3.0 * gershgorin(cur, d));
        v.ga = lanes_for(cur.col.size(), cur.n);
        if (l > 0) {
            std::vector<double> cs(cur.val.size());
            for (size_t k = 0; k < cs.size(); ++k) cs[k] = cur.val[k] / d[cur.col[k]];
            if ((rc = upload(&v.a_ptr, cur.ptr, "AMG level rows", s)) || (rc = upload(&v.a_col, cur.col, "AMG level columns", s)) ||
                (rc = upload(&v.a_val, cur.val, "AMG level values", s)) || (rc = upload(&v.d, d, "AMG level diagonal", s)) ||
                (rc = upload(&v.a_val_cs, cs, "AMG level scaled values", s)))
                return fail(rc);
            FV_HIP(hipStreamSynchronize(s));  // cs goes out of scope
        }
        if ((rc = dev_alloc(&v.b, (size_t)std::max(v.n, 1), "AMG work")) ||
            (rc = dev_alloc(&v.x, (size_t)std::max(v.n, 1), "AMG work")) ||
            (rc = dev_alloc(&v.r, (size_t)std::max(v.n, 1), "AMG work")) ||
            (rc = dev_alloc(&v.y, (size_t)std::max(v.n, 1), "AMG work")))
            return fail(rc);
        if (cur.n <= coarse_size || l + 1 == max_levels) break;
        std::vector<int> agg;
        const int na = aggregate(cur, d, th, agg);
        if ((double)na > 0.6 * (double)cur.n) break;
        const Csr P = prolongator(cur, d, agg, na, v.omega);
        const Csr R = transpose(P);
        Csr next = multiply(R, multiply(cur, P));
        v.nc = na;
        v.agg = std::move(agg);
        v.gp = lanes_for(P.col.size(), P.n);
        v.gr = lanes_for(R.col.size(), R.n);
        if ((rc = upload(&v.p_ptr, P.ptr, "AMG prolongator", s)) || (rc = upload(&v.p_col, P.col, "AMG prolongator", s)) ||
            (rc = upload(&v.p_val, P.val, "AMG prolongator", s)) || (rc = upload(&v.r_ptr, R.ptr, "AMG restriction", s)) ||
            (rc = upload(&v.r_col, R.col, "AMG restriction", s)) || (rc = upload(&v.r_val, R.val, "AMG restriction", s)))
            return fail(rc);
        FV_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
        cur = std::move(next);
        th *= 0.5;
        ++l;
    }
    h->nlev = l + 1;
    h->nlast = cur.n;
    if (cur.n > kAmgMaxCoarse)
        return fail(set_error(FVPCG_UNSUPPORTED, "AMG: last level has %d unknowns (at most %d are solved exactly)",
                              cur.n, kAmgMaxCoarse));
    std::vector<double> inv;
    if (!spd_inverse(cur, inv))
        return fail(set_error(FVPCG_BREAKDOWN, "AMG: the last level is not positive definite"));
    if ((rc = upload(&h->cinv, inv, "AMG coarse inverse", s))) return fail(rc);
    const size_t n0 = (size_t)std::max(A->mesh->n, 1);
    if ((rc = dev_alloc(&h->r, n0, "AMG-PCG vectors")) || (rc = dev_alloc(&h->z, n0, "AMG-PCG vectors")) ||
        (rc = dev_alloc(&h->p, n0, "AMG-PCG vectors")) || (rc = dev_alloc(&h->q, n0, "AMG-PCG vectors")) ||
        (rc = dev_alloc(&h->st, 1, "AMG-PCG state")) || (rc = dev_alloc(&h->partials, (size_t)4 * kMaxGrid, "partials")))
        return fail(rc);
    if (hipHostMalloc((void**)&h->hst, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        h->hst = nullptr;
        return fail(set_error(FVPCG_OUT_OF_MEMORY, "pinned allocation failed"));
    }
    FV_HIP(hipMemsetAsync(h->st, 0, sizeof(DevState), s));
    hipEvent_t* evs[] = {&h->t_begin, &h->t_end, &h->t_it0, &h->t_it1};
    for (hipEvent_t* e : evs) FV_HIP(hipEventCreate(e));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

int amg_levels(const fvpcg_amg* h) { return h->nlev; }
int amg_level_n(const fvpcg_amg* h, int l) { return h->lev[l].n; }
long long amg_level_nnz(const fvpcg_amg* h, int l) { return h->lev[l].nnz; }
const int* amg_level_agg(const fvpcg_amg* h, int l) { return h->lev[l].agg.empty() ? nullptr : h->lev[l].agg.data(); }

// z = M^-1 r (one cycle)
int amg_apply(const fvpcg_amg* ch, const double* r, double* z, hipStream_t s) {
    fvpcg_amg* h = const_cast<fvpcg_amg*>(ch);
    int rc;
    if ((rc = state_put(h, 0.0, 1, s))) return rc;
    if ((rc = enqueue_cycle(h, r, z, false, false, h->st, s))) return rc;
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

// Standard PCG (Section 2) with one AMG cycle as M^-1.
int solve_amg(const fvpcg_amg* ch, const double* b, double* x, double tol, int maxit, int method, hipStream_t s,
              fvpcg_stats* stats) {
    fvpcg_amg* h = const_cast<fvpcg_amg*>(ch);
    const fvpcg_matrix* A = h->mat;
    const fvpcg_mesh* m = A->mesh;
    const int n = m->n;
    const Geom g = geom_for(n, kAmgBs);
    DevState* st = h->st;
    int rc;
    FV_HIP(hipEventRecord(h->t_begin, s));
    if ((rc = state_put(h, tol, maxit, s))) return rc;
    FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_init<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, h->r, st, h->partials));
    FV_LAUNCHED();
    DevState hs;
    if ((rc = state_get(h, &hs, s))) return rc;
    FV_HIP(hipEventRecord(h->t_it0, s));
    const bool pipe = method == FVPCG_PIPECG;
    if (pipe && !h->u) {
        const size_t nn = (size_t)std::max(n, 1);
        if ((rc = dev_alloc(&h->u, nn, "AMG pipelined vectors")) || (rc = dev_alloc(&h->w, nn, "AMG pipelined vectors")) ||
            (rc = dev_alloc(&h->m, nn, "AMG pipelined vectors")) || (rc = dev_alloc(&h->s, nn, "AMG pipelined vectors")))
            return rc;
    }
    if (!hs.done && pipe) {
        // u = M^-1 r; z = q = s = p = 0; w = A u and the first reduction
        if ((rc = enqueue_cycle(h, h->r, h->u, false, false, st, s))) return rc;
        hipLaunchKernelGGL((k_apipe_clear<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->q, h->s, h->p, n, g);
        FV_LAYOUT(m, hipLaunchKernelGGL((k_apipe_init_w<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_,
                                        A->val, A->d, n, g, h->r, h->u, h->w, st, h->partials));
        FV_LAUNCHED();
        int launched = 0, chunk = 1;
        while (launched < maxit) {
            const int cnt = std::min(chunk, maxit - launched);
            for (int k = 0; k < cnt; ++k) {
                if ((rc = enqueue_cycle(h, h->w, h->m, false, false, st, s))) return rc;
                FV_LAYOUT(m, hipLaunchKernelGGL((k_apipe_iter<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s,
                                                cols_, A->val, A->d, n, g, h->m, h->w, h->z, h->q, h->s, h->p, x,
                                                h->r, h->u, st, h->partials));
                FV_LAUNCHED();
            }
            launched += cnt;
            if ((rc = state_get(h, &hs, s))) return rc;
            if (hs.done) break;
            chunk = std::min(chunk * 2, 16);
        }
    } else if (!hs.done) {
        // z = M^-1 r, gamma = (r, z), p = z
        if ((rc = enqueue_cycle(h, h->r, h->z, true, true, st, s))) return rc;
        hipLaunchKernelGGL((k_apcg_p<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->p, n, g, 1, st);
        FV_LAUNCHED();
        int launched = 0, chunk = 1;
        while (launched < maxit) {
            const int cnt = std::min(chunk, maxit - launched);
            for (int k = 0; k < cnt; ++k) {
                FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_spmv<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s,
                                                cols_, A->val, A->d, n, g, h->p, h->q, st, h->partials));
                hipLaunchKernelGGL((k_apcg_xr<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, x, h->p, h->r, h->q, n, g,
                                   st, h->partials);
                if ((rc = enqueue_cycle(h, h->r, h->z, true, false, st, s))) return rc;
                hipLaunchKernelGGL((k_apcg_p<kAmgBs>), dim3(g.grid), dim3(kAmgBs), 0, s, h->z, h->p, n, g, 0, st);
                FV_LAUNCHED();
            }
            launched += cnt;
            if ((rc = state_get(h, &hs, s))) return rc;
            if (hs.done) break;
            chunk = std::min(chunk * 2, 16);
        }
    }
    FV_HIP(hipEventRecord(h->t_it1, s));
    if (hs.zero_b) FV_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, s));
    FV_LAYOUT(m, hipLaunchKernelGGL((k_apcg_true<kAmgBs, W_, CI_>), dim3(g.grid), dim3(kAmgBs), 0, s, cols_, A->val,
                                    A->d, n, g, b, x, st, h->partials));
    FV_LAUNCHED();
    FV_HIP(hipEventRecord(h->t_end, s));
    if ((rc = state_get(h, &hs, s))) return rc;
    if (stats) {
        stats->iters = hs.iter;
        stats->outer_iters = 0;
        stats->status = hs.status;
        stats->b_norm = hs.bnorm;
        stats->r0_norm = hs.r0norm;
        stats->rel_res = hs.bnorm > 0 ? sqrt(hs.rho) / hs.bnorm : 0.0;
        stats->true_rel_res = hs.bnorm > 0 ? sqrt(hs.true_rr) / hs.bnorm : 0.0;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, h->t_begin, h->t_end);
        stats->device_ms = ms;
        (void)hipEventElapsedTime(&ms, h->t_it0, h->t_it1);
        stats->iter_ms = ms;
    }
    return hs.status;
}

}  // namespace fvpcg
