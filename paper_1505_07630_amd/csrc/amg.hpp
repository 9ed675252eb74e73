// Smoothed-aggregation AMG: handle layout shared by the device setup
// (amg_setup.hip) and the cycle and solvers (amg.hip).
//
// The paper compares its Jacobi-preconditioned CG and pipelined CG with
// aggregation-AMG preconditioned versions (Section 5, Fig. pcgs1 and Table
// pcgs2) and names the method's parts: a V-cycle of aggregation-based AMG,
// aggregates from the parallel distance-2 maximal-independent-set method,
// weighted Jacobi with omega = 4/3 as the smoother.  Built as:
//   strength    j ~ i iff j != i, a_ij != 0 and
//               |a_ij| >= theta_l sqrt(|a_ii a_jj|), theta_l = theta / 2^l;
//   aggregates  roots: a distance-2 maximal independent set of the strength
//               graph, found in rounds (an undecided unknown becomes a root
//               when its priority is the largest among the undecided within
//               two strong steps and no root is that close; it drops out when
//               a root is); priorities from SplitMix64 on the counter
//               (level, unknown); aggregate a = the a-th root in index order;
//               round 1: each root's strong neighbours join it; round 2: the
//               rest join the round-1 aggregate of their strong neighbour with
//               the largest |a_ij| (ties: the lowest index);
//   prolongator P = (I - omega D^-1 A) P_t, P_t the aggregate indicator,
//               omega = (4/3) / rho, rho the Gershgorin bound
//               max_i sum_j |a_ij| / a_ii of D^-1 A (the 4/3 taken for the
//               operator scaled to spectral radius 1);
//   coarse      A_c = R (A P) with R = P^T; levels until n <= coarse_size, the
//               level limit, or an aggregation keeping more than 60% of the
//               unknowns; the last level (at most kAmgMaxCoarse unknowns)
//               solved exactly through its inverse;
//   cycle       V(1,1): x = omega D^-1 b; r = b - A x; x += P V(R r);
//               y = x + omega D^-1 (b - A x).
#pragma once

#include <cstdint>

#include "handles.hpp"

namespace fvpcg {

constexpr int kAmgMaxLevels = 16;
constexpr int kAmgMaxCoarse = 2048;  // largest exactly-solved last level
constexpr int kAmgBs = 512;          // level-0 and PCG kernels
constexpr int kAmgCsrBs = 256;       // CSR levels
constexpr uint64_t kStaleGeneration = ~0ull;  // a hierarchy no matrix generation matches (failed refresh)

// The sparse-product kernel chosen for one Galerkin product at setup, kept
// so that a numeric refresh runs the same kernel without sizing it again.
enum ProdMode { kProdDense = 0, kProdTiled = 1, kProdMergeLds = 2, kProdMerge = 3, kProdShort = 4, kProdMergeLds32 = 5 };
struct ProdPlan {
    int mode = kProdMerge;
    int lcap = 0, per_wg = 0;  // heap entries per row and rows per workgroup of the LDS merge
};

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
    long long p_nnz = 0;  // stored entries of P (and of R)
    double *b = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;  // work
    int ga = 1, gp = 1, gr = 1;  // lanes per row for A, P, R (1, 16 or 64)
    int* agg = nullptr;          // device: aggregate of every row (levels with a coarser one)
    // kept for the numeric refresh (levels with a coarser one)
    int *ap_ptr = nullptr, *ap_col = nullptr;  // A P
    double* ap_val = nullptr;
    long long ap_nnz = 0;
    long long *p_off = nullptr, *ap_off = nullptr, *c_off = nullptr;  // row offsets of P, A P, A_c (64-bit)
    ProdPlan plan_p, plan_ap, plan_c;  // kernels of P = S P_t, A P and A_c = R (A P)
};

// lanes per row from the operator's mean row length (measured at 7M cells:
// 44-entry rows run fastest with 16 lanes, hundreds with 64)
inline int lanes_for(size_t nnz, int rows) {
    const double avg = (double)nnz / (double)(rows > 1 ? rows : 1);
    return avg <= 6.0 ? 1 : (avg <= 48.0 ? 16 : 64);
}

// The hierarchy into h (freed by the caller on failure).
int amg_build(fvpcg_amg* h, const fvpcg_matrix* A, double theta, int max_levels, int coarse_size, uint64_t seed,
              hipStream_t s);
// The same hierarchy for the matrix's current coefficients with the
// aggregates, levels and sparsity patterns kept (see fvpcg_amg_refresh).
int amg_refresh(fvpcg_amg* h, hipStream_t s);

}  // namespace fvpcg

struct fvpcg_amg {
    const fvpcg_matrix* mat = nullptr;
    uint64_t generation = 0;  // the matrix's coefficient generation at setup
    int nlev = 0;
    fvpcg::AmgLevel lev[fvpcg::kAmgMaxLevels];
    double* cinv = nullptr;  // inverse of the last level, row-major
    int *a0_ptr = nullptr, *a0_col = nullptr;  // level 0 as CSR, kept for the numeric refresh
    double* a0_val = nullptr;
    long long a0_nnz = 0;
    int nlast = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // PCG vectors
    double *u = nullptr, *w = nullptr, *m = nullptr, *s = nullptr;  // pipelined CG, allocated on first use
    fvpcg::DevState* st = nullptr;
    fvpcg::DevState* hst = nullptr;  // pinned [2]
    double* partials = nullptr;
    hipEvent_t t_begin = nullptr, t_end = nullptr, t_it0 = nullptr, t_it1 = nullptr;
};
