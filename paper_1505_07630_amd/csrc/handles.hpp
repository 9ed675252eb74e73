// Handle layouts (opaque to callers of fvpcg.h).
#pragma once

#include "common.hpp"

namespace fvpcg {

// Per-matrix solve workspace, allocated on first use of each solver kind.
struct Work {
    int n = 0;
    Geom geom{1, 64};
    // FP64 vectors
    double* r = nullptr;
    double* p = nullptr;
    double* q = nullptr;
    double* z = nullptr;
    double* s = nullptr;
    double* w[2] = {nullptr, nullptr};
    double* u = nullptr;
    double* qq = nullptr;   // literal pipelined q
    double* lam = nullptr;  // adjoint solution when grad_b is not requested
    // FP32 vectors (mixed solver)
    float* r32 = nullptr;
    float* r32b = nullptr;  // FP32 right-hand side of the inner solve
    float* w32[2] = {nullptr, nullptr};
    float* z32 = nullptr;
    float* s32 = nullptr;
    float* p32 = nullptr;
    float* c32 = nullptr;
    // reductions and scalars
    double* partials = nullptr;  // [4][grid]
    DevState* st = nullptr;      // device: [0] outer/main, [1] inner (mixed)
    DevState* hst = nullptr;     // pinned host mirror slots [4]
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t_begin = nullptr, t_end = nullptr, t_it0 = nullptr, t_it1 = nullptr;
    bool have_cg = false, have_pipe = false, have_lit = false, have_mixed = false;
};

int work_init(Work& w, int n);
void work_free(Work& w);
int work_need_cg(Work& w);
int work_need_pipe(Work& w, bool literal);
int work_need_mixed(Work& w);

}  // namespace fvpcg

namespace fvpcg {
struct BiWork;  // BiCGSTAB workspace (bicgstab.hip)
}

struct fvpcg_mesh {
    int device = 0;
    int n = 0;
    int F = 0;
    int maxdeg = 0;     // largest row degree
    int bandwidth = -1; // largest |column - row| (-1: not measured)
    int W = 0;       // slots per row: maxdeg rounded up to a kernel width
    int WT = 0;      // kernel specialisation width (== W)
    int* owner = nullptr;
    int* nb = nullptr;
    int* col = nullptr;  // [W][n] column of each slot; padding holds the row itself
    int16_t* col16 = nullptr;  // [W][n] column - row, when every offset fits in int16 (else NULL)
    int* ref = nullptr;  // [W][n] 2*face + (0 upper | 1 lower); -1 for padding
    fvpcg::Geom geom{1, 64};
};

struct fvpcg_matrix {
    const fvpcg_mesh* mesh = nullptr;
    bool sym = false;      // created with lower == NULL
    bool fp32 = false;
    bool diag_ok = false;  // every diagonal entry finite and > 0
    bool vals_sym = true;  // lower == upper on every face (always, when created with lower == NULL)
    uint64_t generation = 0;  // bumped by every coefficient refresh
    double* d = nullptr;       // [n]
    double* val = nullptr;     // [W][n] A[c][col]
    double* val_cs = nullptr;  // [W][n] A[c][col] / d[col] (Jacobi-folded products)
    float* d32 = nullptr;
    float* val32 = nullptr;     // [W][n] FP32 A[c][col]
    float* val32_cs = nullptr;  // [W][n] FP32 A[c][col] / d[col]
    fvpcg::Work* work = nullptr;
    mutable fvpcg::BiWork* bi = nullptr;  // allocated by the first BiCGSTAB solve
};

namespace fvpcg {
// Kernel-width specialisations available for a mesh of row degree W.
inline int pick_wt(int W) {
    if (W <= 4) return 4;
    if (W <= 6) return 6;
    if (W <= 8) return 8;
    if (W <= 16) return 16;
    return 32;
}
}  // namespace fvpcg
