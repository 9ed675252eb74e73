// Mesh and matrix setup: LDU ingest, validation, and the device layout.
//
// The paper stores the matrix in CSR on the GPU (Section 4.1) and suggests
// replacing the lduMatrix's scattered face access with small contiguous
// blocks (Section 5).  Here the LDU arrays are turned, on the device, into a
// slot-major ELL pattern: slot k of row c holds the k-th off-diagonal entry
// of that row in ascending column order (row c owns face f -> column
// neighbour[f], coefficient upper[f]; row c is neighbour of face f -> column
// owner[f], coefficient lower[f]), padded with (column c, value 0).  Element
// (k, c) lives at k*n + c, so the 64 lanes of a wave read 64 consecutive
// entries of a slot: every matrix stream is coalesced.
#include <cstdlib>

#include "handles.hpp"

namespace fvpcg {

namespace {

__global__ void k_validate(const int* __restrict__ owner, const int* __restrict__ nb, int F, int n,
                           unsigned* flags) {
    unsigned bad = 0;
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) {
        int o = owner[f], m = nb[f];
        if (o < 0 || m >= n || o >= m) bad |= 1u;
        if (f + 1 < F) {
            int o2 = owner[f + 1], m2 = nb[f + 1];
            if (!(o < o2 || (o == o2 && m < m2))) bad |= 2u;
        }
    }
    if (bad) atomicOr(flags, bad);
}

__global__ void k_degree(const int* __restrict__ owner, const int* __restrict__ nb, int F, int* deg) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) {
        atomicAdd(&deg[owner[f]], 1);
        atomicAdd(&deg[nb[f]], 1);
    }
}

__global__ void k_maxdeg(const int* __restrict__ deg, int n, int* out) {
    int m = 0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) m = max(m, deg[c]);
    atomicMax(out, m);
}

__global__ void k_fill(const int* __restrict__ owner, const int* __restrict__ nb, int F, int n, int* fill,
                       int* col, int* ref) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x) {
        int o = owner[f], m = nb[f];
        size_t so = (size_t)atomicAdd(&fill[o], 1) * n + o;
        col[so] = m;
        ref[so] = 2 * f;
        size_t sn = (size_t)atomicAdd(&fill[m], 1) * n + m;
        col[sn] = o;
        ref[sn] = 2 * f + 1;
    }
}

// Sort the filled slots of each row by column (the fill order above depends
// on atomic arrival) and pad the rest: the layout is then a pure function of
// the addressing.
__global__ void k_sort_pad(const int* __restrict__ deg, int n, int W, int* col, int* ref) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        int d = deg[c];
        for (int i = 1; i < d; ++i) {
            int kc = col[(size_t)i * n + c], kr = ref[(size_t)i * n + c];
            int j = i - 1;
            while (j >= 0 && col[(size_t)j * n + c] > kc) {
                col[(size_t)(j + 1) * n + c] = col[(size_t)j * n + c];
                ref[(size_t)(j + 1) * n + c] = ref[(size_t)j * n + c];
                --j;
            }
            col[(size_t)(j + 1) * n + c] = kc;
            ref[(size_t)(j + 1) * n + c] = kr;
        }
        for (int k = d; k < W; ++k) {
            col[(size_t)k * n + c] = c;
            ref[(size_t)k * n + c] = -1;
        }
    }
}

// Largest |column - row| over all slots (the matrix bandwidth).
__global__ void k_max_offset(const int* __restrict__ col, int n, int W, int* out) {
    int m = 0;
    const size_t total = (size_t)W * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % (size_t)n);
        m = max(m, abs(col[i] - c));
    }
    atomicMax(out, m);
}

__global__ void k_make_col16(const int* __restrict__ col, int n, int W, int16_t* col16) {
    const size_t total = (size_t)W * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % (size_t)n);
        col16[i] = (int16_t)(col[i] - c);
    }
}

// Coefficients into the slot layout; also the column-scaled copy
// A[c][j] / d[j] used by the Jacobi-folded pipelined kernels, and the FP32
// copies when requested.
__global__ void k_gather_coeffs(const int* __restrict__ ref, const int* __restrict__ col, int n, int W,
                                const double* __restrict__ diag, const double* __restrict__ upper,
                                const double* __restrict__ lower, double* val, double* val_cs, float* val32,
                                float* val32_cs) {
    size_t total = (size_t)W * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        int rf = ref[i];
        double v = 0.0;
        if (rf >= 0) v = (rf & 1) ? lower[rf >> 1] : upper[rf >> 1];
        double vcs = (rf >= 0) ? v / diag[col[i]] : 0.0;
        val[i] = v;
        val_cs[i] = vcs;
        if (val32_cs) {
            val32[i] = (float)v;
            val32_cs[i] = (float)vcs;
        }
    }
}

// flag bit 2: lower differs from upper on some face (or either is NaN); one
// atomic per workgroup that saw a difference (a non-symmetric matrix differs
// on almost every face, so the launch uses at most kCheckGrid workgroups:
// with one atomic per wavefront over every face the same-address atomics
// took 3 ms at 21M faces)
constexpr int kCheckGrid = 1024;
__global__ void k_check_sym(const double* __restrict__ upper, const double* __restrict__ lower, int F,
                            unsigned* flags) {
    bool asym = false;
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x)
        if (!(upper[f] == lower[f])) asym = true;
    if (__syncthreads_or(asym) && threadIdx.x == 0) atomicOr(flags, 2u);
}

__global__ void k_copy_diag(const double* __restrict__ diag, int n, double* d, float* d32, unsigned* flags) {
    unsigned bad = 0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        double v = diag[c];
        d[c] = v;
        if (d32) d32[c] = (float)v;
        if (!(v > 0.0) || !isfinite(v)) bad = 1u;
    }
    if (bad) atomicOr(flags, bad);
}

int grid_for(size_t work) {
    size_t g = (work + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

void mesh_free(fvpcg_mesh* m) {
    if (!m) return;
    dev_free(m->owner);
    dev_free(m->nb);
    dev_free(m->col);
    dev_free(m->col16);
    dev_free(m->ref);
    delete m;
}

// Copy a few device ints to the host through a synchronous copy on `s`.
int read_back(hipStream_t s, void* host, const void* dev, size_t bytes) {
    FV_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    FV_HIP(hipStreamSynchronize(s));
    return FVPCG_OK;
}

}  // namespace

int matrix_refresh(fvpcg_matrix* A, const double* diag, const double* upper, const double* lower, hipStream_t s) {
    const fvpcg_mesh* m = A->mesh;
    const double* lo = lower ? lower : upper;
    unsigned* dflag = nullptr;
    int rc = dev_alloc(&dflag, 1, "diagonal check flag");
    if (rc) return rc;
    unsigned hflag = 0;
    rc = FVPCG_OK;
    do {
        if (hipMemsetAsync(dflag, 0, sizeof(unsigned), s) != hipSuccess) { rc = hip_fail(hipGetLastError(), "memset", __FILE__, __LINE__); break; }
        hipLaunchKernelGGL(k_copy_diag, dim3(grid_for(m->n)), dim3(kBlock), 0, s, diag, m->n, A->d, A->d32, dflag);
        if (lower && m->F > 0)
            hipLaunchKernelGGL(k_check_sym, dim3(std::min(grid_for(m->F), kCheckGrid)), dim3(kBlock), 0, s, upper,
                               lower, m->F, dflag);
        hipLaunchKernelGGL(k_gather_coeffs, dim3(grid_for((size_t)m->W * m->n)), dim3(kBlock), 0, s, m->ref, m->col,
                           m->n, m->W, diag, upper, lo, A->val, A->val_cs, A->val32, A->val32_cs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { rc = hip_fail(e, "coefficient kernels", __FILE__, __LINE__); break; }
        rc = read_back(s, &hflag, dflag, sizeof(unsigned));
    } while (0);
    dev_free(dflag);
    if (rc) return rc;
    A->diag_ok = (hflag & 1u) == 0;
    A->vals_sym = (hflag & 2u) == 0;
    ++A->generation;
    return FVPCG_OK;
}

int mesh_create(int32_t n, int32_t F, const int32_t* owner, const int32_t* nb, hipStream_t s, fvpcg_mesh** out) {
    fvpcg_mesh* m = new (std::nothrow) fvpcg_mesh();
    if (!m) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    FV_HIP(hipGetDevice(&m->device));
    m->n = n;
    m->F = F;
    int rc = FVPCG_OK;
    int* deg = nullptr;
    int* fill = nullptr;
    unsigned* flags = nullptr;
    int* dmax = nullptr;
    auto fail = [&](int code) {
        dev_free(deg);
        dev_free(fill);
        dev_free(flags);
        dev_free(dmax);
        mesh_free(m);
        return code;
    };
    if ((rc = dev_alloc(&m->owner, (size_t)F, "owner"))) return fail(rc);
    if ((rc = dev_alloc(&m->nb, (size_t)F, "neighbour"))) return fail(rc);
    if ((rc = dev_alloc(&flags, 1, "flags"))) return fail(rc);
    if ((rc = dev_alloc(&dmax, 1, "max degree"))) return fail(rc);
    if ((rc = dev_alloc(&deg, (size_t)n, "row degree"))) return fail(rc);
    if ((rc = dev_alloc(&fill, (size_t)n, "row fill"))) return fail(rc);
#define CK(x)                                                                   \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) return fail(hip_fail(e_, #x, __FILE__, __LINE__)); \
    } while (0)
    if (F > 0) {
        CK(hipMemcpyAsync(m->owner, owner, sizeof(int) * (size_t)F, hipMemcpyDeviceToDevice, s));
        CK(hipMemcpyAsync(m->nb, nb, sizeof(int) * (size_t)F, hipMemcpyDeviceToDevice, s));
    }
    CK(hipMemsetAsync(flags, 0, sizeof(unsigned), s));
    CK(hipMemsetAsync(dmax, 0, sizeof(int), s));
    CK(hipMemsetAsync(deg, 0, sizeof(int) * (size_t)n, s));
    CK(hipMemsetAsync(fill, 0, sizeof(int) * (size_t)n, s));
    if (F > 0) {
        hipLaunchKernelGGL(k_validate, dim3(grid_for(F)), dim3(kBlock), 0, s, m->owner, m->nb, F, n, flags);
        CK(hipGetLastError());
    }
    unsigned hflags = 0;
    if ((rc = read_back(s, &hflags, flags, sizeof(unsigned)))) return fail(rc);
    if (hflags & 1u)
        return fail(set_error(FVPCG_INVALID_MESH, "addressing out of range or owner >= neighbour"));
    if (hflags & 2u)
        return fail(set_error(FVPCG_INVALID_MESH, "faces not strictly sorted by (owner, neighbour)"));
    if (F > 0) {
        hipLaunchKernelGGL(k_degree, dim3(grid_for(F)), dim3(kBlock), 0, s, m->owner, m->nb, F, deg);
        hipLaunchKernelGGL(k_maxdeg, dim3(grid_for(n)), dim3(kBlock), 0, s, deg, n, dmax);
        CK(hipGetLastError());
    }
    int W = 0;
    if ((rc = read_back(s, &W, dmax, sizeof(int)))) return fail(rc);
    if (W < 1) W = 1;
    if (W > FVPCG_MAX_ROW_DEGREE)
        return fail(set_error(FVPCG_UNSUPPORTED, "row degree %d exceeds %d", W, FVPCG_MAX_ROW_DEGREE));
    m->maxdeg = W;
    m->W = pick_wt(W);  // pad to the kernel width: the row loops carry no slot guard
    m->WT = m->W;
    W = m->W;
    if ((rc = dev_alloc(&m->col, (size_t)W * n, "ELL columns"))) return fail(rc);
    if ((rc = dev_alloc(&m->ref, (size_t)W * n, "ELL face references"))) return fail(rc);
    if (F > 0) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(F)), dim3(kBlock), 0, s, m->owner, m->nb, F, n, fill, m->col, m->ref);
        CK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_sort_pad, dim3(grid_for(n)), dim3(kBlock), 0, s, deg, n, W, m->col, m->ref);
    CK(hipGetLastError());
    // 16-bit column offsets when the bandwidth allows (FVPCG_COL16=0 keeps int32)
    {
        const char* env = getenv("FVPCG_COL16");
        if (!(env && env[0] == '0')) {
            CK(hipMemsetAsync(dmax, 0, sizeof(int), s));
            hipLaunchKernelGGL(k_max_offset, dim3(grid_for((size_t)W * n)), dim3(kBlock), 0, s, m->col, n, W, dmax);
            CK(hipGetLastError());
            int band = 0;
            if ((rc = read_back(s, &band, dmax, sizeof(int)))) return fail(rc);
            m->bandwidth = band;
            if (band <= 32767) {
                if ((rc = dev_alloc(&m->col16, (size_t)W * n, "ELL column offsets"))) return fail(rc);
                hipLaunchKernelGGL(k_make_col16, dim3(grid_for((size_t)W * n)), dim3(kBlock), 0, s, m->col, n, W,
                                   m->col16);
                CK(hipGetLastError());
            }
        }
    }
    CK(hipStreamSynchronize(s));
#undef CK
    dev_free(deg);
    dev_free(fill);
    dev_free(flags);
    dev_free(dmax);
    m->geom = make_geom(n);
    *out = m;
    return FVPCG_OK;
}

int mesh_destroy(fvpcg_mesh* m) {
    mesh_free(m);
    return FVPCG_OK;
}

void matrix_free(fvpcg_matrix* A) {
    if (!A) return;
    if (A->work) {
        work_free(*A->work);
        delete A->work;
    }
    dev_free(A->d);
    dev_free(A->val);
    dev_free(A->val_cs);
    dev_free(A->d32);
    dev_free(A->val32);
    dev_free(A->val32_cs);
    delete A;
}

int matrix_create(const fvpcg_mesh* m, const double* diag, const double* upper, const double* lower, uint32_t flags,
                  hipStream_t s, fvpcg_matrix** out) {
    fvpcg_matrix* A = new (std::nothrow) fvpcg_matrix();
    if (!A) return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    A->mesh = m;
    A->sym = (lower == nullptr);
    A->fp32 = (flags & FVPCG_FP32_COPY) != 0;
    int rc;
    size_t slots = (size_t)m->W * m->n;
    if ((rc = dev_alloc(&A->d, (size_t)m->n, "diagonal")) || (rc = dev_alloc(&A->val, slots, "ELL values")) ||
        (rc = dev_alloc(&A->val_cs, slots, "ELL scaled values"))) {
        matrix_free(A);
        return rc;
    }
    if (A->fp32) {
        if ((rc = dev_alloc(&A->d32, (size_t)m->n, "FP32 diagonal")) ||
            (rc = dev_alloc(&A->val32, slots, "FP32 ELL values")) ||
            (rc = dev_alloc(&A->val32_cs, slots, "FP32 ELL scaled values"))) {
            matrix_free(A);
            return rc;
        }
    }
    A->work = new (std::nothrow) Work();
    if (!A->work) {
        matrix_free(A);
        return set_error(FVPCG_OUT_OF_MEMORY, "host allocation failed");
    }
    if ((rc = matrix_refresh(A, diag, upper, lower, s))) {
        matrix_free(A);
        return rc;
    }
    *out = A;
    return FVPCG_OK;
}

int matrix_update(fvpcg_matrix* A, const double* diag, const double* upper, const double* lower, hipStream_t s) {
    if (A->sym != (lower == nullptr))
        return set_error(FVPCG_INVALID_ARG, "matrix_update: lower must be %s as at creation",
                         A->sym ? "NULL" : "non-NULL");
    return matrix_refresh(A, diag, upper, lower, s);
}

int matrix_destroy(fvpcg_matrix* A) {
    matrix_free(A);
    return FVPCG_OK;
}

}  // namespace fvpcg
