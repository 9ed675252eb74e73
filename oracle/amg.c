/*
 * CPU oracle, smoothed-aggregation AMG preconditioner for CG -- TEST
 * INFRASTRUCTURE.
 *
 * The paper compares its Jacobi-preconditioned solvers with aggregation-AMG
 * preconditioned CG and pipelined CG (Section 5, Fig. pcgs1 and Table pcgs2:
 * 325 -> 28 CG iterations at 64^3).  It names the method's parts: a V-cycle
 * of aggregation-based AMG, aggregates from the parallel distance-2
 * maximal-independent-set method, and weighted Jacobi with omega = 4/3 as
 * the smoother.  Written from those definitions:
 *   strength    j ~ i  iff  j != i, a_ij != 0 and
 *               |a_ij| >= theta_l sqrt(|a_ii a_jj|), theta_{l+1} = theta_l / 2
 *               (theta = 0: every coupling is strong);
 *   aggregates  roots: a distance-2 maximal independent set of the strength
 *               graph, in the order of seeded SplitMix64 priorities; round 1:
 *               the roots' neighbours; round 2: the rest join a round-1
 *               neighbour's aggregate (or_amg_aggregate states the rules);
 *   prolongator P = (I - omega D^-1 A) P_t, P_t the aggregate indicator,
 *               omega = (4/3) / lambda, lambda = max_i sum_j |a_ij| / a_ii
 *               (Gershgorin bound of rho(D^-1 A)): the paper's 4/3 taken
 *               for the operator scaled to spectral radius 1;
 *   coarse      A_c = P^T A P (Galerkin), R = P^T;
 *   levels      until n <= coarse_size, the level limit, or an aggregation
 *               that keeps more than 60% of the unknowns; the last level
 *               (at most OR_AMG_MAX_COARSE unknowns) is solved exactly
 *               (dense Cholesky);
 *   cycle       V(1,1): x = omega D^-1 b; r = b - A x; x += P V(R r);
 *               x += omega D^-1 (b - A x).
 * The cycle is symmetric and positive definite for SPD A, so it is a valid
 * preconditioner for standard CG.  Plain C, FP64, single thread.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n, m;     /* rows, columns */
    int32_t* ptr;     /* n + 1 */
    int32_t* col;     /* sorted within each row */
    double* val;
} csr_t;

struct or_amg {
    int32_t nlev;
    csr_t A[OR_AMG_MAX_LEVELS], P[OR_AMG_MAX_LEVELS], R[OR_AMG_MAX_LEVELS];
    double* d[OR_AMG_MAX_LEVELS];
    double omega[OR_AMG_MAX_LEVELS];
    int32_t* agg[OR_AMG_MAX_LEVELS];
    double* chol;   /* dense lower factor of the last level, row-major */
    double *b[OR_AMG_MAX_LEVELS], *x[OR_AMG_MAX_LEVELS], *r[OR_AMG_MAX_LEVELS];
};

static void csr_free(csr_t* a)
{
    free(a->ptr); free(a->col); free(a->val);
    memset(a, 0, sizeof(*a));
}

static void sort_row(int32_t* col, double* val, int32_t len)
{
    for (int32_t i = 1; i < len; ++i) {
        int32_t c = col[i]; double v = val[i]; int32_t j = i - 1;
        while (j >= 0 && col[j] > c) { col[j + 1] = col[j]; val[j + 1] = val[j]; --j; }
        col[j + 1] = c; val[j + 1] = v;
    }
}

/* The LDU matrix as CSR: row c holds its diagonal, upper[f] at column
 * neighbour[f] for faces it owns and lower[f] at column owner[f] for faces
 * it neighbours (Section 4.2's nnz = n + 2F). */
static void csr_from_ldu(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                         const double* diag, const double* upper, const double* lower, csr_t* A)
{
    A->n = A->m = n;
    A->ptr = calloc((size_t)n + 1, sizeof(int32_t));
    for (int32_t c = 0; c < n; ++c) A->ptr[c + 1] = 1;
    for (int32_t f = 0; f < nf; ++f) { A->ptr[owner[f] + 1]++; A->ptr[nb[f] + 1]++; }
    for (int32_t c = 0; c < n; ++c) A->ptr[c + 1] += A->ptr[c];
    int32_t nnz = A->ptr[n];
    A->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    A->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t* fill = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t c = 0; c < n; ++c) {
        fill[c] = A->ptr[c] + 1;
        A->col[A->ptr[c]] = c;
        A->val[A->ptr[c]] = diag[c];
    }
    for (int32_t f = 0; f < nf; ++f) {
        int32_t o = owner[f], m = nb[f];
        A->col[fill[o]] = m; A->val[fill[o]++] = upper[f];
        A->col[fill[m]] = o; A->val[fill[m]++] = lower[f];
    }
    for (int32_t c = 0; c < n; ++c) sort_row(A->col + A->ptr[c], A->val + A->ptr[c], A->ptr[c + 1] - A->ptr[c]);
    free(fill);
}

static void csr_diag(const csr_t* A, double* d)
{
    for (int32_t i = 0; i < A->n; ++i) {
        d[i] = 0.0;
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p)
            if (A->col[p] == i) d[i] = A->val[p];
    }
}

/* y = A v */
static void csr_mv(const csr_t* A, const double* v, double* y)
{
    for (int32_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p) s += A->val[p] * v[A->col[p]];
        y[i] = s;
    }
}

static void csr_transpose(const csr_t* A, csr_t* T)
{
    T->n = A->m; T->m = A->n;
    int32_t nnz = A->ptr[A->n];
    T->ptr = calloc((size_t)T->n + 1, sizeof(int32_t));
    T->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    T->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (int32_t p = 0; p < nnz; ++p) T->ptr[A->col[p] + 1]++;
    for (int32_t j = 0; j < T->n; ++j) T->ptr[j + 1] += T->ptr[j];
    int32_t* fill = malloc(sizeof(int32_t) * (size_t)(T->n > 0 ? T->n : 1));
    for (int32_t j = 0; j < T->n; ++j) fill[j] = T->ptr[j];
    for (int32_t i = 0; i < A->n; ++i)  /* rows in order: columns of T come out sorted */
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p) {
            int32_t q = fill[A->col[p]]++;
            T->col[q] = i; T->val[q] = A->val[p];
        }
    free(fill);
}

/* C = X Y: row by row with a dense accumulator; within a row the products
 * are added in the order of X's columns, then Y's columns. */
static void csr_mm(const csr_t* X, const csr_t* Y, csr_t* C)
{
    C->n = X->n; C->m = Y->m;
    C->ptr = calloc((size_t)C->n + 1, sizeof(int32_t));
    double* acc = calloc((size_t)(Y->m > 0 ? Y->m : 1), sizeof(double));
    int32_t* mark = malloc(sizeof(int32_t) * (size_t)(Y->m > 0 ? Y->m : 1));
    for (int32_t k = 0; k < Y->m; ++k) mark[k] = -1;
    int32_t* list = malloc(sizeof(int32_t) * (size_t)(Y->m > 0 ? Y->m : 1));
    size_t cap = 16, nnz = 0;
    C->col = malloc(sizeof(int32_t) * cap);
    C->val = malloc(sizeof(double) * cap);
    for (int32_t i = 0; i < X->n; ++i) {
        int32_t len = 0;
        for (int32_t p = X->ptr[i]; p < X->ptr[i + 1]; ++p) {
            int32_t j = X->col[p];
            double xv = X->val[p];
            for (int32_t q = Y->ptr[j]; q < Y->ptr[j + 1]; ++q) {
                int32_t k = Y->col[q];
                if (mark[k] != i) { mark[k] = i; acc[k] = 0.0; list[len++] = k; }
                acc[k] += xv * Y->val[q];
            }
        }
        /* sort the touched columns */
        for (int32_t a = 1; a < len; ++a) {
            int32_t c = list[a], b = a - 1;
            while (b >= 0 && list[b] > c) { list[b + 1] = list[b]; --b; }
            list[b + 1] = c;
        }
        if (nnz + (size_t)len > cap) {
            while (nnz + (size_t)len > cap) cap *= 2;
            C->col = realloc(C->col, sizeof(int32_t) * cap);
            C->val = realloc(C->val, sizeof(double) * cap);
        }
        for (int32_t a = 0; a < len; ++a) { C->col[nnz] = list[a]; C->val[nnz++] = acc[list[a]]; }
        C->ptr[i + 1] = (int32_t)nnz;
    }
    free(acc); free(mark); free(list);
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based
 * generator: element k of the sequence whose state starts at `seed` is the
 * finaliser applied to seed + (k + 1) * 0x9E3779B97F4A7C15. */
uint64_t or_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Priority of unknown i on level l: 31 random bits from the counter
 * (l, i), then the index itself, so that no two unknowns tie. */
uint64_t or_amg_priority(uint64_t seed, int32_t level, int32_t i)
{
    const uint64_t r = or_splitmix64(seed, ((uint64_t)(uint32_t)level << 32) | (uint32_t)i) >> 33;
    return (r << 31) | (uint32_t)i;
}

static int key_desc(const void* a, const void* b)
{
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? 1 : (x > y ? -1 : 0);
}

/* Strong coupling (the strength graph the aggregation works on): a stored,
 * non-zero off-diagonal entry with |a_ij| >= theta sqrt(|a_ii a_jj|). */
static int strong(const csr_t* A, const double* d, double theta, int32_t i, int32_t p)
{
    const int32_t j = A->col[p];
    return j != i && A->val[p] != 0.0 && fabs(A->val[p]) >= theta * sqrt(fabs(d[i] * d[j]));
}

/* Aggregation by a distance-2 maximal independent set of the strength graph
 * (the parallel aggregation of the paper's AMG, Section 5):
 *   roots: the maximal set of unknowns no two of which are joined by a path
 *          of one or two strong couplings, taken greedily in decreasing
 *          priority (key[i]): an unknown becomes a root unless an earlier
 *          root lies within distance 2 of it.  This is the set the parallel
 *          rule (an undecided unknown joins when its priority is the largest
 *          among the undecided within distance 2 and no root is that close)
 *          arrives at;
 *   numbering: aggregate a is the a-th root in index order;
 *   round 1: every other unknown with a root among its strong neighbours
 *          joins that root's aggregate (there is at most one: two roots are
 *          never two steps apart);
 *   round 2: every unknown still outside joins the round-1 aggregate of its
 *          strong neighbour with the largest |a_ij| (ties: the lowest j).
 * Maximality puts every unknown within distance 2 of a root, so the two
 * rounds place all of them; an unknown without strong couplings is a root of
 * its own.  key == NULL: key[i] = or_amg_priority(seed, level, i).  Returns
 * the number of aggregates, or -1 if an unknown was left out (not possible
 * for a maximal set: kept as a check). */
int32_t or_amg_aggregate(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double theta,
                         const uint64_t* key, uint64_t seed, int32_t level, int32_t* agg)
{
    csr_t A = {n, n, (int32_t*)ptr, (int32_t*)col, (double*)val};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    double* d = malloc(sizeof(double) * nn);
    csr_diag(&A, d);
    uint64_t* order = malloc(sizeof(uint64_t) * nn);
    for (int32_t i = 0; i < n; ++i) order[i] = key ? key[i] : or_amg_priority(seed, level, i);
    /* the index of each unknown is recovered from its key through a lookup */
    int32_t* who = NULL;
    if (key) {
        /* explicit keys: sort (key, i) pairs by key; keys must be distinct */
        uint64_t* pair = malloc(sizeof(uint64_t) * 2 * nn);
        for (int32_t i = 0; i < n; ++i) { pair[2 * i] = key[i]; pair[2 * i + 1] = (uint64_t)i; }
        qsort(pair, (size_t)n, 2 * sizeof(uint64_t), key_desc);
        who = malloc(sizeof(int32_t) * nn);
        for (int32_t i = 0; i < n; ++i) who[i] = (int32_t)pair[2 * i + 1];
        free(pair);
    } else {
        qsort(order, (size_t)n, sizeof(uint64_t), key_desc);
        who = malloc(sizeof(int32_t) * nn);
        for (int32_t i = 0; i < n; ++i) who[i] = (int32_t)(uint32_t)(order[i] & 0x7FFFFFFFull);
    }
    /* state: 0 free, 1 root, 2 within distance 2 of a root */
    unsigned char* state = calloc(nn, 1);
    for (int32_t t = 0; t < n; ++t) {
        const int32_t v = who[t];
        if (state[v] != 0) continue;
        state[v] = 1;
        for (int32_t p = ptr[v]; p < ptr[v + 1]; ++p) {
            if (!strong(&A, d, theta, v, p)) continue;
            const int32_t u = col[p];
            if (state[u] == 0) state[u] = 2;
            for (int32_t q = ptr[u]; q < ptr[u + 1]; ++q)
                if (strong(&A, d, theta, u, q) && state[col[q]] == 0) state[col[q]] = 2;
        }
    }
    int32_t na = 0;
    for (int32_t i = 0; i < n; ++i) agg[i] = state[i] == 1 ? na++ : -1;
    int32_t* agg1 = malloc(sizeof(int32_t) * nn);
    for (int32_t i = 0; i < n; ++i) {                /* round 1 */
        agg1[i] = agg[i];
        if (agg[i] >= 0) continue;
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (strong(&A, d, theta, i, p) && state[col[p]] == 1) { agg1[i] = agg[col[p]]; break; }
    }
    int32_t rc = na;
    for (int32_t i = 0; i < n; ++i) {                /* round 2 */
        agg[i] = agg1[i];
        if (agg1[i] >= 0) continue;
        int32_t best = -1;
        double bw = -1.0;
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int32_t j = col[p];
            if (!strong(&A, d, theta, i, p) || agg1[j] < 0) continue;
            if (fabs(val[p]) > bw) { bw = fabs(val[p]); best = j; }  /* columns ascend: ties keep the lowest j */
        }
        if (best < 0) rc = -1;
        else agg[i] = agg1[best];
    }
    free(agg1); free(state); free(who); free(order); free(d);
    return rc;
}

/* P = (I - omega D^-1 A) P_t, row i: 1 at agg[i], minus omega a_ij / a_ii at
 * agg[j] for every stored a_ij (the diagonal included), in column order. */
static void smoothed_prolongator(const csr_t* A, const double* d, const int32_t* agg, int32_t na, double omega,
                                 csr_t* P)
{
    const int32_t n = A->n;
    csr_t Pt = {n, na, NULL, NULL, NULL};
    Pt.ptr = malloc(sizeof(int32_t) * ((size_t)n + 1));
    Pt.col = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    Pt.val = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i <= n; ++i) Pt.ptr[i] = i;
    for (int32_t i = 0; i < n; ++i) { Pt.col[i] = agg[i]; Pt.val[i] = 1.0; }
    /* S = I - omega D^-1 A as CSR, then P = S P_t */
    csr_t S = {n, n, NULL, NULL, NULL};
    int32_t nnz = A->ptr[n];
    S.ptr = malloc(sizeof(int32_t) * ((size_t)n + 1));
    S.col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    S.val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    memcpy(S.ptr, A->ptr, sizeof(int32_t) * ((size_t)n + 1));
    memcpy(S.col, A->col, sizeof(int32_t) * (size_t)nnz);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p)
            S.val[p] = (A->col[p] == i ? 1.0 : 0.0) - omega * A->val[p] / d[i];
    csr_mm(&S, &Pt, P);
    csr_free(&S);
    csr_free(&Pt);
}

static double gershgorin(const csr_t* A, const double* d)
{
    double lam = 0.0;
    for (int32_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p) s += fabs(A->val[p]);
        s /= d[i];
        if (s > lam) lam = s;
    }
    return lam;
}

static int dense_cholesky(const csr_t* A, double* L)
{
    const int32_t n = A->n;
    memset(L, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t p = A->ptr[i]; p < A->ptr[i + 1]; ++p) L[(size_t)i * n + A->col[p]] = A->val[p];
    for (int32_t j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return 0;
        const double ljj = sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) L[(size_t)i * n + j] = 0.0;
    return 1;
}

or_amg* or_amg_setup(int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                     const double* diag, const double* upper, const double* lower,
                     double theta, int32_t max_levels, int32_t coarse_size, uint64_t seed)
{
    if (max_levels < 1) max_levels = 1;
    if (max_levels > OR_AMG_MAX_LEVELS) max_levels = OR_AMG_MAX_LEVELS;
    or_amg* h = calloc(1, sizeof(or_amg));
    csr_from_ldu(n, nf, owner, nb, diag, upper, lower, &h->A[0]);
    int32_t l = 0;
    double th = theta;
    for (;;) {
        const csr_t* A = &h->A[l];
        h->d[l] = malloc(sizeof(double) * (size_t)(A->n > 0 ? A->n : 1));
        csr_diag(A, h->d[l]);
        h->omega[l] = 4.0 / (3.0 * gershgorin(A, h->d[l]));
        h->b[l] = calloc((size_t)(A->n > 0 ? A->n : 1), sizeof(double));
        h->x[l] = calloc((size_t)(A->n > 0 ? A->n : 1), sizeof(double));
        h->r[l] = calloc((size_t)(A->n > 0 ? A->n : 1), sizeof(double));
        if (A->n <= coarse_size || l + 1 == max_levels) break;
        int32_t* agg = malloc(sizeof(int32_t) * (size_t)A->n);
        int32_t na = or_amg_aggregate(A->n, A->ptr, A->col, A->val, th, NULL, seed, l, agg);
        if (na < 0 || (double)na > 0.6 * (double)A->n) { free(agg); break; }
        h->agg[l] = agg;
        smoothed_prolongator(A, h->d[l], agg, na, h->omega[l], &h->P[l]);
        csr_transpose(&h->P[l], &h->R[l]);
        csr_t AP;
        csr_mm(A, &h->P[l], &AP);
        csr_mm(&h->R[l], &AP, &h->A[l + 1]);
        csr_free(&AP);
        th *= 0.5;
        ++l;
    }
    h->nlev = l + 1;
    const int32_t nc = h->A[l].n;
    if (nc > OR_AMG_MAX_COARSE) { or_amg_free(h); return NULL; }  /* too large to solve densely */
    h->chol = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1) * (size_t)(nc > 0 ? nc : 1));
    if (!dense_cholesky(&h->A[l], h->chol)) { or_amg_free(h); return NULL; }
    return h;
}

/* The hierarchy for new coefficients of the same mesh with the aggregates
 * kept: level 0 from the LDU arrays, then on every level the diagonal, omega
 * from the Gershgorin bound, P = (I - omega D^-1 A) P_t from the stored
 * aggregates, R = P^T and A_c = R (A P), and the last level's factor, all as
 * or_amg_setup computes them.  Returns 0, or -1 if the last level is not
 * positive definite (the handle is then unusable) or n differs. */
int32_t or_amg_refresh(or_amg* h, int32_t n, int32_t nf, const int32_t* owner, const int32_t* nb,
                       const double* diag, const double* upper, const double* lower)
{
    if (!h || n != h->A[0].n) return -1;
    csr_free(&h->A[0]);
    csr_from_ldu(n, nf, owner, nb, diag, upper, lower, &h->A[0]);
    const int32_t last = h->nlev - 1;
    for (int32_t l = 0; l <= last; ++l) {
        const csr_t* A = &h->A[l];
        csr_diag(A, h->d[l]);
        h->omega[l] = 4.0 / (3.0 * gershgorin(A, h->d[l]));
        if (l == last) break;
        const int32_t na = h->A[l + 1].n;  /* the aggregate count */
        csr_free(&h->P[l]);
        csr_free(&h->R[l]);
        csr_free(&h->A[l + 1]);
        smoothed_prolongator(A, h->d[l], h->agg[l], na, h->omega[l], &h->P[l]);
        csr_transpose(&h->P[l], &h->R[l]);
        csr_t AP;
        csr_mm(A, &h->P[l], &AP);
        csr_mm(&h->R[l], &AP, &h->A[l + 1]);
        csr_free(&AP);
    }
    return dense_cholesky(&h->A[last], h->chol) ? 0 : -1;
}

void or_amg_free(or_amg* h)
{
    if (!h) return;
    for (int32_t l = 0; l < OR_AMG_MAX_LEVELS; ++l) {
        csr_free(&h->A[l]); csr_free(&h->P[l]); csr_free(&h->R[l]);
        free(h->d[l]); free(h->agg[l]); free(h->b[l]); free(h->x[l]); free(h->r[l]);
    }
    free(h->chol);
    free(h);
}

int32_t or_amg_levels(const or_amg* h) { return h->nlev; }

void or_amg_level_info(const or_amg* h, int32_t l, int32_t* n, int32_t* nnz, int32_t* n_coarse, double* omega)
{
    *n = h->A[l].n;
    *nnz = h->A[l].ptr[h->A[l].n];
    *n_coarse = l + 1 < h->nlev ? h->A[l + 1].n : 0;
    *omega = h->omega[l];
}

/* Copy out level l's aggregates (n_l entries), or its A / P as CSR
 * (which = 0: A, 1: P); pass NULL arrays to query only the sizes. */
void or_amg_aggregates(const or_amg* h, int32_t l, int32_t* out)
{
    memcpy(out, h->agg[l], sizeof(int32_t) * (size_t)h->A[l].n);
}

int32_t or_amg_export(const or_amg* h, int32_t l, int32_t which, int32_t* rows, int32_t* cols, int32_t* ptr,
                      int32_t* col, double* val)
{
    const csr_t* M = which == 0 ? &h->A[l] : &h->P[l];
    *rows = M->n;
    *cols = M->m;
    const int32_t nnz = M->ptr[M->n];
    if (ptr) memcpy(ptr, M->ptr, sizeof(int32_t) * ((size_t)M->n + 1));
    if (col) memcpy(col, M->col, sizeof(int32_t) * (size_t)nnz);
    if (val) memcpy(val, M->val, sizeof(double) * (size_t)nnz);
    return nnz;
}

static void vcycle(const or_amg* h, int32_t l, const double* b, double* x)
{
    const csr_t* A = &h->A[l];
    const int32_t n = A->n;
    if (l + 1 == h->nlev) {  /* exact: L L^T x = b */
        const double* L = h->chol;
        for (int32_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int32_t k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * x[k];
            x[i] = s / L[(size_t)i * n + i];
        }
        for (int32_t i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int32_t k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
            x[i] = s / L[(size_t)i * n + i];
        }
        return;
    }
    const double* d = h->d[l];
    const double w = h->omega[l];
    double* r = h->r[l];
    for (int32_t i = 0; i < n; ++i) x[i] = w * b[i] / d[i];            /* pre-smooth from 0 */
    csr_mv(A, x, r);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - r[i];                /* residual */
    double* bc = h->b[l + 1];
    double* xc = h->x[l + 1];
    csr_mv(&h->R[l], r, bc);                                            /* restrict */
    vcycle(h, l + 1, bc, xc);
    double* e = r;
    csr_mv(&h->P[l], xc, e);                                            /* prolong */
    for (int32_t i = 0; i < n; ++i) x[i] += e[i];
    csr_mv(A, x, r);
    for (int32_t i = 0; i < n; ++i) x[i] += w * (b[i] - r[i]) / d[i];  /* post-smooth */
}

void or_amg_vcycle(const or_amg* h, const double* b, double* x) { vcycle(h, 0, b, x); }

/* Standard preconditioned CG (Section 2) with M^-1 = one V-cycle. */
int32_t or_amg_pcg(const or_amg* h, const double* b, double* x, double tol, int32_t maxit, or_stats* st)
{
    const csr_t* A = &h->A[0];
    const int32_t n = A->n;
    if (st) memset(st, 0, sizeof(*st));
    double* r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* z = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* p = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* q = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    const double bnorm = sqrt(or_dot(n, b, b));
    int32_t status = OR_NOT_CONVERGED, it = 0;
    double rho = 0.0, gamma = 0.0;
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    csr_mv(A, x, r);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    rho = or_dot(n, r, r);
    if (st) st->r0_norm = sqrt(rho);
    if (sqrt(rho) <= tol * bnorm) { status = OR_OK; goto done; }
    vcycle(h, 0, r, z);
    gamma = or_dot(n, r, z);
    memcpy(p, z, sizeof(double) * (size_t)n);
    for (it = 0; it < maxit;) {
        csr_mv(A, p, q);
        const double delta = or_dot(n, p, q);
        if (!(delta > 0.0) || !isfinite(delta)) { status = OR_BREAKDOWN; break; }
        const double alpha = gamma / delta;
        for (int32_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++it;
        rho = or_dot(n, r, r);
        if (sqrt(rho) <= tol * bnorm) { status = OR_OK; break; }
        if (it >= maxit) break;
        vcycle(h, 0, r, z);
        const double gnew = or_dot(n, r, z);
        const double beta = gnew / gamma;
        gamma = gnew;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
done:
    if (st) {
        st->iters = it;
        st->status = status;
        st->b_norm = bnorm;
        st->rel_res = bnorm > 0 ? sqrt(rho) / bnorm : 0.0;
        csr_mv(A, x, q);
        double tr = 0.0;
        for (int32_t i = 0; i < n; ++i) tr += (b[i] - q[i]) * (b[i] - q[i]);
        st->true_rel_res = bnorm > 0 ? sqrt(tr) / bnorm : 0.0;
    }
    free(r); free(z); free(p); free(q);
    return status;
}

/* Pipelined CG of Ghysels and Vanroose (Section 4.1) with M^-1 = one
 * V-cycle, the literal recurrences (u = M^-1 r, m = M^-1 w, q = M^-1 s are
 * carried):
 *   r0 = b - A x0, u0 = M^-1 r0, w0 = A u0;  per iteration i:
 *   gamma = (r, u), delta = (w, u); stop on ||r|| <= tol ||b||;
 *   m = M^-1 w, n = A m;
 *   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
 *   (i = 0: beta = 0, alpha = gamma / delta);
 *   z = n + beta z, q = m + beta q, s = w + beta s, p = u + beta p;
 *   x += alpha p, r -= alpha s, u -= alpha q, w -= alpha z. */
int32_t or_amg_pipecg(const or_amg* h, const double* b, double* x, double tol, int32_t maxit, or_stats* st)
{
    const csr_t* A = &h->A[0];
    const int32_t n = A->n;
    if (st) memset(st, 0, sizeof(*st));
    const size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(sz), *u = malloc(sz), *w = malloc(sz), *m = malloc(sz), *nv = malloc(sz);
    double *z = calloc((size_t)(n > 0 ? n : 1), sizeof(double)), *q = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *s = calloc((size_t)(n > 0 ? n : 1), sizeof(double)), *p = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    const double bnorm = sqrt(or_dot(n, b, b));
    int32_t status = OR_NOT_CONVERGED, i = 0;
    double rho = 0.0;
    if (bnorm == 0.0) {
        for (int32_t c = 0; c < n; ++c) x[c] = 0.0;
        status = OR_OK;
        goto done;
    }
    csr_mv(A, x, r);
    for (int32_t c = 0; c < n; ++c) r[c] = b[c] - r[c];
    vcycle(h, 0, r, u);
    csr_mv(A, u, w);
    double gamma_prev = 0.0, alpha_prev = 0.0;
    for (i = 0;; ++i) {
        const double gamma = or_dot(n, r, u);
        const double delta = or_dot(n, w, u);
        rho = or_dot(n, r, r);
        if (i == 0 && st) st->r0_norm = sqrt(rho);
        if (sqrt(rho) <= tol * bnorm) { status = OR_OK; break; }
        if (i == maxit) break;
        vcycle(h, 0, w, m);
        csr_mv(A, m, nv);
        double beta, den;
        if (i == 0) { beta = 0.0; den = delta; }
        else { beta = gamma / gamma_prev; den = delta - beta * gamma / alpha_prev; }
        const double alpha = gamma / den;
        if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta)) { status = OR_BREAKDOWN; break; }
        for (int32_t c = 0; c < n; ++c) {
            z[c] = nv[c] + beta * z[c];
            q[c] = m[c] + beta * q[c];
            s[c] = w[c] + beta * s[c];
            p[c] = u[c] + beta * p[c];
            x[c] += alpha * p[c];
            r[c] -= alpha * s[c];
            u[c] -= alpha * q[c];
            w[c] -= alpha * z[c];
        }
        gamma_prev = gamma;
        alpha_prev = alpha;
    }
done:
    if (st) {
        st->iters = i;
        st->status = status;
        st->b_norm = bnorm;
        st->rel_res = bnorm > 0 ? sqrt(rho) / bnorm : 0.0;
        csr_mv(A, x, nv);
        double tr = 0.0;
        for (int32_t c = 0; c < n; ++c) tr += (b[c] - nv[c]) * (b[c] - nv[c]);
        st->true_rel_res = bnorm > 0 ? sqrt(tr) / bnorm : 0.0;
    }
    free(r); free(u); free(w); free(m); free(nv); free(z); free(q); free(s); free(p);
    return status;
}
