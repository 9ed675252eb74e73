"""Pins of the oracle's smoothed-aggregation AMG (oracle/amg.c) against facts
fixed by its definition and by linear algebra, independent of its code:

A0 the priorities' generator (SplitMix64) against its published outputs
A1 distance-2 maximal-independent-set aggregates of a 7-cell line, a 3x3
   grid, weighted rings and an uncoupled cell, worked by hand; on meshes, the
   roots equal those of the parallel rule (written here independently of the
   oracle's sequential greedy), are independent at distance 2 and maximal,
   and every aggregate holds its root's neighbours and lies within two steps
A2 every unknown in exactly one aggregate; no empty aggregate
A3 prolongator row sums: P 1 = (I - omega D^-1 A) 1
A4 Galerkin coarse operators equal SciPy's P^T A P
A5 omega = 4 / (3 * Gershgorin bound of D^-1 A), computed by NumPy
A6 one level: the cycle is the exact solve (dense LU)
A7 the cycle is symmetric positive definite and its error propagator
   I - M A contracts (spectral radius < 1, power iteration)
A8 AMG-PCG reaches the dense solution; iteration counts far below Jacobi-PCG
   and, at 64^3, of the order of Table pcgs2's GPU AMG-CG count 28 (loose:
   the paper's boundary conditions, right-hand side and stopping norm are
   not stated)
A9 AMG-preconditioned pipelined CG: the same iterates as AMG-PCG in exact
   arithmetic (equal at equal count up to rounding), the dense solution
R  refresh with new coefficients of the same mesh, the aggregates kept:
   R1 the same coefficients give the same hierarchy bit for bit; R2 twice
   the coefficients give the same P and every coarse operator doubled,
   exactly; R3 other coefficients give P = (I - w D^-1 A) P_t from the kept
   aggregates with w from NumPy's Gershgorin bound, Galerkin operators equal
   to SciPy's P^T A P, and a cycle that is SPD and contracting
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import fvcases as fc
from tests.helpers import dense

pytestmark = pytest.mark.cpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _csr(ptr, col, val, shape):
    return sp.csr_matrix((val, col, ptr), shape=shape)


def _line(n):
    """n cells on a line, unit faces, Dirichlet at both ends."""
    owner = np.arange(n - 1, dtype=np.int32)
    nb = owner + 1
    diag = np.full(n, 2.0)
    diag[0] = diag[-1] = 3.0
    up = -np.ones(n - 1)
    return fc.Case("line", (n, 1, 1), n, owner, nb, diag, up, up.copy(), np.ones(n))


# ---------------------------------------------------------------- A0
def test_a0_splitmix64_published_values(oracle_lib):
    """The priorities' generator against the published SplitMix64 outputs for
    state 0 (tests/golden/splitmix64.json) and against a Python rendering of
    its definition for other seeds and counters."""
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    for k, v in enumerate(g["seed0_first_outputs"]):
        assert oracle_lib.splitmix64(0, k) == int(v, 16)
    M = (1 << 64) - 1

    def mix(seed, k):
        z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for seed, k in ((1, 0), (1, 12345), (0xDEADBEEF, (3 << 32) | 77), (M, 5)):
        assert oracle_lib.splitmix64(seed, k) == mix(seed, k)
    # priority = 31 random bits of counter (level, i), then i
    p = oracle_lib.amg_priority(1, 2, 99)
    assert p & 0x7FFFFFFF == 99 and p >> 31 == mix(1, (2 << 32) | 99) >> 33


# ---------------------------------------------------------------- A1, A2
def _agg_keys(order, n):
    """Explicit priorities: the unknowns in `order` first (descending), the
    rest after them in index order."""
    key = np.zeros(n, dtype=np.uint64)
    rest = [i for i in range(n) if i not in order]
    for rank, i in enumerate(list(order) + rest):
        key[i] = np.uint64(10 * n - rank)
    return key


def _ring(n, strong_face=None, w=2.0):
    owner = np.array([0] + list(range(n - 1)), dtype=np.int32)
    nb = np.array([n - 1] + list(range(1, n)), dtype=np.int32)
    o = np.lexsort((nb, owner))
    owner, nb = owner[o], nb[o]
    up = -np.ones(n)
    if strong_face is not None:
        up[[k for k in range(n) if (owner[k], nb[k]) == strong_face][0]] = -w
    diag = np.ones(n)
    np.add.at(diag, owner, -up)
    np.add.at(diag, nb, -up)
    return fc.Case("ring", (n, 1, 1), n, owner, nb, diag, up, up.copy(), np.ones(n))


def _csr_ldu(case):
    """The LDU matrix as CSR with its stored pattern: a face whose
    coefficients are zero keeps its two (zero) entries."""
    n, o, m = case.n, case.owner.astype(np.int64), case.neighbour.astype(np.int64)
    rows = np.concatenate([np.arange(n), o, m])
    cols = np.concatenate([np.arange(n), m, o])
    vals = np.concatenate([case.diag, case.upper, case.lower])
    order = np.lexsort((cols, rows))
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, rows + 1, 1)
    A = sp.csr_matrix((vals[order], cols[order], np.cumsum(ptr)), shape=(n, n))
    assert A.has_sorted_indices and A.nnz == n + 2 * case.F
    return A


def _agg(oracle_lib, case, key, theta=0.0):
    A = _csr_ldu(case)
    return oracle_lib.aggregate(A.indptr, A.indices, A.data, theta, key=key)


def test_a1_aggregates_worked_by_hand(oracle_lib):
    # line 0..6.  Priorities 3 first: root 3 rules out 1, 2, 4, 5; then 0
    # and 6 (three steps from 3) become roots.  Aggregates in root-index
    # order: 0 -> 0, 3 -> 1, 6 -> 2; round 1 places 1 (next to 0), 2 and 4
    # (next to 3) and 5 (next to 6).
    line = _line(7)
    agg, na = _agg(oracle_lib, line, _agg_keys([3, 0, 6], 7))
    assert na == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2]
    # priorities 2, then 6: root 2 rules out 0, 1, 3, 4; 6 becomes a root
    # (four steps away) and rules out 5.  Round 1: 1, 3 -> 0 (next to 2),
    # 5 -> 1 (next to 6).  Round 2: 0's only neighbour 1 is in aggregate 0;
    # 4's neighbours 3 (aggregate 0) and 5 (aggregate 1) tie at |a| = 1 and
    # the lower index, 3, wins.
    agg, na = _agg(oracle_lib, line, _agg_keys([2, 6], 7))
    assert na == 2 and agg.tolist() == [0, 0, 0, 0, 0, 1, 1]
    # ring of 7 with the coupling 5-6 twice the others.  Roots 0, then 3
    # (three steps from 0 by 0-1-2-3, four the other way): round 1 puts 1, 6
    # with 0 and 2, 4 with 3.  5 (next to 4 and 6, neither a root) goes in
    # round 2 to its stronger neighbour 6's aggregate (0), not to 4's.
    ring = _ring(7, strong_face=(5, 6))
    agg, na = _agg(oracle_lib, ring, _agg_keys([0, 3], 7))
    assert na == 2 and agg.tolist() == [0, 0, 1, 1, 1, 0, 0]
    # the same with equal couplings: the tie goes to the lower index, 4
    agg, na = _agg(oracle_lib, _ring(7), _agg_keys([0, 3], 7))
    assert na == 2 and agg.tolist() == [0, 0, 1, 1, 1, 1, 0]
    # 3x3 grid, cell i + 3j.  Priorities 0, then 8: root 0 rules out 1, 3
    # (one step) and 2, 4, 6 (two steps); 8 is four steps from 0 and becomes
    # a root.  Round 1: 1, 3 -> 0; 5, 7 -> 1.  Round 2, all couplings equal,
    # lowest-index neighbour: 2 -> 1's (0), 4 -> 1's (0), 6 -> 3's (0).
    grid = fc.laplace((3, 3, 1))
    agg, na = _agg(oracle_lib, grid, _agg_keys([0, 8], 9))
    assert na == 2 and agg.tolist() == [0, 0, 0, 0, 0, 1, 0, 1, 1]
    # centre first: every cell is within two steps of 4, one aggregate
    agg, na = _agg(oracle_lib, grid, _agg_keys([4], 9))
    assert na == 1 and agg.tolist() == [0] * 9
    # a cell with no coupling (the pinned-reference case) is its own root
    c = fc.laplace((3, 3, 1))
    iso = fc.Case("iso", c.shape, c.n, c.owner, c.neighbour, c.diag, c.upper.copy(), c.lower.copy(), c.b)
    for f in range(iso.F):
        if iso.owner[f] == 0:
            iso.upper[f] = iso.lower[f] = 0.0
    agg, na = _agg(oracle_lib, iso, _agg_keys([4], 9))
    assert na == 2 and agg[0] == 0 and np.all(agg[1:] == 1)


def _parallel_mis2(S, key):
    """The parallel rule on the strength graph S (scipy CSR, no diagonal):
    every round each undecided unknown takes the largest (state, key) over
    its closed distance-2 neighbourhood; it joins when that is itself, and
    drops out when that is a root.  Written independently of the oracle's
    sequential greedy; both must give the same set."""
    n = S.shape[0]
    state = np.ones(n, dtype=np.int64)  # 0 out, 1 undecided, 2 root
    G = (S + sp.identity(n, format="csr")).tocsr()
    G2 = (G @ G).tocsr()
    G2.sort_indices()
    key = key.astype(np.uint64)
    while np.any(state == 1):
        tup = list(zip(state.tolist(), key.tolist()))
        best = []
        for i in range(n):
            nbr = G2.indices[G2.indptr[i]:G2.indptr[i + 1]]
            best.append(max(nbr, key=lambda j: tup[j]))
        new = state.copy()
        for i in range(n):
            if state[i] != 1:
                continue
            if best[i] == i:
                new[i] = 2
            elif state[best[i]] == 2:
                new[i] = 0
        state = new
    return np.flatnonzero(state == 2)


@pytest.mark.parametrize("make", [lambda: fc.laplace((7, 6, 5)), lambda: fc.varcoef((8, 7, 6), seed=3),
                                  lambda: fc.cavity((9, 8, 4)), lambda: _ring(11)])
@pytest.mark.parametrize("theta", [0.0, 0.08])
def test_a1_mis2_properties_and_parallel_rule(oracle_lib, make, theta):
    """Roots from the oracle equal the parallel rule's; no two roots within
    two strong steps; every unknown within two steps of a root; each
    aggregate holds its root and every unknown next to it, and its members
    lie within two steps of the root; priorities from SplitMix64."""
    c = make()
    A = _csr_ldu(c)
    d = A.diagonal()
    key = np.array([oracle_lib.amg_priority(1, 0, i) for i in range(c.n)], dtype=np.uint64)
    agg, na = oracle_lib.aggregate(A.indptr, A.indices, A.data, theta, seed=1, level=0)
    agg2, _ = oracle_lib.aggregate(A.indptr, A.indices, A.data, theta, key=key)
    assert np.array_equal(agg, agg2)
    C = A.tocoo()
    keep = (C.row != C.col) & (C.data != 0) & (np.abs(C.data) >= theta * np.sqrt(np.abs(d[C.row] * d[C.col])))
    S = sp.csr_matrix((np.ones(keep.sum()), (C.row[keep], C.col[keep])), shape=A.shape)
    roots = _parallel_mis2(S, key)
    assert na == roots.size and np.array_equal(agg[roots], np.arange(na))
    G = (S + sp.identity(c.n, format="csr")).tocsr()
    within2 = (G @ G).tocsr() != 0
    R = within2[roots][:, roots].toarray()
    assert np.array_equal(R, np.eye(na, dtype=bool))             # independent at distance 2
    assert np.all(np.asarray(within2[:, roots].sum(axis=1)).ravel() >= 1)  # maximal
    near = S[roots].toarray().astype(bool)
    for a, r in enumerate(roots):
        assert agg[r] == a
        assert np.all(agg[np.flatnonzero(near[a])] == a)
        members = np.flatnonzero(agg == a)
        assert np.all(within2[r, members].toarray())


@pytest.mark.parametrize("make", [lambda: fc.laplace((16, 16, 16)), lambda: fc.varcoef((14, 12, 10), seed=3),
                                  lambda: fc.cavity((16, 16, 6))])
def test_a2_partition(oracle_lib, make):
    h = oracle_lib.AMG(make())
    for l in range(h.levels - 1):
        agg = h.aggregates(l)
        nc = h.level_info(l)["n_coarse"]
        assert agg.min() == 0 and agg.max() == nc - 1
        assert np.all(np.bincount(agg, minlength=nc) > 0)


# ---------------------------------------------------------------- A3 - A5
@pytest.mark.parametrize("make", [lambda: fc.laplace((12, 12, 12)), lambda: fc.varcoef((14, 12, 10), seed=3),
                                  lambda: fc.cavity((16, 16, 6))])
def test_a3_a4_a5_prolongator_galerkin_omega(oracle_lib, make):
    h = oracle_lib.AMG(make(), coarse_size=16)
    assert h.levels >= 3
    for l in range(h.levels - 1):
        A = _csr(*h.export(l, "A"))
        P = _csr(*h.export(l, "P"))
        Ac = _csr(*h.export(l + 1, "A"))
        d = A.diagonal()
        lam = np.max(np.asarray(abs(A).sum(axis=1)).ravel() / d)
        w = h.level_info(l)["omega"]
        assert w == pytest.approx(4.0 / (3.0 * lam), rel=1e-14)
        rows = np.asarray(P.sum(axis=1)).ravel()
        expect = 1.0 - w * np.asarray(A.sum(axis=1)).ravel() / d
        assert np.allclose(rows, expect, rtol=0, atol=1e-13)
        ref = (P.T @ A @ P).toarray()
        assert np.allclose(Ac.toarray(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.allclose(Ac.toarray(), Ac.toarray().T, atol=1e-12 * np.abs(ref).max())


# ---------------------------------------------------------------- A6, A7
def test_a6_single_level_is_exact(oracle_lib):
    c = fc.varcoef((5, 4, 3), seed=2)
    h = oracle_lib.AMG(c, coarse_size=1000)
    assert h.levels == 1
    x = h.vcycle(c.b)
    xs = np.linalg.solve(dense(c), c.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-12


@pytest.mark.parametrize("make", [lambda: fc.laplace((10, 10, 10)), lambda: fc.varcoef((12, 10, 8), seed=3),
                                  lambda: fc.cavity((12, 12, 4))])
def test_a7_cycle_spd_and_contracting(oracle_lib, make):
    c = make()
    h = oracle_lib.AMG(c, coarse_size=8)
    assert h.levels >= 3
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(c.n), rng.standard_normal(c.n)
    Mu, Mv = h.vcycle(u), h.vcycle(v)
    assert v @ Mu == pytest.approx(u @ Mv, rel=1e-11)
    for _ in range(3):
        y = rng.standard_normal(c.n)
        assert y @ h.vcycle(y) > 0
    A = dense(c)
    e = rng.standard_normal(c.n)
    for _ in range(60):  # power iteration on E = I - M A
        e = e - h.vcycle(A @ e)
        nrm = np.linalg.norm(e)
        e /= nrm
    assert nrm < 0.9


# ---------------------------------------------------------------- A8
@pytest.mark.parametrize("make", [lambda: fc.laplace((12, 12, 12)), lambda: fc.varcoef((13, 11, 9), seed=6),
                                  lambda: fc.cavity((14, 14, 5))])
def test_a8_pcg_reaches_dense_solution(oracle_lib, make):
    c = make()
    h = oracle_lib.AMG(c, coarse_size=16)
    x, st = h.pcg(c.b, tol=1e-12, maxit=200)
    assert st["status"] == 0
    xs = np.linalg.solve(dense(c), c.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-9
    assert st["true_rel_res"] <= 1e-12 * 1.01


def test_a8_iteration_counts(oracle_lib):
    for c, jac_min in ((fc.laplace((32, 32, 32)), 200), (fc.varcoef((32, 32, 32), seed=2), 200)):
        h = oracle_lib.AMG(c)
        _, st = h.pcg(c.b, tol=1e-8, maxit=500)
        _, sj = oracle_lib.cg(c, c.b, tol=1e-8)
        assert st["status"] == 0 and sj["iters"] >= jac_min
        assert st["iters"] <= sj["iters"] / 8
    c = fc.laplace((64, 64, 64))
    _, st = oracle_lib.AMG(c).pcg(c.b, tol=1e-8, maxit=500)
    assert st["status"] == 0 and 14 <= st["iters"] <= 42


# ---------------------------------------------------------------- A9
@pytest.mark.parametrize("make", [lambda: fc.laplace((12, 12, 12)), lambda: fc.varcoef((13, 11, 9), seed=6),
                                  lambda: fc.cavity((14, 14, 5))])
def test_a9_pipelined_equals_standard(oracle_lib, make):
    c = make()
    h = oracle_lib.AMG(c, coarse_size=16)
    for k in (1, 3, 8):
        xs, _ = h.pcg(c.b, tol=0.0, maxit=k)
        xp, sp = h.pcg(c.b, tol=0.0, maxit=k, pipelined=True)
        assert sp["iters"] == k
        assert np.linalg.norm(xp - xs) / np.linalg.norm(xs) <= 1e-10
    x, st = h.pcg(c.b, tol=1e-12, maxit=200, pipelined=True)
    _, s2 = h.pcg(c.b, tol=1e-12, maxit=200)
    assert st["status"] == 0 and abs(st["iters"] - s2["iters"]) <= 1
    xd = np.linalg.solve(dense(c), c.b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-9


# ---------------------------------------------------------------- R
def _levels(h):
    out = []
    for l in range(h.levels):
        lv = {"A": h.export(l, "A"), "info": h.level_info(l)}
        if l + 1 < h.levels:
            lv["P"] = h.export(l, "P")
            lv["agg"] = h.aggregates(l)
        out.append(lv)
    return out


def _scaled(case, f):
    return fc.Case(case.name, case.shape, case.n, case.owner, case.neighbour, f * case.diag, f * case.upper,
                   f * case.lower, case.b)


@pytest.mark.parametrize("make", [lambda: fc.varcoef((14, 12, 10), seed=3), lambda: fc.cavity((16, 16, 6))])
def test_r1_r2_refresh_same_and_scaled(oracle_lib, make):
    c = make()
    h = oracle_lib.AMG(c, coarse_size=16)
    before = _levels(h)
    h.refresh(c)
    same = _levels(h)
    for a, b in zip(before, same):
        assert a["info"] == b["info"]
        for key in ("A", "P"):
            if key in a:
                for u, v in zip(a[key][:3], b[key][:3]):
                    assert np.array_equal(u, v)
        if "agg" in a:
            assert np.array_equal(a["agg"], b["agg"])
    h.refresh(_scaled(c, 2.0))
    for l, (a, b) in enumerate(zip(before, _levels(h))):
        assert a["info"]["omega"] == b["info"]["omega"]
        assert np.array_equal(a["A"][2] * 2.0, b["A"][2]), l
        if "P" in a:
            assert np.array_equal(a["P"][2], b["P"][2]), l
            assert np.array_equal(a["agg"], b["agg"]), l


@pytest.mark.parametrize("pair", [(lambda: fc.varcoef((14, 12, 10), seed=3, permute=False),
                                   lambda: fc.varcoef((14, 12, 10), seed=9, permute=False)),
                                  (lambda: fc.laplace((12, 12, 12)), lambda: fc.varcoef((12, 12, 12), seed=5,
                                                                                      permute=False))])
def test_r3_refresh_other_coefficients(oracle_lib, pair):
    c1, c2 = pair[0](), pair[1]()
    assert np.array_equal(c1.owner, c2.owner) and np.array_equal(c1.neighbour, c2.neighbour)
    h = oracle_lib.AMG(c1, coarse_size=16)
    aggs = [h.aggregates(l) for l in range(h.levels - 1)]
    sizes = [h.level_info(l)["n"] for l in range(h.levels)]
    h.refresh(c2)
    assert [h.level_info(l)["n"] for l in range(h.levels)] == sizes
    A = _csr_ldu(c2)
    for l in range(h.levels - 1):
        assert np.array_equal(h.aggregates(l), aggs[l])
        Al = _csr(*h.export(l, "A"))
        assert np.allclose(Al.toarray(), A.toarray(), rtol=0, atol=1e-12 * abs(A).max())
        d = A.diagonal()
        lam = np.max(np.asarray(abs(A).sum(axis=1)).ravel() / d)
        w = h.level_info(l)["omega"]
        assert w == pytest.approx(4.0 / (3.0 * lam), rel=1e-14)
        n, nc = A.shape[0], sizes[l + 1]
        Pt = sp.csr_matrix((np.ones(n), aggs[l], np.arange(n + 1)), shape=(n, nc))
        S = sp.identity(n) - w * sp.diags(1.0 / d) @ A
        P_ref = (S @ Pt).toarray()
        P = _csr(*h.export(l, "P")).toarray()
        assert np.allclose(P, P_ref, rtol=0, atol=1e-13)
        Ac_ref = sp.csr_matrix(P_ref).T @ A @ sp.csr_matrix(P_ref)
        Ac = _csr(*h.export(l + 1, "A"))
        assert np.allclose(Ac.toarray(), Ac_ref.toarray(), rtol=0, atol=1e-12 * abs(Ac_ref).max())
        A = Ac
    # the refreshed cycle: symmetric positive definite, error propagator contracting
    n = c2.n
    M = np.column_stack([h.vcycle(e) for e in np.eye(n)])
    assert np.allclose(M, M.T, atol=1e-10 * np.abs(M).max())
    assert np.linalg.eigvalsh((M + M.T) / 2).min() > 0
    E = np.eye(n) - M @ dense(c2)
    assert np.max(np.abs(np.linalg.eigvals(E))) < 1.0
