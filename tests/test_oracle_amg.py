"""Pins of the oracle's smoothed-aggregation AMG (oracle/amg.c) against facts
fixed by its definition and by linear algebra, independent of its code:

A1 aggregates of a 7-cell line, a 3x3 grid and a weighted ring, worked by hand
A2 every unknown in exactly one aggregate; no empty aggregate
A3 prolongator row sums: P 1 = (I - omega D^-1 A) 1
A4 Galerkin coarse operators equal SciPy's P^T A P
A5 omega = 4 / (3 * Gershgorin bound of D^-1 A), computed by NumPy
A6 one level: the cycle is the exact solve (dense LU)
A7 the cycle is symmetric positive definite and its error propagator
   I - M A contracts (spectral radius < 1, power iteration)
A8 AMG-PCG reaches the dense solution; iteration counts far below Jacobi-PCG
   and, at 64^3, no more than Table pcgs2's GPU AMG-CG count (loose: the
   paper's AMG, boundary conditions and right-hand side are not stated)
A9 AMG-preconditioned pipelined CG: the same iterates as AMG-PCG in exact
   arithmetic (equal at equal count up to rounding), the dense solution
"""
import numpy as np
import pytest
import scipy.sparse as sp

import fvcases as fc
from tests.helpers import dense

pytestmark = pytest.mark.cpu


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


# ---------------------------------------------------------------- A1, A2
def test_a1_aggregates_worked_by_hand(oracle_lib):
    # line: pass 1 takes {0,1} (0 and its only neighbour), skips 2 (neighbour 1
    # taken), takes {2,3,4} around 3, skips 5, takes {5,6} around 6
    h = oracle_lib.AMG(_line(7), coarse_size=1)
    assert h.aggregates(0).tolist() == [0, 0, 1, 1, 1, 2, 2]
    # 3x3 grid, cell i + 3j, every coupling strong.  Pass 1: {0,1,3} around
    # 0; 2 (neighbour 1 taken) and 4 (1, 3 taken) are skipped; 5's neighbours
    # 2, 4, 8 are all free: {2,4,5,8}; 6 (3 taken) and 7 (4 taken) are
    # skipped.  Pass 2: 6's only aggregated neighbour is 3 -> aggregate 0; 7's
    # neighbours 4 and 8 tie at |a| = 1, the first (4) wins -> aggregate 1.
    c = fc.laplace((3, 3, 1))
    h = oracle_lib.AMG(c, coarse_size=1)
    assert h.aggregates(0).tolist() == [0, 0, 1, 0, 1, 1, 0, 1, 1]
    # a ring of 7 with coupling 2 between cells 4 and 5, 1 elsewhere: pass 1
    # makes {0,1,6} and {2,3,4}; 5 is skipped (4 and 6 taken) and pass 2 puts
    # it with its stronger neighbour 4, not with 6
    owner = np.array([0, 0, 1, 2, 3, 4, 5], dtype=np.int32)
    nb = np.array([1, 6, 2, 3, 4, 5, 6], dtype=np.int32)
    up = -np.ones(7)
    up[5] = -2.0
    diag = np.ones(7)
    np.add.at(diag, owner, -up)
    np.add.at(diag, nb, -up)
    ring = fc.Case("ring", (7, 1, 1), 7, owner, nb, diag, up, up.copy(), np.ones(7))
    h = oracle_lib.AMG(ring, coarse_size=1)
    assert h.aggregates(0).tolist() == [0, 0, 1, 1, 1, 1, 0]


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
    assert st["status"] == 0 and st["iters"] <= 28


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
