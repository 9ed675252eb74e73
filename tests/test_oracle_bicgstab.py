"""Pins of the oracle's BiCGSTAB (oracle/bicgstab.c) and of the momentum
workload's generator, against facts that do not come from the oracle's code:

B1 the first iteration of a 2x2 non-symmetric system worked by hand
   (tests/golden/bicgstab_2x2.json): alpha, omega, x_1 and r_1
B2 finite termination: a 2x2 system (two eigenvalues) is solved exactly in
   two iterations; a wrong beta breaks it
B3 a diagonal matrix with two distinct values needs at most two iterations
   without preconditioning, and one (half step) with Jacobi
B4 non-symmetric momentum systems: the solution equals the dense solve of
   the LDU matrix built by direct indexing (row owner holds upper), within
   the bound the tolerance gives; the transposed matrix's solution differs
B5 right preconditioning: Jacobi BiCGSTAB on A has the scalars of plain
   BiCGSTAB on A D^-1 (built in the test), and x = D^-1 y
B6 on a symmetric positive definite system it reaches CG's solution
B7 zero right-hand side, exact initial guess, maxit, and the breakdown of a
   skew 2x2 system where (rhat, A r0) = 0
B8 the momentum generator: zero net flux per cell, row sums h^3/dt plus the
   wall terms, off-diagonals <= 0 with lower != upper
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import fvcases as fc
from tests.helpers import dense_from_ldu

pytestmark = pytest.mark.cpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bicgstab_2x2.json")


def _two_by_two():
    g = json.load(open(GOLDEN))
    A = (g["n"], np.array(g["owner"]), np.array(g["neighbour"]), np.array(g["diag"]), np.array(g["upper"]),
         np.array(g["lower"]))
    return g, A, np.array(g["b"])


def _sys(oracle_lib, n, owner, nb, diag, upper, lower):
    return oracle_lib._Sys(n, owner, nb, diag, upper, lower)


def _f(s):
    return float(Fraction(s))


def test_b1_first_iteration_by_hand(oracle_lib):
    g, A, b = _two_by_two()
    S = _sys(oracle_lib, *A)
    assert np.array_equal(dense_from_ldu(*A), np.array(g["dense"], dtype=float))
    x, st, h = oracle_lib.bicgstab(S, b, tol=0.0, maxit=1, precond="none", history=True)
    it1 = g["iteration_1"]
    assert st["iters"] == 1 and st["status"] == oracle_lib.NOT_CONVERGED
    assert h["alpha"][0] == pytest.approx(_f(it1["alpha"]), rel=1e-15)
    assert h["omega"][0] == pytest.approx(_f(it1["omega"]), rel=1e-15)
    assert np.allclose(x, [_f(v) for v in it1["x"]], rtol=1e-15, atol=0)
    r1 = np.array([_f(v) for v in it1["r"]])
    assert h["res"][1] == pytest.approx(np.linalg.norm(r1), rel=1e-14)
    assert h["res"][0] == pytest.approx(np.sqrt(5.0), rel=1e-15)


def test_b2_two_by_two_terminates_in_two(oracle_lib):
    g, A, b = _two_by_two()
    S = _sys(oracle_lib, *A)
    x, st = oracle_lib.bicgstab(S, b, tol=1e-14, maxit=50, precond="none")
    assert st["status"] == oracle_lib.OK
    assert st["iters"] == g["iterations_to_solution"]
    assert np.allclose(x, [_f(v) for v in g["solution"]], rtol=0, atol=1e-15)
    # Jacobi: (A D^-1) is 2x2 as well
    x, st = oracle_lib.bicgstab(S, b, tol=1e-14, maxit=50, precond="jacobi")
    assert st["status"] == oracle_lib.OK and st["iters"] <= 2
    assert np.allclose(x, [_f(v) for v in g["solution"]], rtol=0, atol=1e-15)


def test_b3_diagonal_matrices(oracle_lib):
    n = 40
    d = np.where(np.arange(n) % 2 == 0, 2.0, 5.0)
    b = np.random.default_rng(1).uniform(-1, 1, n)
    e = np.zeros(0, dtype=np.int32)
    S = _sys(oracle_lib, n, e, e, d, np.zeros(0), np.zeros(0))
    x, st = oracle_lib.bicgstab(S, b, tol=1e-14, maxit=10, precond="none")
    assert st["status"] == oracle_lib.OK and st["iters"] <= 2
    assert np.allclose(x, b / d, rtol=1e-14, atol=0)
    x, st, h = oracle_lib.bicgstab(S, b, tol=1e-14, maxit=10, precond="jacobi", history=True)
    assert st["status"] == oracle_lib.OK and st["iters"] == 1
    assert h["alpha"][0] == pytest.approx(1.0, rel=1e-15) and h["omega"][0] == 0.0  # half-step exit
    assert np.allclose(x, b / d, rtol=1e-15, atol=0)


@pytest.mark.parametrize("shape,permute", [((7, 6, 5), False), ((9, 8, 7), True), ((5, 5, 12), True)])
def test_b4_dense_solve(oracle_lib, shape, permute):
    c = fc.momentum(shape, permute=permute)
    A = dense_from_ldu(c.n, c.owner, c.neighbour, c.diag, c.upper, c.lower)
    xs = np.linalg.solve(A, c.b)
    tol = 1e-11
    x, st = oracle_lib.bicgstab(oracle_lib.system(c), c.b, tol=tol, maxit=1000)
    assert st["status"] == oracle_lib.OK
    assert np.linalg.norm(c.b - A @ x) <= tol * np.linalg.norm(c.b) * (1 + 1e-6)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) <= 2 * kappa * tol * np.linalg.norm(xs)
    # transposition matters: the transposed system has another solution
    xt = np.linalg.solve(A.T, c.b)
    assert np.linalg.norm(x - xt) > 1e3 * np.linalg.norm(x - xs)


def test_b5_right_preconditioning_identity(oracle_lib):
    c = fc.momentum((6, 7, 8), permute=True)
    d = c.diag
    Sj = oracle_lib.system(c)
    # A D^-1: unit diagonal, column c scaled by 1/d_c
    Ss = _sys(oracle_lib, c.n, c.owner, c.neighbour, np.ones(c.n), c.upper / d[c.neighbour], c.lower / d[c.owner])
    xj, sj, hj = oracle_lib.bicgstab(Sj, c.b, tol=1e-12, maxit=500, precond="jacobi", history=True)
    y, sy, hy = oracle_lib.bicgstab(Ss, c.b, tol=1e-12, maxit=500, precond="none", history=True)
    assert sj["iters"] == sy["iters"]
    assert np.allclose(hj["alpha"], hy["alpha"], rtol=1e-9, atol=0)
    assert np.allclose(hj["omega"], hy["omega"], rtol=1e-9, atol=0)
    assert np.allclose(xj, y / d, rtol=1e-9, atol=1e-14)


def test_b6_symmetric_matches_cg(oracle_lib):
    c = fc.varcoef((8, 7, 6), permute=True)
    S = oracle_lib.system(c)
    xb, sb = oracle_lib.bicgstab(S, c.b, tol=1e-12, maxit=2000)
    xc, sc = oracle_lib.cg(S, c.b, tol=1e-12, maxit=2000)
    assert sb["status"] == oracle_lib.OK and sc["status"] == oracle_lib.OK
    assert np.allclose(xb, xc, rtol=0, atol=1e-9 * np.abs(xc).max())


def test_b7_edges_and_breakdown(oracle_lib):
    c = fc.momentum((5, 4, 3))
    S = oracle_lib.system(c)
    x, st = oracle_lib.bicgstab(S, np.zeros(c.n), x0=np.ones(c.n))
    assert st["status"] == oracle_lib.OK and st["iters"] == 0 and not x.any()
    A = dense_from_ldu(c.n, c.owner, c.neighbour, c.diag, c.upper, c.lower)
    xs = np.linalg.solve(A, c.b)
    x, st = oracle_lib.bicgstab(S, c.b, x0=xs, tol=1e-8)
    assert st["status"] == oracle_lib.OK and st["iters"] == 0
    x, st = oracle_lib.bicgstab(S, c.b, tol=1e-14, maxit=3)
    assert st["status"] == oracle_lib.NOT_CONVERGED and st["iters"] == 3
    # [[0, 1], [-1, 0]] with b = e_1: v = A r0 is orthogonal to rhat = r0
    K = _sys(oracle_lib, 2, np.array([0]), np.array([1]), np.zeros(2), np.array([1.0]), np.array([-1.0]))
    x, st = oracle_lib.bicgstab(K, np.array([1.0, 0.0]), tol=1e-10, precond="none")
    assert st["status"] == oracle_lib.BREAKDOWN and st["iters"] == 0


def test_b8_momentum_generator():
    shape = (10, 9, 8)
    c = fc.momentum(shape, permute=False, nu=0.02, co=1.5)
    h = 1.0 / shape[0]
    dt = 1.5 * h
    # upper - lower = max(F, 0) - max(-F, 0) = F, the face flux
    flux = c.upper - c.lower
    div = np.zeros(c.n)
    np.add.at(div, c.owner, flux)
    np.add.at(div, c.neighbour, -flux)
    assert np.abs(div).max() < 1e-15
    assert np.abs(flux).max() > 0.1 * h * h
    A = dense_from_ldu(c.n, c.owner, c.neighbour, c.diag, c.upper, c.lower)
    walls = np.zeros(c.n)
    for side in ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax"):
        walls[fc.mesh.boundary_cells(shape, side)] += 2 * 0.02 * h
    assert np.allclose(A.sum(axis=1), h ** 3 / dt + walls, rtol=1e-12, atol=1e-17)
    assert (c.upper < 0).all() and (c.lower < 0).all()
    assert (c.upper != c.lower).sum() > 0.5 * c.F
    cp = fc.momentum(shape, permute=True, nu=0.02, co=1.5)
    assert sorted(cp.diag) == pytest.approx(sorted(c.diag), rel=0, abs=0)
