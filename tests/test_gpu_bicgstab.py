"""BiCGSTAB on the GPU (fvpcg_solve_bicgstab, fvpcg_solve_bicgstab_multi)
against the oracle's (oracle/bicgstab.c) on the non-symmetric momentum
systems: the iterate after a fixed number of iterations, solves to
tolerance, the hand-worked 2x2 case, the half-step exit, determinism, edge
cases, several right-hand sides solved together, and the 192^3 workload."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import fvcases as fc
from tests.gpu_util import DevCase, rel, say, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bicgstab_2x2.json")


@pytest.fixture(scope="module")
def fv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1505_07630_amd as fv

    fv.lib()
    return fv


@pytest.fixture(scope="module")
def orc():
    import oracle

    oracle.build(force=False)
    return oracle


def _small(fv, n, owner, nb, diag, upper, lower):
    import torch

    mesh = fv.Mesh(n, to_dev(np.asarray(owner), torch.int32), to_dev(np.asarray(nb), torch.int32))
    A = fv.Matrix(mesh, to_dev(np.asarray(diag, dtype=np.float64)), to_dev(np.asarray(upper, dtype=np.float64)),
                  to_dev(np.asarray(lower, dtype=np.float64)))
    return mesh, A


# (200, 200, 2) in natural order has bandwidth 40,000 > 32,767: the int32
# column layout instead of int16 offsets.
@pytest.mark.parametrize("shape,permute,precond", [((17, 13, 11), False, "jacobi"), ((24, 20, 18), True, "jacobi"),
                                                   ((24, 20, 18), True, "none"), ((200, 200, 2), False, "jacobi")])
def test_fixed_iterations_match_oracle(fv, orc, shape, permute, precond):
    """Three iterations (tol = 0): the iterate within 1e-12 of the oracle's
    (only the summation order of the inner products differs)."""
    say("bicgstab fixed iterations", shape, permute, precond)
    case = fc.momentum(shape, permute=permute)
    dc = DevCase(case, symmetric=False)
    x, st = fv.solve_bicgstab(dc.A, dc.b, tol=0.0, maxit=3, precond=precond)
    xo, so = orc.bicgstab(case, case.b, tol=0.0, maxit=3, precond=precond)
    assert st["status_name"] == "NOT_CONVERGED" and st["iters"] == 3 == so["iters"]
    assert rel(x.cpu().numpy(), xo) <= 1e-12
    assert st["rel_res"] == pytest.approx(so["rel_res"], rel=1e-10)
    dc.close()


@pytest.mark.parametrize("shape,permute,precond", [((17, 13, 11), False, "jacobi"), ((40, 36, 30), True, "jacobi"),
                                                   ((40, 36, 30), True, "none"), ((9, 70, 5), True, "jacobi"),
                                                   ((200, 200, 2), False, "jacobi")])
def test_solve_matches_oracle(fv, orc, shape, permute, precond):
    """To 1e-12: status OK, iterations within 2 of the oracle's, the solution
    within 1e-9 of the oracle's (both are within tol * cond(A D^-1) ~ 1e-10
    of the exact one), and the true residual at the tolerance."""
    say("bicgstab solve", shape, permute, precond)
    case = fc.momentum(shape, permute=permute)
    dc = DevCase(case, symmetric=False)
    tol = 1e-12
    x, st = fv.solve_bicgstab(dc.A, dc.b, tol=tol, maxit=2000, precond=precond)
    xo, so = orc.bicgstab(case, case.b, tol=tol, maxit=2000, precond=precond)
    assert st["status_name"] == "OK" and so["status"] == orc.OK
    assert abs(st["iters"] - so["iters"]) <= 2
    assert rel(x.cpu().numpy(), xo) <= 1e-9
    assert st["true_rel_res"] <= 10 * tol
    xn = x.cpu().numpy()
    r = case.b - orc.spmv(case, xn)
    assert np.linalg.norm(r) / np.linalg.norm(case.b) == pytest.approx(st["true_rel_res"], rel=1e-3)
    dc.close()


def test_warm_start_matches_oracle(fv, orc):
    """From a non-zero x0 (the solution perturbed), single and two-component
    solves: three fixed iterations within 1e-12 of the oracle's from the same
    x0, and solves to 1e-12 within 1e-9."""
    import torch

    say("bicgstab warm start")
    case = fc.momentum((19, 17, 13), permute=True)
    dc = DevCase(case, symmetric=False)
    B = _rhs3(case)[:2]
    g = np.random.default_rng(21)
    X0 = np.stack([orc.bicgstab(case, B[k], tol=1e-12, maxit=2000)[0] * (1 + 0.1 * g.standard_normal(case.n))
                   for k in range(2)])
    x, st = fv.solve_bicgstab(dc.A, to_dev(B[0]), x=to_dev(X0[0]), tol=0.0, maxit=3)
    xo, _ = orc.bicgstab(case, B[0], x0=X0[0], tol=0.0, maxit=3)
    assert st["iters"] == 3 and rel(x.cpu().numpy(), xo) <= 1e-12
    X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(B), x=to_dev(X0), tol=1e-12, maxit=2000)
    for k in range(2):
        xo, so = orc.bicgstab(case, B[k], x0=X0[k], tol=1e-12, maxit=2000)
        assert sts[k]["status_name"] == "OK" and abs(sts[k]["iters"] - so["iters"]) <= 2
        assert rel(X[k].cpu().numpy(), xo) <= 1e-9
        assert 0 < sts[k]["r0_norm"] < np.linalg.norm(B[k])  # the warm start is closer than x = 0
    dc.close()


def test_two_by_two_by_hand(fv):
    """The hand-worked 2x2 system (tests/golden): the first iterate, then the
    exact solution after two iterations."""
    g = json.load(open(GOLDEN))
    say("bicgstab 2x2")
    mesh, A = _small(fv, g["n"], g["owner"], g["neighbour"], g["diag"], g["upper"], g["lower"])
    b = to_dev(np.array(g["b"]))
    x, st = fv.solve_bicgstab(A, b, tol=0.0, maxit=1, precond="none")
    x1 = np.array([float(Fraction(v)) for v in g["iteration_1"]["x"]])
    assert st["iters"] == 1
    assert np.allclose(x.cpu().numpy(), x1, rtol=1e-15, atol=0)
    x, st = fv.solve_bicgstab(A, b, tol=1e-14, maxit=10, precond="none")
    assert st["status_name"] == "OK" and st["iters"] == g["iterations_to_solution"]
    assert np.allclose(x.cpu().numpy(), [float(Fraction(v)) for v in g["solution"]], rtol=0, atol=1e-15)
    A.close()
    mesh.close()


def test_half_step_exit_on_a_diagonal_matrix(fv):
    """M = D makes A M^-1 = I: s = 0 after the first half step, x = b / d."""
    import torch

    say("bicgstab diagonal")
    n = 3000
    d = np.random.default_rng(4).uniform(1.0, 5.0, n)
    bb = np.random.default_rng(5).uniform(-1.0, 1.0, n)
    mesh = fv.Mesh(n, torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"))
    A = fv.Matrix(mesh, to_dev(d), torch.zeros(0, dtype=torch.float64, device="cuda"),
                  torch.zeros(0, dtype=torch.float64, device="cuda"))
    x, st = fv.solve_bicgstab(A, to_dev(bb), tol=1e-14, maxit=10)
    assert st["status_name"] == "OK" and st["iters"] == 1
    assert np.allclose(x.cpu().numpy(), bb / d, rtol=1e-15, atol=0)
    A.close()
    mesh.close()


def test_deterministic_and_symmetric_handle(fv):
    """Two solves give the same bits; a matrix created without lower (one
    coefficient per face) gives the same bits as one created with lower =
    upper."""
    import torch

    say("bicgstab determinism")
    case = fc.varcoef((20, 18, 16), permute=True)
    ds = DevCase(case, symmetric=True)
    da = DevCase(case, symmetric=False)
    x1, s1 = fv.solve_bicgstab(ds.A, ds.b, tol=1e-10)
    x2, s2 = fv.solve_bicgstab(ds.A, ds.b, tol=1e-10)
    x3, s3 = fv.solve_bicgstab(da.A, da.b, tol=1e-10)
    assert s1["status_name"] == "OK"
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    assert s1["iters"] == s2["iters"] == s3["iters"]
    ds.close()
    da.close()


def test_edges(fv, orc):
    import torch

    say("bicgstab edges")
    case = fc.momentum((6, 5, 4))
    dc = DevCase(case, symmetric=False)
    x = torch.ones(case.n, dtype=torch.float64, device="cuda")
    x, st = fv.solve_bicgstab(dc.A, torch.zeros_like(dc.b), x=x)
    assert st["status_name"] == "OK" and st["iters"] == 0 and not x.any()
    xs, _ = orc.bicgstab(case, case.b, tol=1e-15, maxit=1000)
    x, st = fv.solve_bicgstab(dc.A, dc.b, x=to_dev(xs), tol=1e-8)
    assert st["status_name"] == "OK" and st["iters"] == 0
    x, st = fv.solve_bicgstab(dc.A, dc.b, tol=1e-8, maxit=0)
    assert st["status_name"] == "NOT_CONVERGED" and st["iters"] == 0
    with pytest.raises(fv.FVPCGError):
        fv.solve_bicgstab(dc.A, dc.b, tol=-1.0)
    with pytest.raises(fv.FVPCGError):
        fv.solve_bicgstab(dc.A, dc.b, x=dc.b)
    # an unknown preconditioner code is refused at the C boundary
    import ctypes

    xx = torch.zeros_like(dc.b)
    code = fv.lib().fvpcg_solve_bicgstab(dc.A.handle, ctypes.c_void_p(dc.b.data_ptr()),
                                         ctypes.c_void_p(xx.data_ptr()), 1e-8, 100, 7, None, None)
    assert code == -1 and b"preconditioner" in fv.lib().fvpcg_last_error()
    dc.close()
    # skew 2x2: (rhat, A r0) = 0 at the first iteration
    mesh, A = _small(fv, 2, [0], [1], [0.0, 0.0], [1.0], [-1.0])
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_bicgstab(A, to_dev(np.array([1.0, 0.0])), tol=1e-10, precond="none")
    assert e.value.code == -3
    with pytest.raises(fv.FVPCGError):  # zero diagonal: no Jacobi
        fv.solve_bicgstab(A, to_dev(np.array([1.0, 0.0])), tol=1e-10, precond="jacobi")
    A.close()
    mesh.close()


def _rhs3(case):
    return np.stack([case.b, fc.momentum_rhs(case, 1), fc.momentum_rhs(case, 2)])


def test_multi_matches_single_and_oracle(fv, orc):
    """Three components solved together to 1e-12: each with the iteration
    count of its own single solve and within 1e-12 of it, and within 1e-9 of
    the oracle's solution."""
    say("bicgstab multi vs single")
    case = fc.momentum((24, 20, 18), permute=True)
    dc = DevCase(case, symmetric=False)
    B = _rhs3(case)
    X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(B), tol=1e-12, maxit=2000)
    for k in range(3):
        xs, ss = fv.solve_bicgstab(dc.A, to_dev(B[k]), tol=1e-12, maxit=2000)
        xo, so = orc.bicgstab(case, B[k], tol=1e-12, maxit=2000)
        assert sts[k]["status_name"] == "OK"
        assert sts[k]["iters"] == ss["iters"]
        assert rel(X[k].cpu().numpy(), xs.cpu().numpy()) <= 1e-12
        assert rel(X[k].cpu().numpy(), xo) <= 1e-9
        assert abs(sts[k]["iters"] - so["iters"]) <= 2
    dc.close()


@pytest.mark.parametrize("shape,permute", [((17, 13, 11), True), ((200, 200, 2), False)])
def test_multi_fixed_iterations_vs_oracle(fv, orc, shape, permute):
    say("bicgstab multi fixed iterations", shape)
    case = fc.momentum(shape, permute=permute)
    dc = DevCase(case, symmetric=False)
    B = _rhs3(case)[:2]
    for precond in ("jacobi", "none"):
        X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(B), tol=0.0, maxit=3, precond=precond)
        for k in range(2):
            xo, so = orc.bicgstab(case, B[k], tol=0.0, maxit=3, precond=precond)
            assert sts[k]["iters"] == 3 and sts[k]["status_name"] == "NOT_CONVERGED"
            assert rel(X[k].cpu().numpy(), xo) <= 1e-12
    dc.close()


def test_multi_components_stop_independently(fv, orc):
    """Four components: a zero right-hand side (x = 0 at once), an exact
    initial guess (no iteration, x untouched) and two that iterate; then a
    maxit that stops every component."""
    import torch

    say("bicgstab multi independent stops")
    case = fc.momentum((14, 12, 10), permute=True)
    dc = DevCase(case, symmetric=False)
    R3 = _rhs3(case)
    xs, _ = orc.bicgstab(case, R3[1], tol=1e-15, maxit=1000)
    B = np.stack([R3[0], np.zeros(case.n), R3[1], R3[2]])
    X0 = np.stack([np.zeros(case.n), np.ones(case.n), xs, np.zeros(case.n)])
    X = to_dev(X0)
    X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(B), x=X, tol=1e-10, maxit=1000)
    assert [s["status_name"] for s in sts] == ["OK"] * 4
    assert sts[1]["iters"] == 0 and not X[1].any()
    assert sts[2]["iters"] == 0 and torch.equal(X[2], to_dev(xs))
    for k in (0, 3):
        x1, s1 = fv.solve_bicgstab(dc.A, to_dev(B[k]), tol=1e-10, maxit=1000)
        assert sts[k]["iters"] == s1["iters"] > 0
        assert rel(X[k].cpu().numpy(), x1.cpu().numpy()) <= 1e-12
    X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(R3), tol=1e-14, maxit=4)
    assert [s["iters"] for s in sts] == [4, 4, 4]
    assert all(s["status_name"] == "NOT_CONVERGED" for s in sts)
    # nrhs outside 1..4 is refused at the C boundary
    import ctypes

    xx = torch.zeros(5 * case.n, dtype=torch.float64, device="cuda")
    bb = torch.ones(5 * case.n, dtype=torch.float64, device="cuda")
    code = fv.lib().fvpcg_solve_bicgstab_multi(dc.A.handle, 5, ctypes.c_void_p(bb.data_ptr()),
                                               ctypes.c_void_p(xx.data_ptr()), 1e-8, 100, 1, None, None)
    assert code == -1 and b"nrhs" in fv.lib().fvpcg_last_error()
    dc.close()


def test_multi_breakdown_is_confined(fv):
    """[[0, 1, 0], [-1, 0, 0], [0, 0, 1]]: b = e1 breaks down at once
    ((r, A r) = 0 on the skew block), b = e3 converges in one half step to
    x = e3.  Solved together, the call reports the breakdown, the first
    component's x stays at x0 and the second is exact."""
    import torch

    say("bicgstab multi breakdown")
    mesh, A = _small(fv, 3, [0], [1], [0.0, 0.0, 1.0], [1.0], [-1.0])
    B = to_dev(np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]))
    X = torch.zeros_like(B)
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_bicgstab_multi(A, B, x=X, tol=1e-12, precond="none")
    assert e.value.code == -3
    assert not X[0].any()
    assert torch.equal(X[1], to_dev(np.array([0.0, 0.0, 1.0])))
    A.close()
    mesh.close()


@pytest.fixture(scope="module")
def momentum192():
    say("generating momentum192")
    return fc.make("momentum192")


def test_momentum192(fv, orc, momentum192):
    """The 192^3 workload in the benchmark's launch configuration: three
    iterations against the oracle element by element, then the solve to 1e-8
    with its true residual recomputed by the oracle's product."""
    case = momentum192
    say("momentum192 fixed iterations", case.n)
    dc = DevCase(case, symmetric=False)
    x, st = fv.solve_bicgstab(dc.A, dc.b, tol=0.0, maxit=3)
    xo, so = orc.bicgstab(case, case.b, tol=0.0, maxit=3)
    assert st["iters"] == 3
    assert rel(x.cpu().numpy(), xo) <= 1e-12
    say("momentum192 solve")
    x, st = fv.solve_bicgstab(dc.A, dc.b, tol=case.tol, maxit=5000)
    assert st["status_name"] == "OK"
    r = case.b - orc.spmv(case, x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(case.b) <= case.tol * 1.01
    say("momentum192 three components")
    B = _rhs3(case)
    X, sts = fv.solve_bicgstab_multi(dc.A, to_dev(B), tol=case.tol, maxit=5000)
    assert sts[0]["iters"] == st["iters"]
    assert rel(X[0].cpu().numpy(), x.cpu().numpy()) <= 1e-12
    for k in range(3):
        assert sts[k]["status_name"] == "OK"
        r = B[k] - orc.spmv(case, X[k].cpu().numpy())
        assert np.linalg.norm(r) / np.linalg.norm(B[k]) <= case.tol * 1.01
    dc.close()
