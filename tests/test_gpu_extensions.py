"""Mixed-precision refinement, adjoint gradients and the autograd Function on
the GPU, against the CPU oracle."""
import numpy as np
import pytest

import fvcases as fc
from tests.gpu_util import DevCase, rel, say, to_dev

pytestmark = pytest.mark.gpu


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


# ------------------------------------------------------------------ mixed precision

MIXED_CASES = {
    "varcoef16": lambda: fc.varcoef((16, 16, 16), seed=2),
    "varcoef32_rcm": lambda: fc.varcoef((32, 32, 32), seed=2),
    "varcoef48_rcm": lambda: fc.varcoef((48, 48, 48), seed=2),
    "laplace32": lambda: fc.laplace((32, 32, 32)),
    "ragged_9x7x5": lambda: fc.varcoef((9, 7, 5), seed=6),
}


@pytest.mark.parametrize("name", list(MIXED_CASES))
def test_mixed_matches_fp64_solution(fv, orc, name):
    """FP32 inner / FP64 outer refinement: error against the oracle's FP64
    solution (standard CG to 1e-12) <= 1e-8; FP64 true residual, recomputed
    by the oracle's product, <= the outer tolerance."""
    say("mixed", name)
    case = MIXED_CASES[name]()
    dc = DevCase(case, fp32_copy=True)
    x, st = fv.solve_mixed(dc.A, dc.b, outer_tol=1e-10, inner_tol=1e-5)
    assert st["status"] == 0, st
    xg = x.cpu().numpy()
    xs, _ = orc.cg(case, case.b, tol=1e-12, maxit=100000)
    assert rel(xg, xs) <= 1e-8
    tr = np.linalg.norm(case.b - orc.spmv(case, xg)) / np.linalg.norm(case.b)
    assert tr <= 1e-10 * 1.01
    assert st["true_rel_res"] == pytest.approx(tr, rel=1e-6, abs=1e-15)
    assert 1 <= st["outer_iters"] <= 10
    # the oracle's refinement reaches the same fixed point
    xr, sr = orc.refine(case, case.b, outer_tol=1e-10, inner_tol=1e-5)
    assert sr["status"] == 0 and rel(xr, xs) <= 1e-8
    dc.close()


def test_mixed_hard_case_does_not_diverge(fv, orc):
    """The graded cavity is close to the limit of FP32 refinement (each outer
    step contracts the residual by roughly kappa * eps_fp32, near 1 here):
    the solver either converges or stops with NOT_CONVERGED once an outer
    step no longer reduces the FP64 residual; it never returns a worse x."""
    say("mixed hard case")
    case = fc.cavity((48, 48, 12))
    dc = DevCase(case, fp32_copy=True)
    x, st = fv.solve_mixed(dc.A, dc.b, outer_tol=1e-10, inner_tol=1e-5, max_outer=30)
    assert st["status"] in (0, 1)
    xg = x.cpu().numpy()
    tr = np.linalg.norm(case.b - orc.spmv(case, xg)) / np.linalg.norm(case.b)
    assert tr <= 1e-4
    if st["status"] == 0:
        xs, _ = orc.cg(case, case.b, tol=1e-12, maxit=100000)
        assert rel(xg, xs) <= 1e-7
    dc.close()


def test_mixed_zero_rhs_and_warm_start(fv, orc):
    say("mixed zero rhs")
    import torch

    case = fc.varcoef((10, 10, 10), seed=3)
    dc = DevCase(case, fp32_copy=True)
    x = torch.ones(case.n, dtype=torch.float64, device="cuda")
    x, st = fv.solve_mixed(dc.A, torch.zeros_like(dc.b), x=x)
    assert st["status"] == 0 and torch.count_nonzero(x).item() == 0
    xs, _ = orc.cg(case, case.b, tol=1e-13, maxit=10000)
    x, st = fv.solve_mixed(dc.A, dc.b, x=to_dev(xs))
    assert st["status"] == 0 and st["outer_iters"] == 0 and st["iters"] == 0
    dc.close()


def test_mixed_outer_limit(fv):
    say("mixed outer limit")
    case = fc.varcoef((16, 16, 16), seed=2)
    dc = DevCase(case, fp32_copy=True)
    x, st = fv.solve_mixed(dc.A, dc.b, outer_tol=1e-14, inner_tol=1e-5, max_outer=1)
    assert st["status"] == 1 and st["outer_iters"] == 1
    dc.close()


# ------------------------------------------------------------------ mixed, reliable updates

# (case, tolerance): the graded cavity is ill-conditioned enough that a 1e-10
# residual leaves an error above 1e-8, so it is solved to 1e-12
RELIABLE_CASES = {k: (v, 1e-10) for k, v in MIXED_CASES.items()}
RELIABLE_CASES["cavity_24x24x8"] = (lambda: fc.cavity((24, 24, 8)), 1e-12)


@pytest.mark.parametrize("name", list(RELIABLE_CASES))
def test_mixed_reliable_matches_fp64_solution(fv, orc, name):
    """FP32 pipelined recurrences re-anchored to the FP64 residual every 10
    iterations: error against the oracle's FP64 solution (standard CG to
    1e-13) <= 1e-8, FP64 true residual (the oracle's product) <= tol, and an
    FP32 iteration count within 3 update periods or 15% of the oracle running
    the same algorithm (FP32 rounding orders differ)."""
    say("mixed reliable", name)
    make, tol = RELIABLE_CASES[name]
    case = make()
    dc = DevCase(case, fp32_copy=True)
    x, st = fv.solve_mixed_reliable(dc.A, dc.b, tol=tol, update_every=10)
    assert st["status"] == 0, st
    xg = x.cpu().numpy()
    xs, _ = orc.cg(case, case.b, tol=1e-13, maxit=100000)
    assert rel(xg, xs) <= 1e-8
    tr = np.linalg.norm(case.b - orc.spmv(case, xg)) / np.linalg.norm(case.b)
    assert tr <= tol * 1.01
    assert st["true_rel_res"] == pytest.approx(tr, rel=1e-6, abs=1e-15)
    xo, so = orc.mixed_reliable(case, case.b, tol=tol, update_every=10)
    assert so["status"] == 0
    assert abs(st["iters"] - so["iters"]) <= max(30, 0.15 * so["iters"]), (st["iters"], so["iters"])
    assert st["outer_iters"] >= -(-st["iters"] // 10)
    dc.close()


def test_mixed_reliable_edge_cases(fv, orc):
    say("mixed reliable edge cases")
    import torch

    case = fc.varcoef((10, 10, 10), seed=3)
    dc = DevCase(case, fp32_copy=True)
    x = torch.ones(case.n, dtype=torch.float64, device="cuda")
    x, st = fv.solve_mixed_reliable(dc.A, torch.zeros_like(dc.b), x=x)
    assert st["status"] == 0 and torch.count_nonzero(x).item() == 0 and st["iters"] == 0
    xs, _ = orc.cg(case, case.b, tol=1e-13, maxit=10000)
    x, st = fv.solve_mixed_reliable(dc.A, dc.b, x=to_dev(xs), tol=1e-10)
    assert st["status"] == 0 and st["iters"] == 0 and st["outer_iters"] == 0
    # iteration limit, and an update after every iteration
    x, st = fv.solve_mixed_reliable(dc.A, dc.b, tol=1e-14, update_every=4, maxit=10)
    assert st["status"] == 1 and st["iters"] == 10 and st["outer_iters"] == 3
    x, st = fv.solve_mixed_reliable(dc.A, dc.b, tol=1e-10, update_every=1)
    assert st["status"] == 0 and st["outer_iters"] == st["iters"]
    assert rel(x.cpu().numpy(), xs) <= 1e-8
    # unattainable tolerance: the FP64 residual stagnates, the solve ends
    x, st = fv.solve_mixed_reliable(dc.A, dc.b, tol=1e-30, update_every=5, maxit=100000)
    assert st["status"] == 1 and st["iters"] < 100000
    tr = np.linalg.norm(case.b - orc.spmv(case, x.cpu().numpy())) / np.linalg.norm(case.b)
    assert tr <= 1e-13
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_mixed_reliable(dc.A, dc.b, update_every=0)
    assert e.value.code == fv.INVALID_ARG
    dc.close()
    dc = DevCase(case)  # no FP32 copy
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_mixed_reliable(dc.A, dc.b)
    assert e.value.code == fv.UNSUPPORTED
    dc.close()


# ------------------------------------------------------------------ adjoint

def _loss_setup(orc, case):
    xs, _ = orc.cg(case, case.b, tol=1e-14, maxit=100000)
    return xs


@pytest.mark.parametrize("method", ["cg", "pipecg"])
def test_backward_matches_oracle(fv, orc, method):
    say("backward", method)
    case = fc.batch(3, 10, 14, seed=5).cases[1]
    dc = DevCase(case)
    x, st = fv.solve(dc.A, dc.b, tol=1e-12, method="cg")
    g = x - to_dev(case.x_target)
    grads, sb = fv.solve_backward(dc.A, x, g, tol=1e-12, method=method)
    xo = x.cpu().numpy()
    lam, _ = orc.cg(case, g.cpu().numpy(), tol=1e-14, maxit=100000)
    gd, gu, gl = orc.adjoint_grads(case, xo, lam)
    assert rel(grads["b"].cpu().numpy(), lam) <= 1e-9
    assert rel(grads["diag"].cpu().numpy(), gd) <= 1e-9
    # one coefficient per face (matrix created with lower == NULL): the sum
    assert rel(grads["upper"].cpu().numpy(), gu + gl) <= 1e-9
    dc.close()


def test_backward_nonsymmetric_storage(fv, orc):
    say("backward explicit lower")
    case = fc.batch(2, 9, 9, seed=5).cases[0]
    dc = DevCase(case, symmetric=False)
    x, _ = fv.solve(dc.A, dc.b, tol=1e-12, method="cg")
    g = x - to_dev(case.x_target)
    grads, _ = fv.solve_backward(dc.A, x, g, tol=1e-12, method="cg")
    lam, _ = orc.cg(case, g.cpu().numpy(), tol=1e-14, maxit=100000)
    gd, gu, gl = orc.adjoint_grads(case, x.cpu().numpy(), lam)
    assert rel(grads["upper"].cpu().numpy(), gu) <= 1e-9
    assert rel(grads["lower"].cpu().numpy(), gl) <= 1e-9
    dc.close()


def test_backward_central_differences(fv, orc):
    """Directional derivative of L = 0.5||x - x_t||^2 along random symmetric
    directions in (diag, face coefficients, b), central differences with
    h = 1e-6 through GPU forward solves."""
    say("backward fd")
    import torch

    case = fc.batch(2, 8, 8, seed=5).cases[0]
    dc = DevCase(case)
    xt = to_dev(case.x_target)

    def loss(diag, upper, b):
        A = fv.Matrix(dc.mesh, diag, upper)
        x, st = fv.solve(A, b, tol=1e-14, maxit=20000, method="cg")
        A.close()
        return 0.5 * torch.sum((x - xt) ** 2).item(), x

    L0, x = loss(dc.diag, dc.upper, dc.b)
    grads, _ = fv.solve_backward(dc.A, x, x - xt, tol=1e-14, maxit=20000, method="cg")
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(3):
        dd = to_dev(rng.standard_normal(case.n))
        du = to_dev(rng.standard_normal(case.F))
        db = to_dev(rng.standard_normal(case.n))
        pred = (torch.dot(grads["diag"], dd) + torch.dot(grads["upper"], du) + torch.dot(grads["b"], db)).item()
        Lp, _ = loss(dc.diag + h * dd, dc.upper + h * du, dc.b + h * db)
        Lm, _ = loss(dc.diag - h * dd, dc.upper - h * du, dc.b - h * db)
        fd = (Lp - Lm) / (2 * h)
        assert fd == pytest.approx(pred, rel=1e-5)
    dc.close()


def test_autograd_function(fv, orc):
    say("autograd")
    import torch

    case = fc.batch(2, 7, 7, seed=5).cases[0]
    dc = DevCase(case)
    diag = dc.diag.clone().requires_grad_(True)
    upper = dc.upper.clone().requires_grad_(True)
    b = dc.b.clone().requires_grad_(True)
    x = fv.fv_solve(diag, upper, None, b, dc.mesh, tol=1e-13, method="cg")
    loss = 0.5 * torch.sum((x - to_dev(case.x_target)) ** 2)
    loss.backward()
    xo, _ = orc.cg(case, case.b, tol=1e-14, maxit=100000)
    assert rel(x.detach().cpu().numpy(), xo) <= 1e-10
    lam, _ = orc.cg(case, xo - case.x_target, tol=1e-14, maxit=100000)
    gd, gu, gl = orc.adjoint_grads(case, xo, lam)
    assert rel(b.grad.cpu().numpy(), lam) <= 1e-9
    assert rel(diag.grad.cpu().numpy(), gd) <= 1e-9
    assert rel(upper.grad.cpu().numpy(), gu + gl) <= 1e-9
    # conductivity chain rule through differentiable torch assembly
    k = torch.exp(to_dev(np.random.default_rng(3).standard_normal(case.F))).requires_grad_(True)
    own = torch.from_numpy(case.owner.astype(np.int64)).cuda()
    nbr = torch.from_numpy(case.neighbour.astype(np.int64)).cuda()
    d0 = (dc.diag - torch.zeros_like(dc.diag).index_add_(0, own, -dc.upper).index_add_(0, nbr, -dc.upper))
    dk = d0 + torch.zeros_like(dc.diag).index_add(0, own, k).index_add(0, nbr, k)
    x = fv.fv_solve(dk, -k, None, dc.b, dc.mesh, tol=1e-13, method="cg")
    (0.5 * torch.sum((x - to_dev(case.x_target)) ** 2)).backward()
    xk = x.detach().cpu().numpy()
    ck = fc.Case("k", case.shape, case.n, case.owner, case.neighbour, dk.detach().cpu().numpy(),
                 -k.detach().cpu().numpy(), -k.detach().cpu().numpy(), case.b)
    lk, _ = orc.cg(ck, xk - case.x_target, tol=1e-14, maxit=100000)
    closed = -(lk[case.owner] - lk[case.neighbour]) * (xk[case.owner] - xk[case.neighbour])
    assert rel(k.grad.cpu().numpy(), closed) <= 1e-8
    dc.close()


def test_single_asymmetric_face_detected(fv):
    """One face with lower != upper among 774k (more faces than the
    symmetry check's threads, so each thread checks several): CG refuses
    the matrix; restoring that face makes it acceptable again.  Faces at
    the start, the middle and the end of the list."""
    say("single asymmetric face")
    import torch

    case = fc.varcoef((64, 64, 64), seed=3)
    assert case.F > 1024 * 256
    dc = DevCase(case, symmetric=False)
    try:
        for f in (0, case.F // 2 + 7, case.F - 1):
            lower = dc.upper.clone()
            lower[f] *= 1.0 + 2.0 ** -40
            dc.A.update(dc.diag, dc.upper, lower)
            with pytest.raises(fv.FVPCGError) as e:
                fv.solve(dc.A, dc.b, tol=1e-8, method="pipecg")
            assert e.value.code == fv.UNSUPPORTED, f
            dc.A.update(dc.diag, dc.upper, dc.upper.clone())
            _, st = fv.solve(dc.A, dc.b, tol=1e-8, method="pipecg")
            assert st["status"] == 0, f
    finally:
        dc.close()


def test_nonsymmetric_values_refused_by_cg_paths(fv):
    """CG, its pipelined forms, both mixed solvers, the adjoint and the
    batched solver assume A = A^T: with lower = upper / 2 on every face each
    returns UNSUPPORTED (the adjoint would otherwise solve with A instead of
    A^T); BiCGSTAB solves the same system."""
    say("non-symmetric values refused")
    import torch

    base = fc.batch(1, 6, 6, seed=2).cases[0]
    ns = fc.Case("ns", base.shape, base.n, base.owner, base.neighbour, base.diag, base.upper, 0.5 * base.upper,
                 base.b)
    dn = DevCase(ns, symmetric=False, fp32_copy=True)
    x = torch.zeros_like(dn.b)
    calls = [lambda: fv.solve(dn.A, dn.b, method="cg"), lambda: fv.solve(dn.A, dn.b, method="pipecg"),
             lambda: fv.solve(dn.A, dn.b, method="pipecg_literal"), lambda: fv.solve_mixed(dn.A, dn.b),
             lambda: fv.solve_mixed_reliable(dn.A, dn.b), lambda: fv.solve_backward(dn.A, x, dn.b)]
    for call in calls:
        with pytest.raises(fv.FVPCGError) as e:
            call()
        assert e.value.code == fv.UNSUPPORTED
    xb, st = fv.solve_bicgstab(dn.A, dn.b, tol=1e-10)
    assert st["status"] == 0
    B = fv.Batch(np.array([0, ns.n]), np.array([0, ns.F]), dn.owner, dn.nb, dn.diag, dn.upper, dn.lower)
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_batched(B, dn.b)
    assert e.value.code == fv.UNSUPPORTED
    B.close()
    # the same storage with equal values is accepted
    dn.A.update(dn.diag, dn.upper, dn.upper.clone())
    _, st = fv.solve(dn.A, dn.b, tol=1e-10, method="cg")
    assert st["status"] == 0
    dn.close()
