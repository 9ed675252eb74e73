"""Batched solves (one persistent, graph-captured launch for many uneven
systems): every system against the oracle on that system alone."""
import os

import numpy as np
import pytest

import fvcases as fc
from tests.gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu

PARITY = 1e-10


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


@pytest.fixture(autouse=True)
def _tune_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("FVPCG_TUNE_CACHE", str(tmp_path / "tune.json"))


def dev_batch(fv, bt, symmetric=True):
    import torch

    B = fv.Batch(bt.cell_off, bt.face_off, to_dev(bt.owner, torch.int32), to_dev(bt.neighbour, torch.int32),
                 to_dev(bt.diag), to_dev(bt.upper), None if symmetric else to_dev(bt.lower))
    return B, to_dev(bt.b)


def per_system(bt, v):
    return [v[bt.cell_off[s]:bt.cell_off[s + 1]] for s in range(bt.nsys)]


@pytest.mark.parametrize("method", ["pipecg", "cg"])
def test_batched_matches_oracle_per_system(fv, orc, method):
    say("batched small", method)
    bt = fc.batch(24, 3, 21, seed=5)
    B, b = dev_batch(fv, bt)
    x, stats, code = fv.solve_batched(B, b, tol=1e-8, method=method)
    assert code == 0 and all(s["status"] == 0 for s in stats)
    xs = per_system(bt, x.cpu().numpy())
    for s, case in enumerate(bt.cases):
        k = stats[s]["iters"]
        if method == "cg":
            _, so = orc.cg(case, case.b, tol=1e-8, maxit=20000)
            xo, _ = orc.cg(case, case.b, tol=0.0, maxit=k)
        else:
            _, so = orc.pipecg(case, case.b, tol=1e-8, maxit=20000, folded=True)
            xo, _ = orc.pipecg(case, case.b, tol=0.0, maxit=k, folded=True)
        assert abs(so["iters"] - k) <= 2, (s, so["iters"], k)
        assert rel(xs[s], xo) <= PARITY, s
        assert stats[s]["b_norm"] == pytest.approx(np.linalg.norm(case.b), rel=1e-13)
        assert stats[s]["true_rel_res"] <= 10 * 1e-8
    B.close()


def test_batched_unpreconditioned_and_warm_start(fv, orc):
    say("batched none / warm start")
    bt = fc.batch(6, 4, 9, seed=8)
    B, b = dev_batch(fv, bt)
    x, stats, code = fv.solve_batched(B, b, tol=1e-8, method="pipecg", precond="none")
    assert code == 0
    # warm start at the converged answer: zero iterations everywhere
    x2, stats2, code2 = fv.solve_batched(B, b, x=x.clone(), tol=1e-7, method="cg")
    assert code2 == 0 and all(s["iters"] == 0 for s in stats2)
    B.close()


def test_batched_determinism_and_graph_replay(fv):
    say("batched determinism")
    import torch

    bt = fc.batch(16, 5, 15, seed=9)
    B, b = dev_batch(fv, bt)
    outs = []
    for _ in range(3):  # same arguments: the captured graph is replayed
        x = torch.zeros_like(b)
        x, stats, code = fv.solve_batched(B, b, x=x, tol=1e-9, method="pipecg")
        torch.cuda.synchronize()
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    B.close()


def test_batched_status_per_system(fv):
    say("batched statuses")
    import torch

    bt = fc.batch(5, 4, 8, seed=3)
    b = bt.b.copy()
    b[bt.cell_off[2]:bt.cell_off[3]] = 0.0  # one system with b = 0
    B, _ = dev_batch(fv, bt)
    x = torch.ones(bt.cell_off[-1], dtype=torch.float64, device="cuda")
    x, stats, code = fv.solve_batched(B, to_dev(b), x=x, tol=1e-12, maxit=3, method="cg")
    assert code == 1
    assert stats[2]["status"] == 0 and stats[2]["iters"] == 0
    assert torch.count_nonzero(x[bt.cell_off[2]:bt.cell_off[3]]).item() == 0
    assert all(stats[s]["status"] == 1 and stats[s]["iters"] == 3 for s in (0, 1, 3, 4))
    B.close()


def test_batched_invalid_addressing(fv):
    say("batched invalid")
    import torch

    bt = fc.batch(3, 3, 4, seed=1)
    nb = bt.neighbour.copy()
    nb[bt.face_off[1] - 1] = bt.cell_off[1] - bt.cell_off[0]  # one past system 0's last cell
    with pytest.raises(fv.FVPCGError) as e:
        fv.Batch(bt.cell_off, bt.face_off, to_dev(bt.owner, torch.int32), to_dev(nb, torch.int32), to_dev(bt.diag),
                 to_dev(bt.upper))
    assert e.value.code == fv.INVALID_MESH


def test_batched_backward(fv, orc):
    say("batched backward")
    bt = fc.batch(8, 4, 10, seed=5)
    B, b = dev_batch(fv, bt)
    x, _, _ = fv.solve_batched(B, b, tol=1e-13, method="cg")
    g = x - to_dev(bt.x_target)
    grads, stats, code = fv.solve_batched_backward(B, x, g, tol=1e-13, method="cg")
    assert code == 0
    xs = per_system(bt, x.cpu().numpy())
    gs = per_system(bt, g.cpu().numpy())
    for s, case in enumerate(bt.cases):
        lam, _ = orc.cg(case, gs[s], tol=1e-14, maxit=100000)
        gd, gu, gl = orc.adjoint_grads(case, xs[s], lam)
        cs, ce = bt.cell_off[s], bt.cell_off[s + 1]
        fs, fe = bt.face_off[s], bt.face_off[s + 1]
        assert rel(grads["b"][cs:ce].cpu().numpy(), lam) <= 1e-9
        assert rel(grads["diag"][cs:ce].cpu().numpy(), gd) <= 1e-9
        assert rel(grads["upper"][fs:fe].cpu().numpy(), gu + gl) <= 1e-9
    B.close()


def test_autotune_cache_written(fv, tmp_path):
    say("autotune cache")
    bt = fc.batch(10, 4, 12, seed=2)
    B, b = dev_batch(fv, bt)
    fv.solve_batched(B, b, tol=1e-8, method="pipecg")
    path = os.environ["FVPCG_TUNE_CACHE"]
    text = open(path).read()
    assert "gfx950/nsys10" in text
    B.close()


# ------------------------------------------------------------------ workgroup teams

@pytest.mark.parametrize("method", ["pipecg", "cg"])
def test_batched_teams_match_oracle(fv, orc, monkeypatch, method):
    """Teams forced on: one 40^3 system far above a workgroup's fair share
    (split over many workgroups) beside small queued systems; every system
    against the oracle at its iteration count, bitwise reproducible."""
    say("batched teams", method)
    import torch

    monkeypatch.setenv("FVPCG_TUNE", "0")
    monkeypatch.setenv("FVPCG_BATCH_TEAMS", "1")
    big = fc.varcoef((40, 40, 40), seed=4)
    small = fc.batch(12, 3, 12, seed=6).cases
    bt = fc.concat([big] + small)
    B, b = dev_batch(fv, bt)
    runs = []
    for _ in range(2):
        x, stats, code = fv.solve_batched(B, b, x=torch.zeros_like(b), tol=1e-9, method=method)
        assert code == 0 and all(st["status"] == 0 for st in stats)
        runs.append(x.cpu().numpy())
    assert np.array_equal(runs[0], runs[1])
    xs = per_system(bt, runs[0])
    for s, case in enumerate(bt.cases):
        k = stats[s]["iters"]
        if method == "cg":
            _, so = orc.cg(case, case.b, tol=1e-9, maxit=20000)
            xo, _ = orc.cg(case, case.b, tol=0.0, maxit=k)
        else:
            _, so = orc.pipecg(case, case.b, tol=1e-9, maxit=20000, folded=True)
            xo, _ = orc.pipecg(case, case.b, tol=0.0, maxit=k, folded=True)
        assert abs(so["iters"] - k) <= 2, (s, so["iters"], k)
        assert rel(xs[s], xo) <= PARITY, s
        tr = np.linalg.norm(case.b - orc.spmv(case, xs[s])) / np.linalg.norm(case.b)
        assert stats[s]["true_rel_res"] == pytest.approx(tr, rel=1e-6)
    B.close()


def test_batched_team_barrier_timeout_reports_error(fv, monkeypatch):
    """A zero barrier timeout (set from the host) makes a team's bounded wait
    give up: every workgroup leaves and the call reports DEVICE_ERROR; a batch
    with the normal timeout then solves."""
    say("batched team timeout")
    import torch

    monkeypatch.setenv("FVPCG_TUNE", "0")
    monkeypatch.setenv("FVPCG_BATCH_TEAMS", "1")
    monkeypatch.setenv("FVPCG_BATCH_BARRIER_TIMEOUT_MS", "0")
    bt = fc.concat([fc.varcoef((32, 32, 32), seed=4)])
    B, b = dev_batch(fv, bt)
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_batched(B, b, tol=1e-9, method="pipecg")
    assert e.value.code == fv.DEVICE_ERROR and "barrier" in str(e.value)
    B.close()
    monkeypatch.delenv("FVPCG_BATCH_BARRIER_TIMEOUT_MS")
    B, b = dev_batch(fv, bt)
    x, stats, code = fv.solve_batched(B, b, x=torch.zeros_like(b), tol=1e-9, method="pipecg")
    assert code == 0 and stats[0]["true_rel_res"] <= 1e-8
    B.close()


# ------------------------------------------------------------------ full size

@pytest.fixture(scope="module")
def batch256():
    say("generating batch256")
    return fc.make("batch256")


@pytest.mark.parametrize("method", ["cg", "pipecg"])
def test_batch256_full_size(fv, orc, batch256, method):
    """The 256-system workload (edges 16..64, 22M cells): every system's FP64
    true residual recomputed by the oracle's product, and the smallest
    systems at equal iteration count against the oracle."""
    bt = batch256
    say("batch256 solve", method, bt.cell_off[-1])
    B, b = dev_batch(fv, bt)
    x, stats, code = fv.solve_batched(B, b, tol=1e-8, method=method)
    assert code == 0
    xs = per_system(bt, x.cpu().numpy())
    order = np.argsort([c.n for c in bt.cases])
    for s, case in enumerate(bt.cases):
        tr = np.linalg.norm(case.b - orc.spmv(case, xs[s])) / np.linalg.norm(case.b)
        assert tr <= 1.5e-8, s
        assert stats[s]["true_rel_res"] == pytest.approx(tr, rel=1e-6)
    for s in order[:3]:
        case = bt.cases[s]
        if method == "cg":
            xo, _ = orc.cg(case, case.b, tol=0.0, maxit=stats[s]["iters"])
        else:
            xo, _ = orc.pipecg(case, case.b, tol=0.0, maxit=stats[s]["iters"], folded=True)
        assert rel(xs[s], xo) <= PARITY
    B.close()


def test_batch256_backward_fd(fv, orc, batch256):
    """Gradient of L = 0.5||x - x_t||^2 w.r.t. b and the face coefficients
    (upper = lower, the symmetric storage's combined gradient) of all 256
    systems, by the batched adjoint, each checked by central differences
    (h = 1e-6) along a random direction: for the face coefficients the batch
    is created again from upper +- h du (diagonal unchanged) and solved."""
    import torch

    bt = batch256
    say("batch256 backward")
    B, b = dev_batch(fv, bt)
    xt = to_dev(bt.x_target)
    x, _, _ = fv.solve_batched(B, b, tol=1e-13, method="cg")
    grads, _, code = fv.solve_batched_backward(B, x, x - xt, tol=1e-13, method="cg")
    assert code == 0
    rng = np.random.default_rng(5)
    h = 1e-6
    # along b
    db = to_dev(rng.standard_normal(bt.cell_off[-1]))
    pred = torch.dot(grads["b"], db).item()
    Lp = 0.5 * torch.sum((fv.solve_batched(B, b + h * db, tol=1e-13, method="cg")[0] - xt) ** 2).item()
    Lm = 0.5 * torch.sum((fv.solve_batched(B, b - h * db, tol=1e-13, method="cg")[0] - xt) ** 2).item()
    say(f"[fd] batch256 along b: adjoint {pred:.10e} central difference {(Lp - Lm) / (2 * h):.10e}")
    assert (Lp - Lm) / (2 * h) == pytest.approx(pred, rel=1e-5)
    B.close()
    # along the face coefficients
    owner, nb = to_dev(bt.owner, torch.int32), to_dev(bt.neighbour, torch.int32)
    diag, upper = to_dev(bt.diag), to_dev(bt.upper)
    du = to_dev(rng.standard_normal(bt.face_off[-1]))
    pred_u = torch.dot(grads["upper"], du).item()

    def loss(up):
        Bh = fv.Batch(bt.cell_off, bt.face_off, owner, nb, diag, up)
        xh = fv.solve_batched(Bh, b, tol=1e-13, method="cg")[0]
        Bh.close()
        return 0.5 * torch.sum((xh - xt) ** 2).item()

    fd = (loss(upper + h * du) - loss(upper - h * du)) / (2 * h)
    say(f"[fd] batch256 along the face coefficients: adjoint {pred_u:.10e} central difference {fd:.10e}")
    assert fd == pytest.approx(pred_u, rel=1e-5)
