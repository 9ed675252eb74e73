"""Transient diffusion (implicit Euler, laplacianFoam's heat equation) on
the GPU against the oracle (oracle/transient.c): the assembled coefficients
element by element, and the field after a run of time steps."""
import dataclasses

import numpy as np
import pytest

import fvcases as fc
from tests.gpu_util import rel, say, to_dev

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


class DevTransient:
    def __init__(self, fv, t):
        import torch

        self.t = t
        self.mesh = fv.Mesh(t.n, to_dev(t.owner, torch.int32), to_dev(t.neighbour, torch.int32))
        self.k = to_dev(t.k_face)
        self.w = to_dev(t.w_face)
        self.vol = to_dev(t.vol)
        self.bdiag = to_dev(t.bdiag)
        self.bsrc = to_dev(t.bsrc)
        d0, u0, _ = fv.assemble_transient(self.mesh, self.k, self.w, self.vol, self.bdiag, self.bsrc, t.dt,
                                          to_dev(t.T0))
        self.A = fv.Matrix(self.mesh, d0, u0)

    def close(self):
        self.A.close()
        self.mesh.close()


@pytest.mark.parametrize("permute", [False, True])
def test_assembly_matches_oracle(fv, orc, permute):
    say("transient assembly", permute)
    t = fc.transient((11, 9, 7), permute=permute)
    T = np.random.default_rng(2).standard_normal(t.n)
    dt_ = DevTransient(fv, t)
    d, u, b = fv.assemble_transient(dt_.mesh, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, to_dev(T))
    do, uo, bo = orc.assemble_transient(t, T)
    assert np.array_equal(u.cpu().numpy(), uo)
    assert np.max(np.abs(d.cpu().numpy() - do) / np.abs(do)) <= 1e-14
    assert np.max(np.abs(b.cpu().numpy() - bo) / np.maximum(np.abs(bo), 1e-300)) <= 1e-14
    dt_.close()


@pytest.mark.parametrize("method", ["pipecg", "cg"])
def test_run_matches_oracle(fv, orc, method):
    """Five steps, each solved to 1e-12 from the previous field: the field
    within 1e-9 of the oracle's (Jacobi-PCG per step), total iterations
    within 10%."""
    say("transient run", method)
    import torch

    t = fc.transient((14, 12, 10), permute=True)
    dt_ = DevTransient(fv, t)
    T = torch.zeros(t.n, dtype=torch.float64, device="cuda")
    T, st = fv.transient_run(dt_.A, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, 5, T, tol=1e-12,
                             method=method)
    assert st["status"] == 0 and st["outer_iters"] == 5
    To, so = orc.transient_run(t, 5, tol=1e-12)
    assert so["status"] == 0
    assert rel(T.cpu().numpy(), To) <= 1e-9
    assert abs(st["iters"] - so["iters"]) <= 0.1 * so["iters"] + 5
    dt_.close()


def test_heat_conserved_and_edge_cases(fv, orc):
    say("transient conservation")
    import torch

    t = fc.transient((10, 9, 8), permute=True)
    t = dataclasses.replace(t, bdiag=np.zeros(t.n), bsrc=np.zeros(t.n))
    dt_ = DevTransient(fv, t)
    T0 = np.random.default_rng(5).uniform(size=t.n)
    T = to_dev(T0)
    T, st = fv.transient_run(dt_.A, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, 4, T, tol=1e-13)
    Tn = T.cpu().numpy()
    assert st["status"] == 0
    assert (t.vol @ Tn) == pytest.approx(t.vol @ T0, rel=1e-11)
    assert np.std(Tn) < np.std(T0)
    # zero steps: unchanged
    T2 = to_dev(T0)
    T2, st = fv.transient_run(dt_.A, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, 0, T2)
    assert st["outer_iters"] == 0 and np.array_equal(T2.cpu().numpy(), T0)
    with pytest.raises(fv.FVPCGError) as e:
        fv.transient_run(dt_.A, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, 0.0, 1, T2)
    assert e.value.code == fv.INVALID_ARG
    # a matrix with separate lower coefficients is refused
    A2 = fv.Matrix(dt_.mesh, to_dev(t.vol + 6.0), to_dev(-t.k_face), to_dev(-t.k_face))
    with pytest.raises(fv.FVPCGError) as e:
        fv.transient_run(A2, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, 1, T2)
    assert e.value.code == fv.INVALID_ARG
    A2.close()
    dt_.close()


def test_transient192(fv, orc):
    """10 steps at 7.08M cells (lognormal, permuted + RCM), pipelined CG to
    1e-8 per step: every step converges, the field stays within the bounds
    the data allow (T >= 0: T0 = 0, boundary values 0 and 1, non-negative
    source), and one step's assembly matches the oracle at sampled cells."""
    say("transient192 generate")
    import torch

    t = fc.transient((192, 192, 192), permute=True)
    dt_ = DevTransient(fv, t)
    T = torch.zeros(t.n, dtype=torch.float64, device="cuda")
    say("transient192 run")
    T, st = fv.transient_run(dt_.A, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, 10, T, tol=1e-8)
    assert st["status"] == 0 and st["outer_iters"] == 10
    Tn = T.cpu().numpy()
    assert Tn.min() >= -1e-6
    d, u, b = fv.assemble_transient(dt_.mesh, dt_.k, dt_.w, dt_.vol, dt_.bdiag, dt_.bsrc, t.dt, T)
    do, uo, bo = orc.assemble_transient(t, Tn)
    idx = np.random.default_rng(1).integers(0, t.n, 2000)
    assert np.max(np.abs(d.cpu().numpy()[idx] - do[idx]) / np.abs(do[idx])) <= 1e-14
    assert np.max(np.abs(b.cpu().numpy()[idx] - bo[idx]) / np.maximum(np.abs(bo[idx]), 1e-300)) <= 1e-14
    dt_.close()
