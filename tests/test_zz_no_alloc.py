"""fvpcg_solve_noalloc (work buffers in the library's fixed device array, no
allocation) through the C ABI against fvpcg_solve on the same inputs: the
same kernels in the same order, so the iterates agree bit for bit.  Two
calls in a row, the second on a smaller system; the size limit; b = 0 and a
warm start."""
import numpy as np
import pytest

import fvcases as fc
from tests.gpu_util import DevCase, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1505_07630_amd as fv

    fv.lib()
    return fv


def _both(fv, dc, method, tol=1e-10, maxit=20000, x0=None):
    import torch

    xa = torch.zeros_like(dc.b) if x0 is None else x0.clone()
    xb = torch.zeros_like(dc.b) if x0 is None else x0.clone()
    _, sa = fv.solve(dc.A, dc.b, x=xa, tol=tol, maxit=maxit, method=method)
    _, sb = fv.solve_noalloc(dc.A, dc.b, xb, tol=tol, maxit=maxit, method=method)
    return xa.cpu().numpy(), sa, xb.cpu().numpy(), sb


@pytest.mark.parametrize("method", ["pipecg", "cg", "pipecg_literal"])
def test_noalloc_matches_solve_two_calls(fv, method):
    for shape, seed in (((40, 36, 30), 3), ((17, 13, 11), 9)):  # the second call is smaller
        say("noalloc", method, shape)
        case = fc.varcoef(shape, seed=seed)
        dc = DevCase(case)
        xa, sa, xb, sb = _both(fv, dc, method)
        assert sa["status"] == sb["status"] == 0
        assert sa["iters"] == sb["iters"]
        assert np.array_equal(xa, xb)
        assert sa["true_rel_res"] == sb["true_rel_res"]
        dc.close()


def test_noalloc_edge_cases(fv):
    import torch

    say("noalloc edge cases")
    case = fc.varcoef((12, 11, 10), seed=5)
    dc = DevCase(case)
    # b = 0: x = 0, no iterations
    z = torch.zeros_like(dc.b)
    x = torch.ones_like(dc.b)
    _, st = fv.solve_noalloc(dc.A, z, x, tol=1e-8)
    assert st["status"] == 0 and st["iters"] == 0 and torch.count_nonzero(x).item() == 0
    # warm start and an iteration limit, against the allocating solve
    x0 = to_dev(np.random.default_rng(4).standard_normal(case.n))
    xa, sa, xb, sb = _both(fv, dc, "pipecg", tol=1e-14, maxit=17, x0=x0)
    assert sa["status"] == sb["status"] == 1 and sa["iters"] == sb["iters"] == 17
    assert np.array_equal(xa, xb)
    dc.close()
    # one cell over the limit is refused before any work
    n = fv.NOALLOC_MAX_CELLS + 1
    owner = np.arange(n - 1, dtype=np.int32)
    big = fc.Case("line", (n, 1, 1), n, owner, owner + 1, np.full(n, 3.0), -np.ones(n - 1), -np.ones(n - 1),
                  np.ones(n))
    db = DevCase(big)
    xb = torch.zeros_like(db.b)
    with pytest.raises(fv.FVPCGError) as e:
        fv.solve_noalloc(db.A, db.b, xb)
    assert e.value.code == fv.INVALID_ARG and "work space" in str(e.value)
    db.close()
