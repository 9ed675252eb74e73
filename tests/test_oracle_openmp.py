"""The oracle's OpenMP timing build (liboracle_omp.so) against the
single-thread build: CG and pipelined CG (folded, literal, unpreconditioned)
give bitwise the same iterates and statistics for any thread count, because
each row of the product and the tree of every inner product are evaluated in
the single-thread order."""
import numpy as np
import pytest

import fvcases as fc

pytestmark = pytest.mark.cpu


@pytest.fixture(scope="module")
def case():
    return fc.varcoef((24, 22, 20), seed=4)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_openmp_build_is_bitwise_single_thread(oracle_lib, case, threads):
    oracle_lib.set_threads(threads)
    assert oracle_lib.threads(omp=True) == threads
    runs = [("cg", dict(precond="jacobi")), ("cg", dict(precond="none")),
            ("pipecg", dict(precond="jacobi", folded=True)), ("pipecg", dict(precond="jacobi", folded=False)),
            ("pipecg", dict(precond="none", folded=False))]
    for name, kw in runs:
        f = getattr(oracle_lib, name)
        for tol, maxit in ((1e-9, 5000), (0.0, 37)):
            x1, s1 = f(case, case.b, tol=tol, maxit=maxit, **kw)
            xp, sp = f(case, case.b, tol=tol, maxit=maxit, omp=True, **kw)
            assert s1 == sp, (name, kw)
            assert np.array_equal(x1, xp), (name, kw)
    # warm start and the iteration history
    x0 = np.random.default_rng(2).standard_normal(case.n)
    x1, s1, h1 = oracle_lib.cg(case, case.b, x0=x0, tol=1e-8, history=True)
    xp, sp, hp = oracle_lib.cg(case, case.b, x0=x0, tol=1e-8, history=True, omp=True)
    assert s1 == sp and np.array_equal(x1, xp)
    for k in h1:
        assert np.array_equal(h1[k], hp[k])
    assert oracle_lib.threads(omp=False) == 1
