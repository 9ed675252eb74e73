"""Pins of the oracle's transient diffusion (oracle/transient.c) against
facts fixed by the finite-volume implicit-Euler scheme, independent of its
code:

T1 row sums of the assembled operator: A 1 = V/dt + bdiag (internal face
   terms cancel), and A is symmetric with upper = -k w
T2 k = 0: one step is the pointwise update (V/dt T + bsrc) / (V/dt + bdiag)
T3 no Dirichlet faces and no source: the total heat sum V T is conserved
T4 one step equals the dense solve of the assembled system
T5 with dt -> infinity one step is the steady solution (dense solve of the
   steady operator)
"""
import dataclasses

import numpy as np
import pytest

import fvcases as fc
from tests.helpers import dense_from_ldu

pytestmark = pytest.mark.cpu


def test_t1_row_sums_and_symmetry(oracle_lib):
    t = fc.transient((7, 6, 5), permute=True)
    T = np.random.default_rng(3).standard_normal(t.n)
    diag, upper, b = oracle_lib.assemble_transient(t, T)
    A = dense_from_ldu(t.n, t.owner, t.neighbour, diag, upper, upper)
    assert np.allclose(A @ np.ones(t.n), t.vol / t.dt + t.bdiag, rtol=0, atol=1e-12)
    assert np.array_equal(upper, -t.k_face * t.w_face)
    assert np.allclose(b, t.vol / t.dt * T + t.bsrc, rtol=1e-15, atol=0)


def test_t2_no_conduction_is_pointwise(oracle_lib):
    t = fc.transient((5, 4, 3))
    t = dataclasses.replace(t, k_face=np.zeros(t.F))
    T0 = np.random.default_rng(4).uniform(size=t.n)
    T1, st = oracle_lib.transient_run(t, 1, T0=T0, tol=1e-14)
    expect = (t.vol / t.dt * T0 + t.bsrc) / (t.vol / t.dt + t.bdiag)
    assert st["status"] == 0
    assert np.allclose(T1, expect, rtol=1e-13, atol=0)


def test_t3_heat_is_conserved_without_boundaries(oracle_lib):
    t = fc.transient((8, 7, 6), permute=True)
    t = dataclasses.replace(t, bdiag=np.zeros(t.n), bsrc=np.zeros(t.n))
    T0 = np.random.default_rng(5).uniform(size=t.n)
    T, st = oracle_lib.transient_run(t, 5, T0=T0, tol=1e-13)
    assert st["status"] == 0
    assert (t.vol @ T) == pytest.approx(t.vol @ T0, rel=1e-11)
    assert np.std(T) < np.std(T0)  # diffusion smooths


def test_t4_step_is_the_dense_solve(oracle_lib):
    t = fc.transient((6, 5, 4), permute=True)
    T0 = np.random.default_rng(6).uniform(size=t.n)
    diag, upper, b = oracle_lib.assemble_transient(t, T0)
    A = dense_from_ldu(t.n, t.owner, t.neighbour, diag, upper, upper)
    T1, _ = oracle_lib.transient_run(t, 1, T0=T0, tol=1e-14)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(T1 - xs) / np.linalg.norm(xs) <= 1e-12


def test_t5_large_step_is_steady_state(oracle_lib):
    t = fc.transient((6, 5, 4))
    # steady operator: L + B, assembled by hand from the definitions
    L = np.zeros((t.n, t.n))
    a = t.k_face * t.w_face
    for f in range(t.F):
        o, m = t.owner[f], t.neighbour[f]
        L[o, o] += a[f]
        L[m, m] += a[f]
        L[o, m] -= a[f]
        L[m, o] -= a[f]
    steady = np.linalg.solve(L + np.diag(t.bdiag), t.bsrc)
    T1, _ = oracle_lib.transient_run(t, 1, dt=1e12, tol=1e-14)
    assert np.linalg.norm(T1 - steady) / np.linalg.norm(steady) <= 1e-9
