"""Pins of the oracle's PISO step (oracle/piso.c) against facts fixed by the
finite-volume method and by linear algebra, independent of its code:

S1 momentum matrix: lower - upper = -phi (upwind), symmetric for phi = 0,
   row sums V/dt + wall terms for a divergence-free flux (dense matrix)
S2 Gauss gradient exact for a linear pressure field in interior cells
S3 one step against the same step composed here with dense solves (NumPy)
   of the momentum predictor and of the pinned pressure system
S4 after every corrector the face fluxes are discretely divergence-free
S5 a fluid at rest with a resting lid stays exactly at rest
S6 without the lid the kinetic energy decays at every step (implicit Euler
   with upwind convection and no-slip walls is dissipative)
S7 renumbering the cells (random permutation + RCM, faces re-oriented)
   gives the same fields, cell for cell
S8 the reference cell's pressure is exactly 0; the lid drives the flow
"""
import numpy as np
import pytest

import fvcases as fc

pytestmark = pytest.mark.cpu


def _dense(n, owner, nb, diag, upper, lower):
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = diag
    A[owner, nb] = upper
    A[nb, owner] = lower
    return A


def _rest(pc, lid=0.0):
    return fc.Piso(pc.name, pc.shape, pc.n, pc.owner, pc.neighbour, pc.face_dir, pc.face_sgn, pc.bwall,
                   pc.blid * lid, pc.bgrad, np.zeros_like(pc.U0), np.zeros(pc.n), np.zeros(pc.F), pc.h, pc.nu,
                   pc.dt, pc.meta, pc.new_index)


@pytest.mark.parametrize("permute", [False, True])
def test_s1_momentum_matrix(oracle_lib, permute):
    pc = fc.piso((7, 6, 5), permute=permute)
    diag, upper, lower, bH = oracle_lib.piso_momentum(pc, pc.phi0, pc.U0)
    assert np.allclose(lower - upper, -pc.phi0, rtol=0, atol=1e-15 * (1 + np.abs(upper).max()))
    A = _dense(pc.n, pc.owner, pc.neighbour, diag, upper, lower)
    V = pc.h ** 3
    assert np.allclose(A.sum(axis=1), V / pc.dt + pc.bwall, rtol=1e-12, atol=1e-15)
    assert np.allclose(bH, V / pc.dt * pc.U0 + np.vstack([pc.blid, 0 * pc.blid, 0 * pc.blid]), rtol=1e-15)
    d0, u0, l0, _ = oracle_lib.piso_momentum(pc, np.zeros(pc.F), pc.U0)
    assert np.array_equal(u0, l0)
    assert np.all(np.linalg.eigvalsh(_dense(pc.n, pc.owner, pc.neighbour, d0, u0, l0)) > 0)


def test_s2_gradient_exact_for_linear_pressure(oracle_lib):
    pc = fc.piso((8, 7, 6))
    nx, ny, nz = pc.shape
    c = np.arange(pc.n)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    x, y, z = (i + 0.5) * pc.h, (j + 0.5) * pc.h, (k + 0.5) * pc.h
    p = 0.7 * x - 1.3 * y + 2.1 * z + 0.4
    g = oracle_lib.piso_gradp(pc, p)
    inner = (i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)
    assert np.allclose(g[0][inner], 0.7, atol=1e-12)
    assert np.allclose(g[1][inner], -1.3, atol=1e-12)
    assert np.allclose(g[2][inner], 2.1, atol=1e-12)
    # a wall cell along x: the zero-gradient face gives the one-sided value
    e = (i == 0) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)
    assert np.allclose(g[0][e], 0.35, atol=1e-12)


@pytest.mark.parametrize("n_corr", [1, 2])
def test_s3_step_against_dense_composition(oracle_lib, n_corr):
    pc = fc.piso((6, 5, 4), permute=True)
    n, V = pc.n, pc.h ** 3
    U, p, phi = pc.U0.copy(), np.random.default_rng(3).standard_normal(n), pc.phi0.copy()
    p[0] = 0.0
    Uo, po, phio, st, _, _ = oracle_lib.piso_run(pc, 1, n_corr=n_corr, U=U, p=p, phi=phi, tol_u=1e-14,
                                                 tol_p=1e-14)
    assert st == 0
    diag, upper, lower, bH = oracle_lib.piso_momentum(pc, phi, U)
    A = _dense(n, pc.owner, pc.neighbour, diag, upper, lower)
    g = oracle_lib.piso_gradp(pc, p)
    Ud = np.vstack([np.linalg.solve(A, bH[k] - V * g[k]) for k in range(3)])
    pd = p
    for _ in range(n_corr):
        s = oracle_lib.piso_pressure_system(pc, diag, upper, lower, bH, Ud)
        L = _dense(n, pc.owner, pc.neighbour, s["pdiag"], s["pupper"], s["pupper"])
        pd = np.linalg.solve(L, s["prhs"])
        phid = s["phiHbyA"] - s["cf"] * (pd[pc.neighbour] - pd[pc.owner])
        Ud = s["HbyA"] - s["rAU"] * oracle_lib.piso_gradp(pc, pd)
    scale = np.abs(Ud).max()
    assert np.abs(Uo - Ud).max() <= 1e-10 * scale
    assert np.abs(po - pd).max() <= 1e-10 * np.abs(pd).max()
    assert np.abs(phio - phid).max() <= 1e-10 * np.abs(phid).max()
    assert np.abs(oracle_lib.piso_div(pc, phid)).max() <= 1e-13 * np.abs(phid).max()


@pytest.mark.parametrize("permute", [False, True])
def test_s4_divergence_free_after_correction(oracle_lib, permute):
    pc = fc.piso((9, 8, 7), permute=permute)
    for n_corr in (1, 2, 3):
        _, _, phi, st, _, _ = oracle_lib.piso_run(pc, 2, n_corr=n_corr, tol_u=1e-12, tol_p=1e-13)
        assert st == 0
        assert np.abs(oracle_lib.piso_div(pc, phi)).max() <= 1e-10 * np.abs(phi).max()


def test_s5_rest_stays_at_rest(oracle_lib):
    pc = _rest(fc.piso((6, 6, 6)))
    U, p, phi, st, iu, ip = oracle_lib.piso_run(pc, 3, tol_u=1e-10, tol_p=1e-10)
    assert st == 0 and iu == 0 and ip == 0
    assert not U.any() and not p.any() and not phi.any()


def test_s6_energy_decays_without_lid(oracle_lib):
    pc = fc.piso((10, 9, 8))
    pc = fc.Piso(pc.name, pc.shape, pc.n, pc.owner, pc.neighbour, pc.face_dir, pc.face_sgn, pc.bwall,
                 0 * pc.blid, pc.bgrad, pc.U0, pc.p0, pc.phi0, pc.h, pc.nu, pc.dt, pc.meta)
    U, p, phi = pc.U0, pc.p0, pc.phi0
    e = [0.5 * np.sum(U ** 2)]
    for _ in range(5):
        U, p, phi, st, _, _ = oracle_lib.piso_run(pc, 1, U=U, p=p, phi=phi, tol_u=1e-12, tol_p=1e-12)
        assert st == 0
        e.append(0.5 * np.sum(U ** 2))
    assert all(b < a for a, b in zip(e, e[1:])), e


def test_s7_renumbering_invariance(oracle_lib):
    nat = fc.piso((7, 6, 5))
    per = fc.piso((7, 6, 5), permute=True)
    a = oracle_lib.piso_run(nat, 3, tol_u=1e-13, tol_p=1e-13)
    b = oracle_lib.piso_run(per, 3, tol_u=1e-13, tol_p=1e-13)
    ni = per.new_index
    assert np.abs(b[0][:, ni] - a[0]).max() <= 1e-10 * np.abs(a[0]).max()
    # the pinned reference cell differs (cell 0 of each numbering): compare
    # pressure differences, which the reference does not change
    pa, pb = a[1], b[1][ni]
    assert np.abs((pb - pb.mean()) - (pa - pa.mean())).max() <= 1e-8 * np.abs(pa).max()


def test_s8_reference_and_lid(oracle_lib):
    pc = _rest(fc.piso((8, 8, 4)), lid=1.0)
    U, p, phi, st, _, _ = oracle_lib.piso_run(pc, 3, tol_u=1e-12, tol_p=1e-12)
    assert st == 0 and p[0] == 0.0
    nx, ny, nz = pc.shape
    top = (np.arange(pc.n) // nx) % ny == ny - 1
    assert U[0][top].mean() > 0.05 and np.abs(phi).max() > 0
