"""The synthetic workloads: seeded FV Laplacian systems in LDU form.

The paper evaluates on a Dirichlet heat equation in a cube (laplacianFoam) and
the pressure equation of a lid-driven cavity (icoFoam) (Section 5, test cases;
Table pcgs2 for the steady 7-point Laplacian).  Those OpenFOAM case files are
not used; these generators stand in for them with the same structure: a
7-point hexahedral stencil, LDU addressing, Dirichlet or Neumann boundaries.

Named workloads (full size; every builder also takes a smaller shape):

* ``laplace32``   32^3 uniform, unit face coefficients, Dirichlet 0 on z-min,
                  b ~ U[-1,1].
* ``varcoef192``  192^3, face conductivities lognormal(0,1), Dirichlet 0 on
                  x-min and x-max, cells randomly permuted then RCM-renumbered,
                  b ~ U[-1,1].
* ``cavity256``   256x256x64 with cell heights graded by 1.02 per cell toward
                  the lid (y-max), Neumann walls, cell 0 pinned by elimination,
                  b = -div(U) of a random cell velocity, zero mean.
* ``batch256``    256 independent cubes, edge uniform in {16..64}, as
                  varcoef but natural order, plus x_target ~ U[-1,1].
* ``momentum192`` 192^3 non-symmetric momentum system (implicit Euler,
                  upwind convection of a divergence-free flux, nu = 0.01,
                  Courant 2), permuted + RCM like varcoef.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np

from . import mesh as M
from . import rng as R

CACHE_VERSION = 1


@dataclasses.dataclass
class Case:
    name: str
    shape: tuple
    n: int
    owner: np.ndarray      # int32[F]
    neighbour: np.ndarray  # int32[F]
    diag: np.ndarray       # float64[n]
    upper: np.ndarray      # float64[F]
    lower: np.ndarray      # float64[F]
    b: np.ndarray          # float64[n]
    tol: float = 1e-8
    seed: int = 0
    meta: dict = dataclasses.field(default_factory=dict)
    x_target: Optional[np.ndarray] = None

    @property
    def F(self) -> int:
        return int(self.owner.shape[0])

    @property
    def nnz(self) -> int:
        return self.n + 2 * self.F

    def hashes(self) -> dict:
        return {
            "addressing": R.sha256(self.owner, self.neighbour),
            "coefficients": R.sha256(self.diag, self.upper, self.lower),
            "rhs": R.sha256(self.b),
        }


def _finish(name, shape, n, owner, nb, diag, upper, lower, b, tol, seed, meta, x_target=None):
    return Case(
        name=name, shape=tuple(shape), n=int(n),
        owner=np.ascontiguousarray(owner, dtype=np.int32),
        neighbour=np.ascontiguousarray(nb, dtype=np.int32),
        diag=np.ascontiguousarray(diag, dtype=np.float64),
        upper=np.ascontiguousarray(upper, dtype=np.float64),
        lower=np.ascontiguousarray(lower, dtype=np.float64),
        b=np.ascontiguousarray(b, dtype=np.float64),
        tol=tol, seed=seed, meta=meta,
        x_target=None if x_target is None else np.ascontiguousarray(x_target, dtype=np.float64),
    )


def laplace(shape=(32, 32, 32), seed=1, dirichlet=("zmin",), tol=1e-8, rhs="uniform", name="laplace"):
    """Uniform mesh, unit face coefficients (upper = lower = -1); each
    Dirichlet side adds 2 to the diagonal of its cells (value 0 at the face).
    rhs: 'uniform' (U[-1,1], stream rhs) or 'ones'."""
    nx, ny, nz = shape
    n = nx * ny * nz
    owner, nb, _ = M.structured_faces(nx, ny, nz)
    bcells = np.concatenate([M.boundary_cells(shape, s) for s in dirichlet]) if dirichlet else np.zeros(0, np.int64)
    diag, upper, lower = M.assemble_ldu(n, owner, nb, np.ones(owner.shape), bcells, np.full(bcells.shape, 2.0))
    if rhs == "uniform":
        b = R.uniform(R.stream(seed, "rhs"), n)
    elif rhs == "ones":
        b = np.ones(n)
    else:
        raise ValueError(rhs)
    meta = {"dirichlet": list(dirichlet), "coef": "unit", "ordering": "natural"}
    return _finish(name, shape, n, owner, nb, diag, upper, lower, b, tol, seed, meta)


def varcoef(shape=(192, 192, 192), seed=2, permute=True, tol=1e-8, name="varcoef"):
    """Lognormal(0,1) conductivities on internal faces and on the Dirichlet
    faces of x-min then x-max (drawn in that order from stream coef);
    Dirichlet 0 on x-min/x-max; b ~ U[-1,1] in natural order; then cells
    randomly permuted (stream perm) and renumbered by RCM."""
    nx, ny, nz = shape
    n = nx * ny * nz
    owner, nb, _ = M.structured_faces(nx, ny, nz)
    gcoef = R.stream(seed, "coef")
    k_int = R.lognormal(gcoef, owner.shape[0])
    bl = M.boundary_cells(shape, "xmin")
    bh = M.boundary_cells(shape, "xmax")
    k_b = R.lognormal(gcoef, bl.shape[0] + bh.shape[0])
    bcells = np.concatenate([bl, bh])
    diag, upper, lower = M.assemble_ldu(n, owner, nb, k_int, bcells, 2.0 * k_b)
    b = R.uniform(R.stream(seed, "rhs"), n)
    meta = {"dirichlet": ["xmin", "xmax"], "coef": "lognormal(0,1)", "ordering": "natural"}
    if permute:
        p1 = R.stream(seed, "perm").permutation(n).astype(np.int64)
        p2 = M.rcm_order(n, p1[owner], p1[nb])
        new_index = p2[p1]
        owner, nb, upper, lower, _ = M.renumber(n, owner, nb, upper, lower, new_index)
        d2 = np.empty_like(diag)
        d2[new_index] = diag
        b2 = np.empty_like(b)
        b2[new_index] = b
        diag, b = d2, b2
        meta["ordering"] = "random permutation, then reverse Cuthill-McKee"
        meta["bandwidth"] = M.bandwidth(owner, nb)
    return _finish(name, shape, n, owner, nb, diag, upper, lower, b, tol, seed, meta)


def graded_spacing(m, length, ratio):
    """m cell widths on [0, length], each ``ratio`` times smaller than the
    previous one (ratio > 1 grades toward the high end)."""
    w = ratio ** (-np.arange(m, dtype=np.float64))
    return w * (length / w.sum())


def cavity(shape=(256, 256, 64), seed=3, ratio=1.02, tol=1e-9, name="cavity"):
    """Pressure-equation stand-in for the lid-driven cavity: box
    [0,1]x[0,1]x[0, nz/nx] with nx uniform cells in x and z and ny cells in y
    graded by ``ratio`` per cell toward the lid (y-max).  w_f = |S_f|/|d_f|,
    Neumann on every wall.  Cell 0 (the x-min/y-min/z-min corner, far from
    the lid) is pinned to 0 by elimination: the couplings of its faces are set
    to zero in both triangles (the diagonals keep them) and b[0] = 0, so A
    stays symmetric positive definite and x[0] = 0.
    b = -div(U): U ~ U[-1,1]^3 per cell (stream vel), face flux
    0.5*(U_owner + U_neighbour).S_f on internal faces and 0 on walls;
    b -= mean(b); then b[0] = 0."""
    nx, ny, nz = shape
    n = nx * ny * nz
    owner, nb, direction = M.structured_faces(nx, ny, nz)
    h = 1.0 / nx
    dx = np.full(nx, h)
    dz = np.full(nz, h)
    dy = graded_spacing(ny, 1.0, ratio)
    w = M.geometric_weights(shape, direction, owner, dx, dy, dz)
    diag, upper, lower = M.assemble_ldu(n, owner, nb, w)
    pinned = (owner == 0) | (nb == 0)
    upper[pinned] = 0.0
    lower[pinned] = 0.0
    U = R.uniform(R.stream(seed, "vel"), 3 * n).reshape(n, 3)
    i, j, k = M.cell_ijk(shape, owner)
    area = np.where(direction == 0, dy[j] * dz[k], np.where(direction == 1, dx[i] * dz[k], dx[i] * dy[j]))
    d_idx = direction.astype(np.int64)
    phi = 0.5 * (U[owner, d_idx] + U[nb, d_idx]) * area
    div = np.zeros(n)
    np.add.at(div, owner, phi)
    np.add.at(div, nb, -phi)
    b = -div
    b -= b.mean()
    b[0] = 0.0
    meta = {"boundary": "Neumann walls, cell 0 pinned", "grading": ratio, "dy_first": float(dy[0]),
            "dy_last": float(dy[-1]), "ordering": "natural", "pinned_faces": int(pinned.sum())}
    return _finish(name, shape, n, owner, nb, diag, upper, lower, b, tol, seed, meta)


@dataclasses.dataclass
class Batch:
    """Concatenated independent systems; addressing is local to each system."""
    name: str
    cases: list
    cell_off: np.ndarray   # int32[nsys+1]
    face_off: np.ndarray   # int32[nsys+1]
    owner: np.ndarray
    neighbour: np.ndarray
    diag: np.ndarray
    upper: np.ndarray
    lower: np.ndarray
    b: np.ndarray
    x_target: np.ndarray
    tol: float = 1e-8
    seed: int = 0

    @property
    def nsys(self) -> int:
        return len(self.cases)


def batch(nsys=256, edge_lo=16, edge_hi=64, seed=5, tol=1e-8, name="batch"):
    """nsys cubes with edge e_s uniform in {edge_lo..edge_hi} (stream sizes);
    per system: lognormal conductivities (stream coef, consumed system after
    system), Dirichlet 0 on x-min/x-max, natural order, b ~ U[-1,1] (stream
    rhs) and x_target ~ U[-1,1] (stream target)."""
    edges = R.stream(seed, "sizes").integers(edge_lo, edge_hi + 1, size=nsys)
    gcoef = R.stream(seed, "coef")
    grhs = R.stream(seed, "rhs")
    gtgt = R.stream(seed, "target")
    cases = []
    for s, e in enumerate(edges):
        e = int(e)
        shape = (e, e, e)
        n = e ** 3
        owner, nb, _ = M.structured_faces(e, e, e)
        k_int = R.lognormal(gcoef, owner.shape[0])
        bl = M.boundary_cells(shape, "xmin")
        bh = M.boundary_cells(shape, "xmax")
        k_b = R.lognormal(gcoef, bl.shape[0] + bh.shape[0])
        diag, upper, lower = M.assemble_ldu(n, owner, nb, k_int, np.concatenate([bl, bh]), 2.0 * k_b)
        b = R.uniform(grhs, n)
        xt = R.uniform(gtgt, n)
        cases.append(_finish(f"{name}[{s}]", shape, n, owner, nb, diag, upper, lower, b, tol, seed,
                             {"edge": e, "ordering": "natural"}, x_target=xt))
    return concat(cases, name=name, tol=tol, seed=seed)


def concat(cases, name="batch", tol=1e-8, seed=0):
    """Batch of the given systems, in order (a missing x_target reads as 0)."""
    nsys = len(cases)
    cell_off = np.zeros(nsys + 1, dtype=np.int64)
    face_off = np.zeros(nsys + 1, dtype=np.int64)
    cell_off[1:] = np.cumsum([c.n for c in cases])
    face_off[1:] = np.cumsum([c.F for c in cases])
    if cell_off[-1] >= 2 ** 31 or face_off[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 offsets")
    cat = lambda attr: np.concatenate([getattr(c, attr) for c in cases])
    xt = np.concatenate([c.x_target if c.x_target is not None else np.zeros(c.n) for c in cases])
    return Batch(name=name, cases=list(cases), cell_off=cell_off.astype(np.int32),
                 face_off=face_off.astype(np.int32), owner=cat("owner"), neighbour=cat("neighbour"),
                 diag=cat("diag"), upper=cat("upper"), lower=cat("lower"), b=cat("b"), x_target=xt, tol=tol,
                 seed=seed)


@dataclasses.dataclass
class Transient:
    """Inputs of a transient diffusion run (laplacianFoam, implicit Euler):
    per internal face a conductivity k_f and geometric weight w_f = |S_f|/|d_f|,
    per cell a volume V_c, the Dirichlet contributions to the diagonal
    (bdiag = sum of 2 k_b w_b over the cell's Dirichlet faces) and to the
    right-hand side (bsrc = sum of 2 k_b w_b T_b plus a volumetric source),
    the initial field T0 and the time step dt."""
    name: str
    shape: tuple
    n: int
    owner: np.ndarray
    neighbour: np.ndarray
    k_face: np.ndarray
    w_face: np.ndarray
    vol: np.ndarray
    bdiag: np.ndarray
    bsrc: np.ndarray
    T0: np.ndarray
    dt: float
    tol: float = 1e-8

    @property
    def F(self) -> int:
        return int(self.owner.shape[0])


def transient(shape=(32, 32, 32), seed=7, dt=0.25, permute=False, tol=1e-8, name="transient"):
    """Unit cubes (w_f = 1, V_c = 1), lognormal(0,1) conductivities (stream
    coef, internal faces then the Dirichlet faces of x-min and x-max), T_b = 1
    on x-min and 0 on x-max, a source U[0,1] per cell (stream src), T0 = 0;
    optionally randomly permuted and RCM-renumbered (stream perm) like the
    lognormal workload."""
    nx, ny, nz = shape
    n = nx * ny * nz
    owner, nb, _ = M.structured_faces(nx, ny, nz)
    gcoef = R.stream(seed, "coef")
    k_int = R.lognormal(gcoef, owner.shape[0])
    bl = M.boundary_cells(shape, "xmin")
    bh = M.boundary_cells(shape, "xmax")
    k_b = R.lognormal(gcoef, bl.shape[0] + bh.shape[0])
    bdiag = np.zeros(n)
    np.add.at(bdiag, np.concatenate([bl, bh]), 2.0 * k_b)
    bsrc = R.uniform(R.stream(seed, "src"), n) * 0.5 + 0.5
    np.add.at(bsrc, bl, 2.0 * k_b[: bl.shape[0]] * 1.0)
    w = np.ones(owner.shape[0])
    vol = np.ones(n)
    if permute:
        p1 = R.stream(seed, "perm").permutation(n).astype(np.int64)
        p2 = M.rcm_order(n, p1[owner], p1[nb])
        new_index = p2[p1]
        owner, nb, _, _, order = M.renumber(n, owner, nb, k_int, k_int, new_index)
        k_int = k_int[order]
        w = w[order]

        def moved(a):
            out = np.empty_like(a)
            out[new_index] = a
            return out

        bdiag, bsrc, vol = moved(bdiag), moved(bsrc), moved(vol)
    return Transient(name=name, shape=tuple(shape), n=n, owner=np.ascontiguousarray(owner, dtype=np.int32),
                     neighbour=np.ascontiguousarray(nb, dtype=np.int32), k_face=np.ascontiguousarray(k_int),
                     w_face=np.ascontiguousarray(w), vol=np.ascontiguousarray(vol), bdiag=bdiag, bsrc=bsrc,
                     T0=np.zeros(n), dt=float(dt), tol=tol)


def momentum(shape=(192, 192, 192), seed=11, nu=0.01, co=2.0, permute=True, tol=1e-8, name="momentum"):
    """Momentum-predictor stand-in for icoFoam (Section 2: its momentum
    equation is solved with BiCGSTAB): the x-velocity equation of implicit
    Euler with first-order upwind convection on cubes of side h = 1/nx in the
    box [0,1] x [0, ny h] x [0, nz h].

    Face fluxes are those of U = curl(psi e_z) with
    psi = a sin(pi x) sin(pi y / Ly) (1 + 0.5 sin(2 pi z / Lz + theta)),
    taken exactly as psi differences along each x- and y-face's edges (zero
    on z-faces and walls), so every cell's net outflow is zero up to rounding;
    a scales max |U| to 1 and theta ~ U[0, 2 pi) (stream vel).  Per internal
    face (owner o -> neighbour m, flux F > 0 from o to m), D = nu h:
        upper = -D - max(-F, 0),  lower = -D - max(F, 0);
    diag = h^3/dt + sum over the cell's faces of (D + its outflow, if any)
    + 2 nu h per wall face (no slip); the lid (y-max) moves at u = 1, adding
    2 nu h to b there; b = h^3/dt u_old + h^3 g with u_old, g ~ U[-1,1]
    (streams vel, src); dt = co h (Courant number co at |U| = 1).  Then,
    as the lognormal workload, cells randomly permuted and RCM-renumbered
    (stream perm).  Row sums are h^3/dt plus the wall terms: diagonally
    dominant, lower != upper wherever the flux is non-zero."""
    nx, ny, nz = shape
    n = nx * ny * nz
    h = 1.0 / nx
    Ly, Lz = ny * h, nz * h
    owner, nb, direction = M.structured_faces(nx, ny, nz)
    gvel = R.stream(seed, "vel")
    theta = 2.0 * np.pi * gvel.random()
    a = 1.0 / (1.5 * np.pi * max(1.0, 1.0 / Ly))

    def psi(x, y, z):
        return a * np.sin(np.pi * x) * np.sin(np.pi * y / Ly) * (1.0 + 0.5 * np.sin(2.0 * np.pi * z / Lz + theta))

    i, j, k = M.cell_ijk(shape, owner)
    zc = (k + 0.5) * h
    flux = np.zeros(owner.shape[0])
    m = direction == 0
    xf = (i[m] + 1) * h
    flux[m] = (psi(xf, (j[m] + 1) * h, zc[m]) - psi(xf, j[m] * h, zc[m])) * h
    m = direction == 1
    yf = (j[m] + 1) * h
    flux[m] = -(psi((i[m] + 1) * h, yf, zc[m]) - psi(i[m] * h, yf, zc[m])) * h
    D = nu * h
    dt = co * h
    vol = h ** 3
    upper = -D - np.maximum(-flux, 0.0)
    lower = -D - np.maximum(flux, 0.0)
    diag = np.full(n, vol / dt)
    np.add.at(diag, owner, D + np.maximum(flux, 0.0))
    np.add.at(diag, nb, D + np.maximum(-flux, 0.0))
    walls = ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax")
    for side in walls:
        np.add.at(diag, M.boundary_cells(shape, side), 2.0 * nu * h)
    u_old = R.uniform(gvel, n)
    g = R.uniform(R.stream(seed, "src"), n)
    b = vol / dt * u_old + vol * g
    np.add.at(b, M.boundary_cells(shape, "ymax"), 2.0 * nu * h * 1.0)
    meta = {"nu": nu, "courant": co, "dt": dt, "h": h, "theta": theta, "ordering": "natural",
            "max_cell_peclet": float(np.abs(flux).max() / D) if flux.size else 0.0}
    if permute:
        p1 = R.stream(seed, "perm").permutation(n).astype(np.int64)
        p2 = M.rcm_order(n, p1[owner], p1[nb])
        new_index = p2[p1]
        owner, nb, upper, lower, _ = M.renumber(n, owner, nb, upper, lower, new_index)
        d2 = np.empty_like(diag)
        d2[new_index] = diag
        b2 = np.empty_like(b)
        b2[new_index] = b
        diag, b = d2, b2
        meta["ordering"] = "random permutation, then reverse Cuthill-McKee"
        meta["bandwidth"] = M.bandwidth(owner, nb)
    return _finish(name, shape, n, owner, nb, diag, upper, lower, b, tol, seed, meta)


@dataclasses.dataclass
class Piso:
    """Inputs of an icoFoam-style PISO run (incompressible Navier-Stokes,
    implicit Euler, upwind convection) in a lid-driven box of cubes of side h:
    the LDU addressing, per internal face its axis (face_dir 0/1/2) and the
    orientation of owner -> neighbour along that axis (face_sgn +1/-1), per
    cell the no-slip wall coefficient bwall = 2 nu h per wall face (lid
    included), the lid source blid = 2 nu h U_lid per lid face (x-velocity
    only) and bgrad[d] = the sum of the outward unit normals (+-1) of its
    boundary faces along axis d (zero-gradient pressure at the walls); the
    initial fields U0[3][n], p0[n] and face fluxes phi0[F]."""
    name: str
    shape: tuple
    n: int
    owner: np.ndarray
    neighbour: np.ndarray
    face_dir: np.ndarray
    face_sgn: np.ndarray
    bwall: np.ndarray
    blid: np.ndarray
    bgrad: np.ndarray
    U0: np.ndarray
    p0: np.ndarray
    phi0: np.ndarray
    h: float
    nu: float
    dt: float
    meta: dict = dataclasses.field(default_factory=dict)
    new_index: Optional[np.ndarray] = None  # natural cell c -> its number here (None: natural order)

    @property
    def F(self) -> int:
        return int(self.owner.shape[0])


def piso(shape=(32, 32, 32), seed=13, nu=0.01, co=1.0, u_lid=1.0, permute=False, name="piso"):
    """Lid-driven cavity for icoFoam's PISO loop (Section 2 names icoFoam;
    the paper's cavity case is stood in for): cubes of side h = 1/nx in
    [0,1] x [0, ny h] x [0, nz h], no-slip walls, the y-max lid moving at
    u = u_lid in x, viscosity nu, dt = co h / u_lid.  The initial state is
    the discretely divergence-free flow of the momentum workload's stream
    function (face fluxes from psi differences, stream vel), cell velocities
    the mean of the two face fluxes per axis over the face area, p0 = 0.
    Optionally randomly permuted and RCM-renumbered (stream perm), which
    flips face_sgn where owner and neighbour swap."""
    nx, ny, nz = shape
    n = nx * ny * nz
    h = 1.0 / nx
    Ly, Lz = ny * h, nz * h
    owner, nb, direction = M.structured_faces(nx, ny, nz)
    gvel = R.stream(seed, "vel")
    theta = 2.0 * np.pi * gvel.random()
    a = 1.0 / (1.5 * np.pi * max(1.0, 1.0 / Ly))

    def psi(x, y, z):
        return a * np.sin(np.pi * x) * np.sin(np.pi * y / Ly) * (1.0 + 0.5 * np.sin(2.0 * np.pi * z / Lz + theta))

    i, j, k = M.cell_ijk(shape, owner)
    zc = (k + 0.5) * h
    phi = np.zeros(owner.shape[0])
    m = direction == 0
    xf = (i[m] + 1) * h
    phi[m] = (psi(xf, (j[m] + 1) * h, zc[m]) - psi(xf, j[m] * h, zc[m])) * h
    m = direction == 1
    yf = (j[m] + 1) * h
    phi[m] = -(psi((i[m] + 1) * h, yf, zc[m]) - psi(i[m] * h, yf, zc[m])) * h
    # cell velocities: per axis, the mean of the cell's two face fluxes along it over h^2
    U0 = np.zeros((3, n))
    for d in range(3):
        md = direction == d
        np.add.at(U0[d], owner[md], 0.5 * phi[md] / h ** 2)
        np.add.at(U0[d], nb[md], 0.5 * phi[md] / h ** 2)
    bwall = np.zeros(n)
    blid = np.zeros(n)
    bgrad = np.zeros((3, n))
    for side, d, sgn in (("xmin", 0, -1.0), ("xmax", 0, 1.0), ("ymin", 1, -1.0), ("ymax", 1, 1.0),
                         ("zmin", 2, -1.0), ("zmax", 2, 1.0)):
        cells = M.boundary_cells(shape, side)
        np.add.at(bwall, cells, 2.0 * nu * h)
        np.add.at(bgrad[d], cells, sgn)
        if side == "ymax":
            np.add.at(blid, cells, 2.0 * nu * h * u_lid)
    sgn = np.ones(owner.shape[0], dtype=np.int8)
    meta = {"ordering": "natural", "u_lid": u_lid, "courant": co}
    new_index = None
    if permute:
        p1 = R.stream(seed, "perm").permutation(n).astype(np.int64)
        p2 = M.rcm_order(n, p1[owner], p1[nb])
        new_index = p2[p1]
        swapped = new_index[owner] > new_index[nb]
        owner, nb, _, _, order = M.renumber(n, owner, nb, phi, phi, new_index)
        direction = direction[order]
        sgn = np.where(swapped, -1, 1).astype(np.int8)[order]
        phi = (np.where(swapped, -phi, phi))[order]

        def moved(v):
            out = np.empty_like(v)
            out[..., new_index] = v
            return out

        U0, bwall, blid, bgrad = moved(U0), moved(bwall), moved(blid), moved(bgrad)
        meta["ordering"] = "random permutation, then reverse Cuthill-McKee"
        meta["bandwidth"] = M.bandwidth(owner, nb)
    return Piso(name=name, shape=tuple(shape), n=n, owner=np.ascontiguousarray(owner, dtype=np.int32),
                neighbour=np.ascontiguousarray(nb, dtype=np.int32), face_dir=np.ascontiguousarray(direction,
                dtype=np.int8), face_sgn=np.ascontiguousarray(sgn), bwall=bwall, blid=blid,
                bgrad=np.ascontiguousarray(bgrad), U0=np.ascontiguousarray(U0), p0=np.zeros(n),
                phi0=np.ascontiguousarray(phi), h=h, nu=nu, dt=co * h / max(u_lid, 1.0), meta=meta,
                new_index=new_index)


def momentum_rhs(case, component, seed=12):
    """Right-hand side of another velocity component (1 = y, 2 = z) of a
    momentum case: the recipe of its b without the lid term,
    (h^3/dt) u_old + h^3 g with fresh u_old, g ~ U[-1,1] (streams vel and
    src of seed + component).  Independent draws per cell, so the cell order
    of the case does not matter."""
    h, dt = case.meta["h"], case.meta["dt"]
    vol = h ** 3
    u_old = R.uniform(R.stream(seed + component, "vel"), case.n)
    g = R.uniform(R.stream(seed + component, "src"), case.n)
    return vol / dt * u_old + vol * g


# ---------------------------------------------------------------------------
# Named full-size workloads, with an on-disk cache for the large ones.

def _cache_dir():
    return os.environ.get("FVCASES_CACHE", "/tmp/fvcases_cache")


_FIELDS = ("owner", "neighbour", "diag", "upper", "lower", "b")


def _cached(key, builder):
    d = os.path.join(_cache_dir(), f"v{CACHE_VERSION}_{key}")
    meta_path = os.path.join(d, "meta.json")
    import json
    if os.path.exists(meta_path):
        try:
            with open(meta_path) as f:
                info = json.load(f)
            arrs = {k: np.load(os.path.join(d, k + ".npy"), allow_pickle=False) for k in _FIELDS}
            return Case(name=info["name"], shape=tuple(info["shape"]), n=info["n"], tol=info["tol"],
                        seed=info["seed"], meta=info["meta"], **arrs)
        except Exception:
            pass
    case = builder()
    try:
        os.makedirs(d, exist_ok=True)
        for k in _FIELDS:
            np.save(os.path.join(d, k + ".npy"), getattr(case, k), allow_pickle=False)
        with open(meta_path + ".tmp", "w") as f:
            json.dump({"name": case.name, "shape": list(case.shape), "n": case.n, "tol": case.tol,
                       "seed": case.seed, "meta": case.meta}, f)
        os.replace(meta_path + ".tmp", meta_path)
    except OSError:
        pass
    return case


def make(name: str, cache: bool = True):
    """Full-size named workload."""
    if name == "laplace32":
        return laplace((32, 32, 32), seed=1, name=name)
    if name == "varcoef192":
        b = lambda: varcoef((192, 192, 192), seed=2, name=name)
        return _cached("varcoef192_s2", b) if cache else b()
    if name == "cavity256":
        b = lambda: cavity((256, 256, 64), seed=3, name=name)
        return _cached("cavity256_s3", b) if cache else b()
    if name == "batch256":
        return batch(256, 16, 64, seed=5, name=name)
    if name == "momentum192":
        b = lambda: momentum((192, 192, 192), seed=11, name=name)
        return _cached("momentum192_s11", b) if cache else b()
    raise KeyError(name)
