"""Structured hexahedral meshes and finite-volume Laplacian assembly in LDU form.

This module builds *inputs* only: cell/face addressing and the coefficients of
the cell-centred finite-volume discretisation of -div(k grad T) on a box of
hexahedra.  It performs none of the solver's arithmetic (no products with the
matrix, no Krylov steps); both the HIP path and the CPU oracle receive the
arrays it returns.

LDU conventions (the OpenFOAM lduMatrix layout that the paper names in its
Section 5 discussion of the CUDA/OpenFOAM interface, with nnz = n + 2F as in
the Section 4.2 work model):

* cells are numbered c = i + nx*(j + ny*k) in natural order;
* internal face f joins owner[f] < neighbour[f]; faces are sorted strictly by
  (owner, neighbour);
* row owner[f] holds upper[f] in column neighbour[f]; row neighbour[f] holds
  lower[f] in column owner[f]; diag[c] is the diagonal.

The stored operator is the SPD form -div(k grad .): diag > 0 and
upper = lower <= 0 (the Section 2 heat equation is printed garbled; this is the
diffusion operator it describes).
"""
from __future__ import annotations

import numpy as np


def structured_faces(nx: int, ny: int, nz: int):
    """Internal faces of an nx*ny*nz box of hexahedra in LDU order.

    Returns (owner, neighbour, direction, owner_cell_ijk) where direction is
    0/1/2 for faces normal to x/y/z.  Face count is
    (nx-1)*ny*nz + nx*(ny-1)*nz + nx*ny*(nz-1).
    """
    n = nx * ny * nz
    c = np.arange(n, dtype=np.int64)
    i = c % nx
    j = (c // nx) % ny
    k = c // (nx * ny)
    owners = []
    nbs = []
    dirs = []
    for d, (mask, step) in enumerate(((i < nx - 1, 1), (j < ny - 1, nx), (k < nz - 1, nx * ny))):
        o = c[mask]
        owners.append(o)
        nbs.append(o + step)
        dirs.append(np.full(o.shape, d, dtype=np.int8))
    owner = np.concatenate(owners)
    nb = np.concatenate(nbs)
    direction = np.concatenate(dirs)
    # (owner, neighbour) lexicographic: neighbour offsets 1 < nx < nx*ny are
    # already increasing per owner, so a stable sort on owner suffices.
    order = np.argsort(owner, kind="stable")
    owner = owner[order]
    nb = nb[order]
    direction = direction[order]
    return owner, nb, direction


def cell_ijk(shape, cells):
    nx, ny, _ = shape
    cells = np.asarray(cells, dtype=np.int64)
    return cells % nx, (cells // nx) % ny, cells // (nx * ny)


def boundary_cells(shape, side: str):
    """Cells adjacent to one side of the box ('xmin', 'xmax', 'ymin', ...),
    in increasing natural index."""
    nx, ny, nz = shape
    c = np.arange(nx * ny * nz, dtype=np.int64)
    i, j, k = cell_ijk(shape, c)
    sel = {
        "xmin": i == 0, "xmax": i == nx - 1,
        "ymin": j == 0, "ymax": j == ny - 1,
        "zmin": k == 0, "zmax": k == nz - 1,
    }[side]
    return c[sel]


def geometric_weights(shape, direction, owner, dx, dy, dz):
    """w_f = |S_f| / |d_f| for an orthogonal box mesh with per-index spacings
    dx[i], dy[j], dz[k] (face area over distance between cell centres)."""
    i, j, k = cell_ijk(shape, owner)
    w = np.empty(owner.shape, dtype=np.float64)
    m = direction == 0
    w[m] = dy[j[m]] * dz[k[m]] / (0.5 * (dx[i[m]] + dx[i[m] + 1]))
    m = direction == 1
    w[m] = dx[i[m]] * dz[k[m]] / (0.5 * (dy[j[m]] + dy[j[m] + 1]))
    m = direction == 2
    w[m] = dx[i[m]] * dy[j[m]] / (0.5 * (dz[k[m]] + dz[k[m] + 1]))
    return w


def boundary_weight(shape, side, cells, dx, dy, dz):
    """|S_b| / (half cell width): the face-to-centre coefficient of a
    Dirichlet boundary face (twice the interior weight on a uniform mesh)."""
    i, j, k = cell_ijk(shape, cells)
    if side[0] == "x":
        return dy[j] * dz[k] / (0.5 * dx[i])
    if side[0] == "y":
        return dx[i] * dz[k] / (0.5 * dy[j])
    return dx[i] * dy[j] / (0.5 * dz[k])


def assemble_ldu(n, owner, nb, face_coeff, bcells=None, bcoeff=None):
    """Cell-centred FV Laplacian: upper = lower = -c_f, diag = sum of the
    coefficients of every face (internal and Dirichlet) touching the cell.
    Neumann faces contribute nothing."""
    face_coeff = np.asarray(face_coeff, dtype=np.float64)
    diag = np.zeros(n, dtype=np.float64)
    np.add.at(diag, owner, face_coeff)
    np.add.at(diag, nb, face_coeff)
    if bcells is not None and len(bcells):
        np.add.at(diag, bcells, np.asarray(bcoeff, dtype=np.float64))
    upper = -face_coeff
    lower = upper.copy()
    return diag, upper, lower


def renumber(n, owner, nb, upper, lower, new_index):
    """Relabel cells by new_index[old] and restore the LDU face order
    (owner < neighbour, sorted).  A face whose ends swap also swaps its
    upper/lower coefficients, so the matrix is the same operator permuted."""
    a = new_index[owner]
    b = new_index[nb]
    swap = a > b
    o2 = np.where(swap, b, a)
    n2 = np.where(swap, a, b)
    up2 = np.where(swap, lower, upper)
    lo2 = np.where(swap, upper, lower)
    key = o2.astype(np.int64) * n + n2
    order = np.argsort(key, kind="stable")
    return o2[order], n2[order], up2[order], lo2[order], order


def rcm_order(n, owner, nb):
    """Reverse Cuthill-McKee ordering of the cell graph (SciPy's
    implementation); returns new_index[old]."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    rows = np.concatenate([owner, nb]).astype(np.int32)
    cols = np.concatenate([nb, owner]).astype(np.int32)
    data = np.ones(rows.shape, dtype=np.int8)
    g = sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    order = reverse_cuthill_mckee(g, symmetric_mode=True)
    new_index = np.empty(n, dtype=np.int64)
    new_index[order] = np.arange(n, dtype=np.int64)
    return new_index


def bandwidth(owner, nb):
    """Largest |owner - neighbour| over the faces."""
    return int(np.max(np.abs(nb.astype(np.int64) - owner))) if len(owner) else 0
