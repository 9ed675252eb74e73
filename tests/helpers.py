"""Independent checkers for the oracle: dense matrices built by direct
indexing (not by the oracle's face loop), closed-form spectra of the
uniform-grid finite-volume Laplacian, and Lanczos matrices from CG scalars."""
from __future__ import annotations

import numpy as np


def dense_from_ldu(n, owner, nb, diag, upper, lower):
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = diag
    A[owner, nb] = upper
    A[nb, owner] = lower
    return A


def dense(case):
    return dense_from_ldu(case.n, case.owner.astype(np.int64), case.neighbour.astype(np.int64),
                          case.diag, case.upper, case.lower)


# 1-D cell-centred FV second difference with unit coefficients on m cells.
# A Dirichlet end (value 0 at the face, coefficient 2) or a Neumann end.

def eig_1d(m, left, right):
    """Eigenpairs (mu[k], V[:, k]) of the 1-D operator; ends 'D' or 'N'."""
    j = np.arange(m) + 0.5
    if left == "N" and right == "N":
        k = np.arange(m)
        mu = 4 * np.sin(np.pi * k / (2 * m)) ** 2
        V = np.cos(np.pi * np.outer(j, k) / m)
    elif left == "D" and right == "D":
        k = np.arange(1, m + 1)
        mu = 4 * np.sin(np.pi * k / (2 * m)) ** 2
        V = np.sin(np.pi * np.outer(j, k) / m)
    elif left == "D" and right == "N":
        k = np.arange(1, m + 1)
        mu = 4 * np.sin(np.pi * (2 * k - 1) / (4 * m)) ** 2
        V = np.sin(np.pi * np.outer(j, 2 * k - 1) / (2 * m))
    elif left == "N" and right == "D":
        mu, V = eig_1d(m, "D", "N")
        V = V[::-1, :].copy()
    else:
        raise ValueError((left, right))
    return mu, V


def eig_3d(shape, ends):
    """ends = ((xl, xr), (yl, yr), (zl, zr)); returns the 1-D factors."""
    return [eig_1d(m, *e) for m, e in zip(shape, ends)]


def tensor_vec(vx, vy, vz):
    """v[c] for c = i + nx*(j + ny*k)."""
    return np.einsum("k,j,i->kji", vz, vy, vx).ravel()


def lanczos_from_cg(alpha, beta):
    """Tridiagonal Lanczos matrix T_k implied by k CG steps:
    T[j,j] = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T[j,j+1] = sqrt(beta_j)/alpha_j."""
    k = len(alpha)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return T
