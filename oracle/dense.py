"""Dense brute-force reference for tiny grids (TEST INFRASTRUCTURE ONLY).

The 7-point Poisson operator is assembled as an explicit matrix, straight
from its definition: for interior point p, (A u)_p = (6 u_p - sum of its six
neighbours) / h^2, where a neighbour in the halo contributes its (known)
Dirichlet value to the right-hand side instead of a matrix entry.  With
b = f + (halo neighbours)/h^2 the discrete problem is A u = b, and

    Jacobi:   u' = D^-1 (b - (A - D) u),  D = diag(A) = 6/h^2
    residual: r  = b - A u

The exact discrete solution comes from a dense LU solve (numpy.linalg.solve).
None of this shares code with the loop oracle or with the GPU path.
"""
from __future__ import annotations

import numpy as np


def interior_index(nx, ny, nz):
    """Map interior (i,j,k), 1-based, to the unknown number (Fortran order)."""
    return lambda i, j, k: (i - 1) + nx * ((j - 1) + ny * (k - 1))


def assemble(nx: int, ny: int, nz: int, h: float):
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = interior_index(nx, ny, nz)
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                p = idx(i, j, k)
                A[p, p] = 6.0 / h ** 2
                for (a, b, c) in ((i - 1, j, k), (i + 1, j, k), (i, j - 1, k),
                                  (i, j + 1, k), (i, j, k - 1), (i, j, k + 1)):
                    if 1 <= a <= nx and 1 <= b <= ny and 1 <= c <= nz:
                        A[p, idx(a, b, c)] = -1.0 / h ** 2
    return A


def rhs(f_padded: np.ndarray, halo_padded: np.ndarray, h: float):
    """b = f + (sum of halo neighbours)/h^2 over the interior (vector)."""
    nz, ny, nx = (s - 2 for s in f_padded.shape)
    idx = interior_index(nx, ny, nz)
    b = np.zeros(nx * ny * nz)
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                p = idx(i, j, k)
                acc = f_padded[k, j, i]
                for (a, bb, c) in ((i - 1, j, k), (i + 1, j, k), (i, j - 1, k),
                                   (i, j + 1, k), (i, j, k - 1), (i, j, k + 1)):
                    if not (1 <= a <= nx and 1 <= bb <= ny and 1 <= c <= nz):
                        acc += halo_padded[c, bb, a] / h ** 2
                b[p] = acc
    return b


def to_vec(a_padded: np.ndarray):
    return a_padded[1:-1, 1:-1, 1:-1].reshape(-1).copy()


def from_vec(v: np.ndarray, like_padded: np.ndarray):
    out = like_padded.copy()
    nz, ny, nx = (s - 2 for s in like_padded.shape)
    out[1:-1, 1:-1, 1:-1] = v.reshape(nz, ny, nx)
    return out


def jacobi(A: np.ndarray, b: np.ndarray, u: np.ndarray):
    d = np.diag(A)
    off = A - np.diag(d)
    return (b - off @ u) / d


def residual(A: np.ndarray, b: np.ndarray, u: np.ndarray):
    return b - A @ u


def exact(A: np.ndarray, b: np.ndarray):
    return np.linalg.solve(A, b)
