"""Plain solvers for batched block-bidiagonal systems (Section 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The chunked Newton update (Eq. batched-update) solves, per series, the
lower block-bidiagonal system whose diagonal blocks are D_j = I - dt_j j_j and
whose sub-diagonal blocks are -I (the chunk Jacobian of Section 2.3):

    D_1 x_1 = r_1,    -x_{j-1} + D_j x_j = r_j    (j = 2..m).

The chunked adjoint (Appendix A.2) solves the transposed, upper system

    D_j^T x_j - x_{j+1} = r_j    (j = m..1,  x_{m+1} = 0).

``dense_solve`` is the plain definition: assemble the full (m n) x (m n)
matrix and call ``numpy.linalg.solve``.  ``thomas`` is Thomas's algorithm
(Alg. thomas) for the same systems.
"""
from __future__ import annotations

import numpy as np


def assemble(D, transpose=False):
    """Full matrices [B, m n, m n] of the (transposed) chunk system with diagonal blocks D [B, m, n, n]."""
    D = np.asarray(D, dtype=np.float64)
    B, m, n, _ = D.shape
    A = np.zeros((B, m * n, m * n))
    eye = np.eye(n)
    for j in range(m):
        A[:, j * n:(j + 1) * n, j * n:(j + 1) * n] = D[:, j]
        if j > 0:
            A[:, j * n:(j + 1) * n, (j - 1) * n:j * n] = -eye
    if transpose:
        A = np.transpose(A, (0, 2, 1)).copy()
    return A


def dense_solve(D, r, transpose=False):
    """x [B, m, n] solving the lower (or, with ``transpose``, the upper) chunk system."""
    D = np.asarray(D, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    B, m, n, _ = D.shape
    if m == 0:
        return np.zeros((B, 0, n))
    A = assemble(D, transpose)
    x = np.linalg.solve(A, r.reshape(B, m * n, 1))
    return x.reshape(B, m, n)


def thomas(D, r, transpose=False):
    """Thomas's algorithm (Alg. thomas) with sub-diagonal blocks -I.

    Lower: x_1 = D_1^{-1} r_1, x_{j} = D_j^{-1} (r_j + x_{j-1}).
    Upper (transposed): x_m = D_m^{-T} r_m, x_j = D_j^{-T} (r_j + x_{j+1}).
    """
    D = np.asarray(D, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    B, m, n, _ = D.shape
    x = np.zeros((B, m, n))
    carry = np.zeros((B, n))
    steps = range(m - 1, -1, -1) if transpose else range(m)
    for j in steps:
        A = np.transpose(D[:, j], (0, 2, 1)) if transpose else D[:, j]
        carry = np.linalg.solve(A, (r[:, j] + carry)[..., None])[..., 0]
        x[:, j] = carry
    return x
