"""Pins of the plain block-bidiagonal solvers (Section 3) and of the reading of
parallel cyclic reduction the GPU implements."""
import numpy as np
import pytest

from oracle import blockbidiag as bb


def random_blocks(rng, B, m, n, scale=0.3):
    # diagonally dominant-ish blocks like I - dt j
    return np.eye(n)[None, None] + (scale / np.sqrt(n)) * rng.standard_normal((B, m, n, n))


def blockwise_apply(D, x, transpose=False):
    """J x computed block by block (no assembled matrix)."""
    B, m, n, _ = D.shape
    out = np.empty_like(x)
    for j in range(m):
        if transpose:
            out[:, j] = np.einsum("bki,bk->bi", D[:, j], x[:, j])
            if j + 1 < m:
                out[:, j] -= x[:, j + 1]
        else:
            out[:, j] = np.einsum("bik,bk->bi", D[:, j], x[:, j])
            if j > 0:
                out[:, j] -= x[:, j - 1]
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8])
def test_dense_solution_satisfies_the_blockwise_equations(n):
    rng = np.random.default_rng(n)
    for m in (1, 2, 3, 7, 16, 33):
        D = random_blocks(rng, 3, m, n)
        r = rng.standard_normal((3, m, n))
        for tr in (False, True):
            x = bb.dense_solve(D, r, transpose=tr)
            scale = np.abs(D).max() * np.abs(x).max() + np.abs(r).max()
            assert np.abs(blockwise_apply(D, x, tr) - r).max() <= 1e-13 * scale


@pytest.mark.parametrize("n", [2, 3, 4])
def test_thomas_equals_dense(n):
    rng = np.random.default_rng(10 + n)
    for m in list(range(1, 66)):
        D = random_blocks(rng, 2, m, n)
        r = rng.standard_normal((2, m, n))
        for tr in (False, True):
            x = bb.dense_solve(D, r, tr)
            assert np.abs(bb.thomas(D, r, tr) - x).max() <= 1e-11 * np.abs(x).max()


def test_transpose_dot_product_identity():
    rng = np.random.default_rng(3)
    D = random_blocks(rng, 4, 40, 3)
    u = rng.standard_normal((4, 40, 3))
    v = rng.standard_normal((4, 40, 3))
    a = np.sum(bb.dense_solve(D, u) * v, axis=(1, 2))
    b = np.sum(u * bb.dense_solve(D, v, transpose=True), axis=(1, 2))
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_paper_four_block_split():
    """One PCR level on a general 4-block bidiagonal system (Section 3.2): the
    red system (x1, x3) and the green system (x2, x4) carry the solution."""
    rng = np.random.default_rng(4)
    n = 3
    A = [np.eye(n) + 0.3 * rng.standard_normal((n, n)) for _ in range(4)]
    Bs = [0.5 * rng.standard_normal((n, n)) for _ in range(3)]
    y = [rng.standard_normal(n) for _ in range(4)]
    full = np.zeros((4 * n, 4 * n))
    for i in range(4):
        full[i * n:(i + 1) * n, i * n:(i + 1) * n] = A[i]
        if i:
            full[i * n:(i + 1) * n, (i - 1) * n:i * n] = Bs[i - 1]
    x = np.linalg.solve(full, np.concatenate(y)).reshape(4, n)
    inv = np.linalg.inv
    red = np.block([[A[0], np.zeros((n, n))], [-Bs[1] @ inv(A[1]) @ Bs[0], A[2]]])
    red_rhs = np.concatenate([y[0], y[2] - Bs[1] @ inv(A[1]) @ y[1]])
    green = np.block([[A[1], np.zeros((n, n))], [-Bs[2] @ inv(A[2]) @ Bs[1], A[3]]])
    green_rhs = np.concatenate([y[1] - Bs[0] @ inv(A[0]) @ y[0], y[3] - Bs[2] @ inv(A[2]) @ y[2]])
    xr = np.linalg.solve(red, red_rhs).reshape(2, n)
    xg = np.linalg.solve(green, green_rhs).reshape(2, n)
    np.testing.assert_allclose(xr, x[[0, 2]], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(xg, x[[1, 3]], rtol=1e-12, atol=1e-14)


def normalized_pcr(D, r):
    """The normalized reading of PCR: with sub-diagonal blocks -I, M_j = D_j^{-1},
    z_j = D_j^{-1} r_j, then ceil(log2 m) Jacobi-style levels reading the
    previous level: z_j += M_j z_{j-s}, M_j = M_j M_{j-s} for j >= s."""
    B, m, n, _ = D.shape
    M = np.linalg.inv(D)
    z = np.einsum("bjik,bjk->bji", M, r)
    s = 1
    while s < m:
        Mn, zn = M.copy(), z.copy()
        zn[:, s:] = z[:, s:] + np.einsum("bjik,bjk->bji", M[:, s:], z[:, :-s])
        Mn[:, s:] = np.einsum("bjik,bjkl->bjil", M[:, s:], M[:, :-s])
        M, z = Mn, zn
        s *= 2
    return z


def test_normalized_pcr_reading_equals_dense_for_every_length():
    rng = np.random.default_rng(6)
    for m in range(1, 66):
        D = random_blocks(rng, 2, m, 2)
        r = rng.standard_normal((2, m, 2))
        x = bb.dense_solve(D, r)
        assert np.abs(normalized_pcr(D, r) - x).max() <= 1e-11 * np.abs(x).max()
