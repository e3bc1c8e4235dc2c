"""Pins of the oracle's five-point stencil and matmul (CPU only)."""
import numpy as np


def test_stencil_quadratic_gives_four(orc):
    n = 9
    a = np.arange(n + 2, dtype=np.float64)
    A, B = np.meshgrid(a, a, indexing="ij")
    res = orc.stencil5(A ** 2 + B ** 2)
    np.testing.assert_array_equal(res, np.full((n, n), 4.0))


def test_stencil_cubic_in_rows_is_asymmetric(orc):
    """u[a][b] = a^3 gives 6(i+1) at output (i, j): a transposed index fails."""
    n = 7
    a = np.arange(n + 2, dtype=np.float64)
    A, B = np.meshgrid(a, a, indexing="ij")
    res = orc.stencil5(A ** 3)
    ref = 6.0 * (np.arange(n)[:, None] + 1) * np.ones((1, n))
    np.testing.assert_array_equal(res, ref)
    res_t = orc.stencil5(B ** 3)
    np.testing.assert_array_equal(res_t, ref.T)


def test_stencil_linear_is_zero(orc):
    a = np.arange(10, dtype=np.float64)
    A, B = np.meshgrid(a, a, indexing="ij")
    np.testing.assert_array_equal(orc.stencil5(3 * A - 2 * B + 1), np.zeros((8, 8)))


def test_stencil_vs_slicing(orc):
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 8):
        u = rng.uniform(-1, 1, size=(n + 2, n + 2))
        ref = u[:-2, 1:-1] + u[1:-1, :-2] - 4 * u[1:-1, 1:-1] + u[1:-1, 2:] + u[2:, 1:-1]
        np.testing.assert_allclose(orc.stencil5(u), ref, rtol=0, atol=1e-15)
        ii = rng.integers(0, n, size=5)
        jj = rng.integers(0, n, size=5)
        np.testing.assert_allclose(orc.stencil5_select(u, ii, jj), ref[ii, jj], rtol=0, atol=1e-15)


def test_matmul_identity_and_permutation(orc):
    rng = np.random.default_rng(1)
    n = 12
    a = rng.normal(size=(n, n))
    np.testing.assert_array_equal(orc.matmul(a, np.eye(n)), a)
    P = np.eye(n)[rng.permutation(n)]
    np.testing.assert_array_equal(orc.matmul(P, a), P @ a)


def test_matmul_small_integers_exact(orc):
    rng = np.random.default_rng(2)
    a = rng.integers(-5, 6, size=(17, 17)).astype(np.float64)
    b = rng.integers(-5, 6, size=(17, 17)).astype(np.float64)
    c = orc.matmul(a, b)
    np.testing.assert_array_equal(c, (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64))
    ii = np.array([0, 16, 5])
    jj = np.array([3, 16, 0])
    np.testing.assert_array_equal(orc.matmul_select(a, b, ii, jj), c[ii, jj])


def test_matmul_nonsymmetric_order(orc):
    """c = a b, not b a or a^T b."""
    a = np.array([[1.0, 2.0], [0.0, 1.0]])
    b = np.array([[1.0, 0.0], [3.0, 1.0]])
    np.testing.assert_array_equal(orc.matmul(a, b), np.array([[7.0, 2.0], [3.0, 1.0]]))
