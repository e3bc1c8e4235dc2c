"""Pins of the measurement kernels' oracle definitions (CPU only): closed
forms and an independent construction of each."""
import numpy as np

from oracle import ubench as U


def test_stream_and_strided():
    a, b = np.arange(12.0), np.arange(12.0) * 3
    np.testing.assert_array_equal(U.stream([a, b]), 4 * np.arange(12.0))
    np.testing.assert_array_equal(U.strided(np.arange(100.0), 10, 7), np.arange(10.0) * 7)


def test_fma_closed_form_and_update_matrix():
    # no trips: sum_v (t/256 + v/32) = t/8 + 31*32/2/32
    t = np.arange(512) % 256
    np.testing.assert_array_equal(U.fma(2, 0), t / 8 + 15.5)
    # one trip = 64 updates, each the identity but row v: -1/2 at v, 1 at v+16
    M = np.eye(32)
    for k in range(64):
        v = k % 32
        step = np.eye(32)
        step[v] = 0.0
        step[v, v] = -0.5
        step[v, (v + 16) % 32] = 1.0
        M = step @ M
    r0 = np.array([[tt * 2.0 ** -8 + v * 2.0 ** -5 for v in range(32)] for tt in range(256)])
    for iters in (1, 2, 3):
        r = r0 @ np.linalg.matrix_power(M, iters).T
        np.testing.assert_allclose(U.fma(1, iters), r.sum(axis=1), rtol=0, atol=1e-12)


def test_mfma_against_a_matrix_product():
    lanes = np.arange(64)
    a = (3 * lanes) % 7 - 3
    b = (5 * lanes) % 9 - 4
    A = np.array([[a[i + 16 * k] for k in range(4)] for i in range(16)], dtype=float)   # 16 x 4
    B = np.array([[b[j + 16 * k] for j in range(16)] for k in range(4)], dtype=float)   # 4 x 16
    D = A @ B
    w = U.mfma(1, 3, "f32").reshape(4, 64, 4)[0]
    for l in (0, 5, 17, 38, 63):
        for r in range(4):
            assert w[l, r] == 8 * 3 * D[4 * (l // 16) + r, l % 16]
    # 32-deep BF16 products: each lane's value fills 8 of the k positions
    wb = U.mfma(1, 1, "bf16").reshape(4, 64, 4)[0]
    np.testing.assert_array_equal(wb, 8 * 8 * w / (8 * 3))


def test_rotations():
    x = np.arange(2 * 256 * 4, dtype=float)
    np.testing.assert_array_equal(U.lds(x, 2, 64, 4), x)          # a full turn
    y = U.lds(x, 2, 1, 4).reshape(-1, 4)
    np.testing.assert_array_equal(y[0], x.reshape(-1, 4)[1])       # lane 0 takes lane 1's
    np.testing.assert_array_equal(y[63], x.reshape(-1, 4)[0])      # lane 63 takes lane 0's
    n4 = 300
    v = np.arange(4 * n4, dtype=float) + 1
    o = U.overlap(v, n4, 1).reshape(-1, 4)
    np.testing.assert_array_equal(o[0], v.reshape(-1, 4)[1])
    # vector 299 is lane 43 of wave 4 (256 + 43); lane 44 of that wave is past the end
    np.testing.assert_array_equal(o[299], np.zeros(4))
    np.testing.assert_array_equal(U.overlap(v, n4, 64), v)


def test_tile_read_patterns():
    """Pattern a sums each row's values in column class j mod 16, pattern b
    each column's values in row class i mod 16 (built here by reshapes)."""
    rng = np.random.default_rng(3)
    for n in (16, 48):
        x = rng.integers(-9, 9, (n, n)).astype(np.float64)
        a = x.reshape(n, n // 16, 16).sum(axis=1)            # [i][j mod 16]
        b = x.reshape(n // 16, 16, n).sum(axis=0)            # [i mod 16][j]
        want_a = np.array([[a[i, j % 16] for j in range(n)] for i in range(n)])
        want_b = np.array([[b[i % 16, j] for j in range(n)] for i in range(n)])
        np.testing.assert_array_equal(U.tile_read(x, n, 0), want_a.reshape(-1))
        np.testing.assert_array_equal(U.tile_read(x, n, 1), want_b.reshape(-1))
