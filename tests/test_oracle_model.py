"""Pins of the oracle's least-squares calibration, prediction and error
statistics (CPU only)."""
import math

import numpy as np
import pytest

from oracle import model as M


def test_fit_recovers_consistent_parameters():
    rng = np.random.default_rng(0)
    F = rng.uniform(1.0, 10.0, size=(40, 6)) * np.array([1e9, 1e6, 1e3, 1.0, 1e-3, 1e7])
    p_true = np.array([2e-12, 3e-9, 1e-6, 5e-3, 7.0, 4e-11])
    t = F @ p_true
    for rel in (True, False):
        out = M.fit(F, t, relative=rel)
        np.testing.assert_allclose(out["p"], p_true, rtol=1e-10)
        assert out["rank"] == 6
        assert out["resid"] < 1e-10 * (1 if rel else np.linalg.norm(t))
        assert out["negative"] == []


def test_fit_relative_is_row_scaled_least_squares():
    """Relative fit minimises sum_k (1 - f_k.p / t_k)^2: check the normal
    equations (gradient zero) at the solution of a noisy, full-rank system."""
    rng = np.random.default_rng(1)
    F = rng.uniform(1, 5, size=(30, 3))
    t = F @ np.array([1.0, 2.0, 3.0]) * rng.uniform(0.9, 1.1, size=30)
    p = M.fit(F, t, relative=True)["p"]
    A = F / t[:, None]
    grad = A.T @ (A @ p - 1.0)
    assert np.max(np.abs(grad)) < 1e-10


def test_fit_rank_deficient_min_norm():
    """Duplicated column: the solution splits the weight evenly (min-norm in
    the equilibrated coordinates) and the rank is reported."""
    rng = np.random.default_rng(2)
    a = rng.uniform(1, 2, size=20)
    b = rng.uniform(1, 2, size=20)
    F = np.stack([a, a, b], axis=1)
    t = 4.0 * a + 1.0 * b
    out = M.fit(F, t, relative=False)
    assert out["rank"] == 2
    np.testing.assert_allclose(out["p"], [2.0, 2.0, 1.0], rtol=1e-10)


def test_fit_flags_negative_and_rejects_bad_input():
    F = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    t = np.array([1.0, -0.5, 0.5])
    assert M.fit(F, t, relative=False)["negative"] == [1]
    with pytest.raises(ValueError):
        M.fit(F, t, relative=True)            # t <= 0
    with pytest.raises(ValueError):
        M.fit(np.zeros((0, 2)), np.zeros(0))
    with pytest.raises(ValueError):
        M.fit(np.array([[np.nan, 1.0]]), np.array([1.0]))


def test_predict_mape_geomean():
    F = np.array([[1.0, 2.0], [3.0, 4.0]])
    p = np.array([0.5, 0.25])
    np.testing.assert_allclose(M.predict(F, p), [1.0, 2.5])
    assert M.mape([1.1, 1.8], [1.0, 2.0]) == pytest.approx(0.1)
    assert M.geomean_rel_err([1.1, 1.8], [1.0, 2.0]) == pytest.approx(0.1)
    assert M.geomean_rel_err([1.0, 2.2], [1.0, 2.0]) == pytest.approx(math.sqrt(1e-6 * 0.1))


def test_overlap_model_shape():
    """The switched sum reduces to max(c_g, c_o) + c_ovh when the edge is sharp
    and to the average of the two when the costs are equal."""
    F = np.array([[1.0, 2.0, 5.0], [1.0, 6.0, 1.0], [1.0, 3.0, 3.0]])
    group = [0, 1, 2]
    p = [1.0, 1.0, 1.0]
    t = M.overlap_predict(F, group, p, edge=1e6)
    np.testing.assert_allclose(t, [1 + 5, 1 + 6, 1 + 3], rtol=1e-12)
    t0 = M.overlap_predict(F, group, p, edge=0.0)
    np.testing.assert_allclose(t0, [1 + 3.5, 1 + 3.5, 1 + 3], rtol=1e-12)


def test_overlap_fit_recovers_law():
    rng = np.random.default_rng(11)
    F = np.column_stack([np.ones(40), rng.integers(16, 4096, 40), rng.uniform(1e8, 1e10, 40),
                         rng.uniform(1e8, 1e10, 40), rng.uniform(1e11, 1e13, 40)])
    group = [0, 0, 1, 1, 2]
    p_true = np.array([5e-6, 2e-9, 2e-13, 1.5e-13, 7e-15])
    edge_true = 3e4
    t = M.overlap_predict(F, group, p_true, edge_true)
    fit = M.overlap_fit(F, t, group, p_true * rng.uniform(0.7, 1.4, 5), edge_true * 0.6)
    assert np.max(np.abs(M.overlap_predict(F, group, fit["p"], fit["edge"]) / t - 1)) < 1e-6


def _nnls_brute_force(A, b):
    """Exact NNLS of a tiny system: over every support set S, the
    unconstrained least-squares solution on S, kept if it is >= 0; the
    feasible one of least residual is the minimiser (the optimum is the
    unconstrained optimum on its own support)."""
    import itertools
    n = A.shape[1]
    best, best_r = np.zeros(n), np.linalg.norm(b)
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            x = np.zeros(n)
            x[list(S)] = np.linalg.lstsq(A[:, S], b, rcond=None)[0]
            if np.all(x >= 0):
                r = np.linalg.norm(A @ x - b)
                if r < best_r - 1e-14:
                    best, best_r = x, r
    return best


def _negative_case(seed):
    """Timings from a law with one cost column that the data would fit with a
    negative weight: the last feature is nearly a difference of two others."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(1.0, 10.0, size=(25, 4)) * np.array([1e3, 1e6, 1e9, 1e6])
    F[:, 3] = 0.9 * F[:, 1] + rng.uniform(0, 3e5, 25)
    t = F[:, :3] @ np.array([1e-6, 2e-9, 3e-12]) - 1e-9 * F[:, 3] * 0.5
    t *= rng.uniform(0.95, 1.05, 25)
    return F, np.abs(t) + 1e-6


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("relative", [True, False])
def test_nonneg_fit_is_brute_force_nnls(seed, relative):
    F, t = _negative_case(seed)
    un = M.fit(F, t, relative=relative)
    out = M.fit(F, t, relative=relative, nonneg=True)
    assert np.all(out["p"] >= 0)
    A = F / t[:, None] if relative else F
    b = np.ones_like(t) if relative else t
    sc = 1.0 / np.linalg.norm(A, axis=0)
    ref = _nnls_brute_force(A * sc, b) * sc
    np.testing.assert_allclose(out["p"], ref, rtol=1e-8, atol=1e-12 * np.max(np.abs(ref)))
    if not un["negative"]:
        np.testing.assert_allclose(out["p"], un["p"], rtol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_nonneg_fit_kkt(seed):
    """Karush-Kuhn-Tucker conditions of min ||A p - b||, p >= 0: with
    g = A^T (A p - b), g_j = 0 where p_j > 0 and g_j >= 0 where p_j = 0."""
    F, t = _negative_case(seed)
    p = M.fit(F, t, relative=True, nonneg=True)["p"]
    A = F / t[:, None]
    sc = 1.0 / np.linalg.norm(A, axis=0)
    y = p / sc
    g = (A * sc).T @ ((A * sc) @ y - 1.0)
    tol = 1e-9 * np.sqrt(len(t))
    assert np.all(y >= 0)
    assert np.all(np.abs(g[y > 0]) <= tol)
    assert np.all(g[y == 0] >= -tol)


def test_overlap_fit_nonneg_bounds():
    rng = np.random.default_rng(12)
    F = np.column_stack([np.ones(40), rng.integers(16, 4096, 40), rng.uniform(1e8, 1e10, 40),
                         rng.uniform(1e8, 1e10, 40), rng.uniform(1e11, 1e13, 40)])
    group = [0, 0, 1, 1, 2]
    p_true = np.array([5e-6, 0.0, 2e-13, 1.5e-13, 7e-15])
    t = M.overlap_predict(F, group, p_true, 3e4) * rng.uniform(0.98, 1.02, 40)
    fit = M.overlap_fit(F, t, group, np.abs(p_true) + 1e-10, 2e4, nonneg=True)
    assert np.all(fit["p"] >= 0)
    assert M.mape(M.overlap_predict(F, group, fit["p"], fit["edge"]), t) < 0.02
