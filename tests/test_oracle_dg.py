"""Pins of the DG inputs and the FP64 oracle to closed forms, invariants,
library routines and brute force (CPU only)."""
import math

import numpy as np
import pytest

from paper_1904_09538_amd import inputs as I

# ---------------------------------------------------------------- GLL nodes / D1


def _closed_form_nodes(p):
    """Interior GLL nodes in closed form (roots of P_p')."""
    if p == 1:
        return [-1.0, 1.0]
    if p == 2:
        return [-1.0, 0.0, 1.0]
    if p == 3:
        s = 1 / math.sqrt(5)
        return [-1.0, -s, s, 1.0]
    if p == 4:
        s = math.sqrt(3 / 7)
        return [-1.0, -s, 0.0, s, 1.0]
    if p == 5:
        a = math.sqrt(1 / 3 - 2 * math.sqrt(7) / 21)
        b = math.sqrt(1 / 3 + 2 * math.sqrt(7) / 21)
        return [-1.0, -b, -a, a, b, 1.0]
    if p == 6:
        a = math.sqrt((15 - 2 * math.sqrt(15)) / 33)
        b = math.sqrt((15 + 2 * math.sqrt(15)) / 33)
        return [-1.0, -b, -a, 0.0, a, b, 1.0]
    if p == 7:
        # y = x^2 solves 3003 y^3 - 3465 y^2 + 945 y - 35 = 0
        ys = sorted(np.roots([3003.0, -3465.0, 945.0, -35.0]).real)
        r = [math.sqrt(y) for y in ys]
        return [-1.0] + [-v for v in reversed(r)] + r + [1.0]
    raise ValueError


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_nodes_closed_form(p):
    x = I.gll_nodes(p)
    np.testing.assert_allclose(x, _closed_form_nodes(p), atol=1e-14, rtol=0)


def test_gll_d1_p3_worked_values():
    d = I.gll_diff_1d(3)
    s5 = math.sqrt(5)
    row0 = [-3.0, (5 + 5 * s5) / 4, -(5 * s5 - 5) / 4, 0.5]
    row1 = [-(1 + s5) / 4, 0.0, s5 / 2, -(s5 - 1) / 4]
    np.testing.assert_allclose(d[0], row0, atol=1e-13)
    np.testing.assert_allclose(d[1], row1, atol=1e-13)
    # rows 2,3 by centro-antisymmetry D[p-i][p-j] = -D[i][j]
    np.testing.assert_allclose(d[::-1, ::-1], -d, atol=1e-13)


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_d1_differentiates_polynomials(p):
    x = I.gll_nodes(p)
    d = I.gll_diff_1d(p)
    for k in range(p + 1):
        deriv = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(d @ x ** k - deriv)) <= 3e-13 * max(1, p ** 2)
    assert np.max(np.abs(d.sum(axis=1))) < 1e-13 * p * p


# ---------------------------------------------------------------- DG forward


def _nodal_monomial(p, a, b, c):
    x = I.gll_nodes(p)
    X0, X1, X2 = np.meshgrid(x, x, x, indexing="ij")   # axis 0 slowest
    return (X0 ** a * X1 ** b * X2 ** c).ravel(), (X0, X1, X2)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_dg_forward_exact_on_polynomials(orc, p):
    """D_m applied to nodal x^a y^z z^c (a,b,c <= p) is the exact derivative
    along axis m at the nodes; constants map to 0."""
    D = I.gll_dmats(p)
    rng = np.random.default_rng(11)
    elems, derivs = [], []
    for _ in range(6):
        a, b, c = (int(v) for v in rng.integers(0, p + 1, size=3))
        f, (X0, X1, X2) = _nodal_monomial(p, a, b, c)
        elems.append(f)
        d0 = (a * X0 ** max(a - 1, 0) * X1 ** b * X2 ** c).ravel()
        d1 = (b * X0 ** a * X1 ** max(b - 1, 0) * X2 ** c).ravel()
        d2 = (c * X0 ** a * X1 ** b * X2 ** max(c - 1, 0)).ravel()
        derivs.append(np.stack([d0, d1, d2]))
    elems.append(np.full((p + 1) ** 3, 3.5))                 # a constant
    derivs.append(np.zeros((3, (p + 1) ** 3)))
    u = np.stack(elems)
    out = orc.dg_forward(D, u)
    ref = np.stack(derivs, axis=1)                          # [3][E][n]
    scale = max(1.0, float(np.max(np.abs(ref))))
    assert np.max(np.abs(out - ref)) <= 1e-12 * scale * p * p


def test_dg_forward_brute_force_vs_einsum(orc):
    rng = np.random.default_rng(5)
    for nmat in (1, 2, 3):
        for nunit in (1, 3, 8):
            for nelem in (1, 2, 5):
                D = rng.normal(size=(nmat, nunit, nunit))
                u = rng.normal(size=(nelem, nunit))
                out = orc.dg_forward(D, u)
                ref = np.einsum("mij,ej->mei", D, u)
                np.testing.assert_allclose(out, ref, rtol=1e-14, atol=1e-14)


def test_dg_forward_integer_exact_and_asymmetric(orc):
    """Integer data: exact.  A non-symmetric D catches a transposed operand and
    distinct matrices catch a wrong m index."""
    rng = np.random.default_rng(9)
    D = rng.integers(-4, 5, size=(3, 7, 7)).astype(np.float64)
    u = rng.integers(-8, 9, size=(4, 7)).astype(np.float64)
    out = orc.dg_forward(D, u)
    for m in range(3):
        for e in range(4):
            for i in range(7):
                assert out[m, e, i] == sum(D[m, i, j] * u[e, j] for j in range(7))


def test_dg_forward_select_matches_full(orc):
    D = I.random_dmats(27)
    u = I.uniform_u(50, 27)
    full = orc.dg_forward(D, u)
    sel = np.array([0, 7, 49, 13])
    part = orc.dg_forward_select(D, u, sel)
    np.testing.assert_array_equal(part, full[:, sel, :].transpose(1, 0, 2))


def test_dg_batched_reduces_to_plain(orc):
    order = I.batched_orders(40, seed=2, max_order=4)
    off = I.batched_offsets(order)
    D_sets = {p: I.gll_dmats(p) for p in range(1, 5)}
    u = np.random.default_rng(0).uniform(-1, 1, size=int(off[-1]))
    out = orc.dg_batched(order, off, D_sets, u)
    for e in range(40):
        p = int(order[e])
        n = (p + 1) ** 3
        ref = orc.dg_forward(D_sets[p], u[off[e]:off[e] + n][None, :])[:, 0, :]
        np.testing.assert_array_equal(out[:, off[e]:off[e] + n], ref)


def test_batched_orders_distribution():
    o = I.batched_orders(200000)
    ps = np.arange(1, 8)
    w = 1 / (ps + 1)
    w /= w.sum()
    freq = np.array([(o == p).mean() for p in ps])
    assert np.max(np.abs(freq - w)) < 0.005
    assert o.min() >= 1 and o.max() <= 7


# ---------------------------------------------------------------- adjoint


def test_adjoint_dot_product_identity(orc):
    """out is linear in u and in D, so <g, out> = <grad_u, u> = <grad_D, D>."""
    rng = np.random.default_rng(3)
    D = rng.normal(size=(3, 27, 27))
    u = rng.normal(size=(17, 27))
    g = rng.normal(size=(3, 17, 27))
    out = orc.dg_forward(D, u)
    gu, gD = orc.dg_adjoint(D, u, g)
    L = float(np.sum(g * out))
    assert abs(float(np.sum(gu * u)) - L) <= 1e-12 * abs(L) + 1e-12
    assert abs(float(np.sum(gD * D)) - L) <= 1e-12 * abs(L) + 1e-12


def test_adjoint_central_differences(orc):
    """L is linear in each argument: central differences have no truncation
    error, so they equal the analytic gradient to rounding."""
    rng = np.random.default_rng(4)
    D = rng.normal(size=(2, 5, 5))
    u = rng.normal(size=(3, 5))
    g = rng.normal(size=(2, 3, 5))
    gu, gD = orc.dg_adjoint(D, u, g)
    h = 1e-6

    def L(Dx, ux):
        return float(np.sum(g * orc.dg_forward(Dx, ux)))
    for idx in np.ndindex(u.shape):
        up, um = u.copy(), u.copy()
        up[idx] += h
        um[idx] -= h
        assert abs((L(D, up) - L(D, um)) / (2 * h) - gu[idx]) < 1e-8
    for idx in np.ndindex(D.shape):
        Dp, Dm = D.copy(), D.copy()
        Dp[idx] += h
        Dm[idx] -= h
        assert abs((L(Dp, u) - L(Dm, u)) / (2 * h) - gD[idx]) < 1e-8


def test_adjoint_vs_einsum(orc):
    rng = np.random.default_rng(8)
    D = rng.normal(size=(3, 8, 8))
    u = rng.normal(size=(6, 8))
    g = rng.normal(size=(3, 6, 8))
    gu, gD = orc.dg_adjoint(D, u, g)
    np.testing.assert_allclose(gu, np.einsum("mij,mei->ej", D, g), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gD, np.einsum("mei,ej->mij", g, u), rtol=1e-13, atol=1e-13)
    only_u, none_d = orc.dg_adjoint(D, u, g, want_D=False)
    assert none_d is None
    np.testing.assert_array_equal(only_u, gu)


def test_adjoint_D_select_matches_full(orc):
    rng = np.random.default_rng(6)
    u = rng.normal(size=(40, 8))
    g = rng.normal(size=(3, 40, 8))
    _, gD = orc.dg_adjoint(rng.normal(size=(3, 8, 8)), u, g)
    mm, ii, jj = np.array([0, 2, 1]), np.array([7, 0, 3]), np.array([1, 7, 3])
    np.testing.assert_array_equal(orc.dg_adjoint_D_select(u, g, mm, ii, jj), gD[mm, ii, jj])
