"""Symbolic counting over the affine loop-nest IR (paper_1904_09538_amd/affine.py,
the paper's Section "Gathering Kernel Statistics").

Pins: the paper's worked triangle domain against brute-force enumeration and
its closed form; the IR schedules of the stencil, the matmul and the DG
forward against the library's closed-form counts (themselves pinned to the
hardware counters in test_counters.py); the reconstructed quasi-polynomials
against direct enumeration at sizes they were not built from; the stencil's
footprint and access-to-footprint ratio against their plain definitions."""
from fractions import Fraction

import pytest

from paper_1904_09538_amd import affine as A


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _feats(L, *args, **kw):
    return dict(zip(L.feature_names(), (int(x) for x in L.perf_features_count(*args, **kw))))


@pytest.mark.parametrize("n,p", [(0, 0), (5, 0), (5, 2), (9, 4), (3, 7)])
def test_triangle_count_is_brute_force(n, p):
    want = sum(1 for i in range(p, n) for j in range(p, i + 1))
    assert A.count(A.triangle(), {"n": n, "p": p}).get("point", 0) == want


def test_triangle_quasi_polynomial_is_the_closed_form():
    # interpolation points inside the chamber p <= n: n from 10, p from 0
    q = A.symbolic_count(A.triangle(), "point", ["n", "p"], {}, start=[10, 0], degree=2)
    assert q.is_polynomial()
    for n in range(0, 12):
        for p in range(0, n + 1):
            # (n - p)(n - p + 1) / 2 points on the chamber p <= n
            assert q(n=n, p=p) == Fraction((n - p) * (n - p + 1), 2)


def test_quasi_polynomial_period_from_floor_divisors():
    # ceil(n / 4) trips of 3 operations: a quasi-polynomial of period 4
    k = [A.loop("b", 0, A.ceil_div("n", 4), A.Stmt("s", {"op": 3}))]
    q = A.symbolic_count(k, "op", ["n"], {}, start=[0])
    assert q.period == 4 and not q.is_polynomial()
    for n in (0, 1, 5, 1003, 10 ** 9 + 7):
        assert q(n=n) == 3 * (-(-n // 4))


def test_quasi_polynomial_rejects_wrong_degree():
    k = A.triangle()
    with pytest.raises(ValueError):
        A.quasi_polynomial(lambda n, p: A.count(k, {"n": n, "p": p}).get("point", 0), ["n", "p"],
                           period=1, degree=1, start=[10, 0])


@pytest.mark.parametrize("n", [4, 260, 516])
def test_stencil_schedule_matches_closed_form(L, n):
    f = _feats(L, "stencil", "f32", n)
    c = A.count(A.stencil_vec(4), {"n": n})
    assert c["bytes:u"] == f["gld_st_u"]
    assert c["bytes:res"] == f["gst_st_res"]
    assert c["flops"] == f["valu_f32"]


@pytest.mark.parametrize("n", [16, 144])
def test_matmul_schedule_matches_closed_form(L, n):
    f = _feats(L, "matmul", "f32", n, num_cu=256)
    c = A.count(A.matmul_tiles(), {"n": n})
    assert c["bytes:a"] + c["bytes:b"] == f["gld_mm_ab"]
    assert c["bytes:c"] == f["gst_mm_c"]
    assert c["mfma_flops"] == f["mfma_f32"]


@pytest.mark.parametrize("E", [1, 17, 100])
def test_dg_schedule_matches_closed_form(L, E):
    # order 5 (216 nodes, K padded to 224 = 4 x 56), 16 elements per wave-tile,
    # 11 panels resident of 42, so four operator groups each re-read u
    tile = {"elems_per_wave": 16, "waves": 8, "groups_per_cu": 1, "d_panels": 11}
    f = _feats(L, "dg", "f32", E, 216, 3, tile, 256)
    c = A.count(A.dg_vec(216, 56, 1, 4), {"E": E})
    assert c["bytes:u"] == f["gld_dg_u"]
    assert c["bytes:u_l2"] == f["gld_dg_u_l2"]
    assert c["bytes:out"] == f["gst_dg_out"]
    assert c["mfma_flops"] == f["mfma_f32"]


def test_dg_symbolic_counts_extrapolate():
    k = A.dg_vec(64, 16, 1, 1)
    out = A.symbolic_count(k, "bytes:out", ["E"], {}, start=[1], degree=1, period=16)
    mf = A.symbolic_count(k, "mfma_flops", ["E"], {}, start=[1], degree=1, period=16)
    assert out.is_polynomial() and out(E=10 ** 6) == 3 * 64 * 4 * 10 ** 6
    for E in (33, 250):
        assert mf(E=E) == A.count(k, {"E": E})["mfma_flops"]
    assert mf(E=10 ** 6 + 3) == 3 * 4 * 16 * 2048 * (-(-(10 ** 6 + 3) // 16))


@pytest.mark.parametrize("n", [1, 6, 13])
def test_stencil_footprint_and_afr(n):
    k = A.stencil_reference()
    # the five-point neighbourhoods of the n x n interior cover the (n + 2)^2
    # grid less its four corners
    assert A.footprint(k, {"n": n}, "u") == (n + 2) ** 2 - 4
    assert A.afr(k, {"n": n}, "u") == Fraction(5 * n * n, (n + 2) ** 2 - 4)
    assert A.afr(k, {"n": n}, "res") == 1
