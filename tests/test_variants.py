"""Program variants on the host (no GPU): the library's closed-form counts
(perf_variant_count) against the oracle's brute-force walk of the same
schedules, for every variant, every work-removed twin and ragged sizes;
argument validation; and the oracle's twin outputs pinned to the walk (on
all-ones inputs a work-item's sum is the number of loads it issues, so the
sums over all work-items must equal the walk's kept load bytes / 4) and to
small cases worked by hand."""
import numpy as np
import pytest

from oracle import variants as OV

ALL_KEEPS = [(False, 0)] + [(True, k) for k in range(8)]


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _cases():
    out = []
    for n in (0, 16, 48, 64):
        out += [("mm_pf", dict(n=n)), ("mm_nopf", dict(n=n))]
    for k in ("dg_nopf", "dg_pfu", "dg_pfdm", "dg_pfdmt"):
        for E, nu, M in ((0, 64, 3), (1, 64, 3), (17, 64, 3), (40, 32, 1), (33, 16, 8), (16, 48, 2)):
            out.append((k, dict(n=E, nunit=nu, nmat=M)))
    for k in ("fd16", "fd18"):
        for n in (0, 1, 13, 14, 15, 16, 17, 30, 33):
            out.append((k, dict(n=n, ld_u=n + 2, ld_res=max(n, 1))))
    return out


def test_feature_names_agree(L, orc):
    assert L.variant_feature_names() == orc.VARIANT_FEATURES


@pytest.mark.parametrize("kind,kw", _cases())
def test_closed_form_is_the_walk(L, orc, kind, kw):
    for twin, keep in ALL_KEEPS:
        if kind.startswith("fd") and keep & 2:
            continue
        got = L.perf_variant_count(kind, work_removed=twin, keep=keep, **kw)
        want = orc.variant_features(kind, kw["n"], kw.get("nunit", 0), kw.get("nmat", 0), twin, keep)
        np.testing.assert_array_equal(got, want, err_msg=f"{kind} {kw} twin={twin} keep={keep}")


def test_counts_of_the_paper_shapes(L):
    f = dict(zip(L.variant_feature_names(), L.perf_variant_count("dg_pfdmt", 1 << 10, nunit=64, nmat=3)))
    # 64 x 4 work-groups of 256: 3 x 64 u loads and 3 x 4 D tile loads per work-item
    assert f["workgroups"] == 256 and f["gld_dg_dmpft_u"] == 4 * 3 * 64 * 65536
    assert f["gld_dg_dmpf_dm"] == 4 * 3 * 4 * 65536 and f["barrier_x_wg"] == 2 * 3 * 4 * 256
    assert f["valu_f32_sg"] == 2 * 3 * 64 * 64 * (1 << 10)     # 2 nmat nunit^2 nelem
    s = dict(zip(L.variant_feature_names(), L.perf_variant_count("fd18", 32, ld_u=34, ld_res=32)))
    assert s["workgroups"] == 4 and s["gld_fd18_u"] == 4 * 324 * 4 and s["gst_fd18_res"] == 4 * 32 * 32


@pytest.mark.parametrize("kind,kw", [
    ("mm_pf", dict(n=24)), ("mm_nopf", dict(n=-16)), ("dg_nopf", dict(n=5, nunit=24, nmat=3)),
    ("dg_pfu", dict(n=5, nunit=64, nmat=9)), ("dg_pfdm", dict(n=5, nunit=528, nmat=3)),
    ("fd16", dict(n=10, ld_u=11, ld_res=10)), ("fd18", dict(n=10, ld_u=12, ld_res=9))])
def test_refused_shapes(L, orc, kind, kw):
    with pytest.raises(L.DGError):
        L.perf_variant_count(kind, **kw)
    with pytest.raises(L.DGError):
        L.variant_shape(kind, **kw)


def test_refused_keeps(L, orc):
    with pytest.raises(L.DGError):
        L.perf_variant_count("dg_nopf", 16, nunit=64, nmat=3, keep=1)            # keep on a full kernel
    with pytest.raises(L.DGError):
        L.perf_variant_count("fd16", 16, ld_u=18, ld_res=16, work_removed=True, keep=2)
    with pytest.raises(L.DGError):
        L.perf_variant_count("mm_pf", 16, work_removed=True, keep=8)
    with pytest.raises(ValueError):
        orc.variant_features("fd16", 16, 0, 0, True, 2)


def test_run_validates_before_launch(L):
    # rejected descriptors and NULL arrays return before anything touches a GPU
    import ctypes
    d = L._v_desc("dg_nopf", 16, 24, 3)
    assert L.lib().dg_variant_run(ctypes.byref(d), None, None, None, None) == L.DG_EINVAL
    d = L._v_desc("mm_pf", 32)
    assert L.lib().dg_variant_run(ctypes.byref(d), None, None, None, None) == L.DG_EINVAL
    d = L._v_desc("dg_nopf", 0, 64, 3)              # nothing to do
    assert L.lib().dg_variant_run(ctypes.byref(d), None, None, None, None) == L.DG_OK


def _sizes(kind, kw):
    n, nu, M = kw["n"], kw.get("nunit", 0), kw.get("nmat", 0)
    if kind.startswith("mm"):
        return np.ones((n, n)), np.ones((n, n))
    if kind.startswith("dg"):
        return np.ones((n, nu) if kind != "dg_pfdmt" else (nu, n)), np.ones((M, nu, nu))
    return np.ones((n + 2, n + 2)), None


LOADS = {"mm_pf": ("gld_mm_pf_a", "gld_mm_pf_b"), "mm_nopf": ("gld_mm_nopf_a", "gld_mm_nopf_b"),
         "dg_nopf": ("gld_dg_nopf_u", "gld_dg_dm"), "dg_pfu": ("gld_dg_upf_u", "gld_dg_dm"),
         "dg_pfdm": ("gld_dg_dmpf_u", "gld_dg_dmpf_dm"), "dg_pfdmt": ("gld_dg_dmpft_u", "gld_dg_dmpf_dm"),
         "fd16": ("gld_fd16_u", None), "fd18": ("gld_fd18_u", None)}


@pytest.mark.parametrize("kind,kw", [c for c in _cases() if c[1]["n"] > 0])
def test_twin_sums_count_the_walks_loads(orc, kind, kw):
    """All-ones inputs: each work-item's sum is its number of kept loads."""
    a, b = _sizes(kind, kw)
    names = orc.VARIANT_FEATURES
    for keep in (1, 2, 3):
        if kind.startswith("fd") and keep & 2:
            continue
        dest, res = OV.twin(kind, keep, kw["n"], a, b, kw.get("nunit", 0), kw.get("nmat", 0))
        assert res is None
        c = dict(zip(names, orc.variant_features(kind, kw["n"], kw.get("nunit", 0), kw.get("nmat", 0), True, keep)))
        want = (c[LOADS[kind][0]] if keep & 1 else 0) + (c[LOADS[kind][1]] if keep & 2 else 0)
        assert dest.sum() == want // 4
        assert dest.size * 4 == c["gst_ub"]


def test_twin_hand_cases():
    # untiled matmul keeping a: every c[i][j] is the row sum of a
    a = np.arange(16 * 16, dtype=np.float64).reshape(16, 16)
    _, res = OV.twin("mm_nopf", 1 | 4, 16, a, None)
    assert np.array_equal(res, np.repeat(a.sum(axis=1)[:, None], 16, axis=1))
    # tiled matmul keeping b, n = 32: work-item (i, j) loads b[i % 16][j] and b[16 + i % 16][j]
    b = np.arange(32 * 32, dtype=np.float64).reshape(32, 32)
    _, res = OV.twin("mm_pf", 2 | 4, 32, None, b)
    assert res[5, 7] == b[5, 7] + b[21, 7] and res[21, 7] == res[5, 7]
    # stencil keeping its input and result: res = the grid's top-left n x n block
    u = np.arange(7 * 7, dtype=np.float64).reshape(7, 7)
    _, res = OV.twin("fd16", 1 | 4, 5, u, ld_res=6)
    assert np.array_equal(res[:, :5], u[:5, :5]) and np.all(np.isnan(res[:, 5]))
    # an 18 x 18 work-group's last work-item (row 17, column 17) of group (0, 0)
    dest, _ = OV.twin("fd18", 1, 40, np.arange(42 * 42, dtype=np.float64).reshape(42, 42))
    assert dest[323] == 17 * 42 + 17
    # nothing kept: zeros, one per work-item
    dest, _ = OV.twin("dg_pfu", 0, 20, nunit=32, nmat=3)
    assert dest.shape == (2 * 2 * 256,) and not dest.any()


def test_study_recovers_a_known_model(L, tmp_path):
    """The study's analysis on synthetic times drawn from a known overlap
    model over the plan's exact counts: the calibration (measurement kernels
    only) must reproduce the variants' times and their order."""
    import json
    from paper_1904_09538_amd import variant_study as V
    names = L.variant_feature_names()
    rng = np.random.default_rng(3)
    truth = {k: float(rng.uniform(0.5, 2.0)) * s for k, s in
             {"launch": 4e-6, "workgroups": 1e-10, "barrier_x_wg": 2e-11, "valu_f32_sg": 8e-15, "lds_sg": 1.5e-14}
             .items()}
    for k in names:
        truth.setdefault(k, float(rng.uniform(0.3, 3.0)) * 1e-13)
    group = [V.group_of(k) for k in names]
    p = np.array([truth[k] for k in names])
    rows = [dict(r, features=V.counts(r, L)) for r in V.plan(quick=True)]
    F = np.array([r["features"] for r in rows], dtype=np.float64)
    t = L.perf_model_predict_overlap(F, group, p, 5e4)
    path = tmp_path / "rows.jsonl"
    with open(path, "w") as fh:
        fh.write(json.dumps({"meta": True, "device": "synthetic", "feature_names": names}) + "\n")
        for r, tr in zip(rows, t):
            fh.write(json.dumps(dict(r, t={"mean": float(tr)})) + "\n")
    s = V.fit(str(path), L)
    assert s["n_variant_rows"] == sum(1 for r in rows if r["set"] == "variant")
    for v, d in s["per_variant"].items():
        assert d["geomean_rel_err_overlap"] < 0.02, (v, d)
    for fam, r in s["ranking"].items():
        assert r["kendall_tau_mean"] == 1.0, fam
