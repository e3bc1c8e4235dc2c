"""The library's closed-form operation counts against the oracle's brute-force
enumeration of the same documented schedules (bit-exact int64), the paper's
worked point-count example, and the library's FP64 model fit against the
oracle fit (CPU only)."""
import ctypes
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def test_feature_names_agree(orc, L):
    assert L.feature_names() == orc.FEATURES


@pytest.mark.parametrize("p,n", [(0, 0), (0, 1), (2, 7), (3, 3), (1, 11), (5, 40)])
def test_paper_point_count_example(orc, p, n):
    """#{p <= i < n, p <= j < i+1} = (n^2 + p^2 - 2np + n - p) / 2."""
    assert orc.count_triangle(p, n) == (n * n + p * p - 2 * n * p + n - p) // 2
    assert (n * n + p * p - 2 * n * p + n - p) % 2 == 0


def _dg_cases():
    rng = np.random.default_rng(123)
    cases = []
    for dtype in ("f32", "f64", "bf16", "fp8"):
        for nunit in (1, 5, 8, 27, 64, 100, 125, 216, 343, 512):
            for _ in range(3):
                nmat = int(rng.choice([1, 2, 3]))
                E = int(rng.choice([1, 15, 17, 129, 300, 1000, 4097]))
                waves = int(rng.choice([1, 2, 3, 4, 6, 8]))
                epw = int(rng.choice([16, 32, 64]))
                per_cu = int(rng.choice([1, 2, 3]))
                P = nmat * ((nunit + 15) // 16)
                ppg = int(rng.choice([1, 2, max(1, P // 3), P]))
                flags = int(rng.choice([0, 2])) if dtype == "fp8" else 0
                cases.append((dtype, nunit, nmat, E, waves, epw, per_cu, ppg, flags))
    # full-size points of the calibration grid
    cases += [("f32", 64, 3, 1 << 21, 4, 16, 3, 12, 0), ("f32", 27, 3, 1 << 20, 4, 64, 2, 6, 0),
              ("f32", 125, 3, 1 << 18, 4, 64, 1, 12, 0), ("bf16", 216, 3, 1 << 16, 4, 32, 1, 21, 8)]
    # the staged low-precision body (rows of a multiple of 8 nodes): one or two
    # row blocks per wave, whole and split row groups, idle waves, ragged ends,
    # up to 16 waves, and its refusals (too few waves to stage a tile, two
    # blocks per wave past nunit 256, d_panels not a multiple of waves)
    for dtype in ("bf16", "fp8"):
        for nunit, nmat, E, waves, epw, per_cu, rb in (
                (8, 3, 1, 1, 16, 4, 2), (8, 3, 4097, 1, 32, 2, 1), (40, 2, 300, 2, 16, 3, 4),
                (40, 2, 300, 3, 16, 3, 3), (64, 3, 1001, 2, 16, 2, 4), (64, 1, 17, 2, 32, 1, 4),
                (64, 3, 129, 6, 16, 2, 6), (216, 3, 5001, 7, 16, 2, 14), (216, 3, 5001, 9, 16, 3, 9),
                (216, 5, 333, 7, 32, 1, 14), (216, 3, 1 << 16, 7, 16, 2, 14), (216, 3, 300, 12, 16, 2, 12),
                (216, 3, 300, 8, 16, 2, 16), (512, 3, 700, 16, 16, 1, 16), (512, 3, 700, 16, 32, 1, 16),
                (256, 8, 200, 8, 16, 2, 8), (216, 3, 300, 4, 16, 2, 8), (216, 3, 300, 2, 16, 2, 4),
                (512, 3, 100, 8, 16, 1, 16), (64, 3, 100, 3, 16, 2, 7), (40, 2, 300, 1, 16, 3, 2)):
            cases.append((dtype, nunit, nmat, E, waves, epw, per_cu, rb, 0))
    # BF16 with the element data rounded in the kernel (FP32 u, 4 bytes a
    # value): staged shapes, and its refusals (two column blocks, the LDS-panel
    # body, rows off a multiple of 8, FP8 input)
    for nunit, nmat, E, waves, epw, per_cu, rb, flags in (
            (8, 3, 4097, 1, 16, 2, 1, 16), (64, 3, 1001, 2, 16, 2, 4, 16), (216, 3, 5001, 7, 16, 2, 14, 16),
            (216, 3, 1 << 16, 7, 16, 2, 14, 16), (512, 3, 700, 16, 16, 1, 16, 16), (216, 3, 300, 12, 16, 2, 12, 16),
            (216, 3, 300, 7, 32, 2, 14, 16), (216, 3, 300, 7, 16, 2, 14, 24), (27, 3, 300, 4, 16, 2, 2, 16)):
        cases.append(("bf16", nunit, nmat, E, waves, epw, per_cu, rb, flags))
    cases.append(("fp8", 216, 3, 300, 7, 16, 2, 14, 16))
    return cases


@pytest.mark.parametrize("case", _dg_cases())
def test_dg_counts_match_brute_force(orc, L, case):
    dtype, nunit, nmat, E, waves, epw, per_cu, ppg, flags = case
    tile = dict(elems_per_wave=epw, waves=waves, groups_per_cu=per_cu, d_panels=ppg, flags=flags)
    try:
        got = L.perf_features_count("dg", dtype, E, nunit, nmat, tile, num_cu=256)
    except L.DGError:
        got = None
    try:
        ref = orc.features("dg", dtype, E, nunit, nmat, epw, waves, per_cu, ppg, flags, 256)
    except ValueError:
        ref = None
    # a shape the library documents as unavailable (element tile of 64 with
    # large rows, operator panels beyond the LDS) is refused by both sides
    assert (got is None) == (ref is None), (got is None, ref is None)
    if got is not None:
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dtype,n", list(itertools.product(["f32"], [4, 8, 100, 1000, 1024, 2048, 4096,
                                                                       16384])) +
                         [("f32", 5), ("f32", 1030), ("f64", 64), ("f64", 257)])
def test_stencil_counts_match_brute_force(orc, L, dtype, n):
    np.testing.assert_array_equal(L.perf_features_count("stencil", dtype, n),
                                  orc.features("stencil", dtype, n))


@pytest.mark.parametrize("n", [1, 7, 16, 100, 128, 130, 512, 1000, 2048])
@pytest.mark.parametrize("num_cu", [0, 7, 256])
def test_matmul_counts_match_brute_force(orc, L, n, num_cu):
    np.testing.assert_array_equal(L.perf_features_count("matmul", "f32", n, num_cu=num_cu),
                                  orc.features("matmul", "f32", n, num_cu=num_cu))


def test_matmul_serial_chain_is_the_busiest_unit():
    """Hand counts: n = 2048 gives 16 x 16 = 256 work-groups of 128 k-chunks,
    one per unit on 256 units; n = 2560 gives 400, two on the busiest unit
    (320 chunks); on 7 units 256 work-groups put 37 on the busiest."""
    from paper_1904_09538_amd import _lib as L
    k = L.feature_names().index("serial_steps")
    assert L.perf_features_count("matmul", "f32", 2048, num_cu=256)[k] == 128
    assert L.perf_features_count("matmul", "f32", 2560, num_cu=256)[k] == 2 * 160
    assert L.perf_features_count("matmul", "f32", 2048, num_cu=7)[k] == 37 * 128
    assert L.perf_features_count("matmul", "f32", 2048)[k] == 128


def test_empty_counts(orc, L):
    for wgs in (1, 16, 4096):
        np.testing.assert_array_equal(L.perf_features_count("empty", "f32", wgs),
                                      orc.features("empty", "f32", wgs))


def test_dg_counts_invariants(L):
    """Counts that the method fixes regardless of the launch shape."""
    # (tile, element rows read by the first operator group): every input once,
    # except that the pipelined loads of a paired-store launch (rows of a
    # multiple of 32 nodes, even panel groups) take whole 16-element
    # wave-tiles, the rows past the end re-reading the last element
    for tile, rows in ((dict(elems_per_wave=16, waves=4, groups_per_cu=3, d_panels=12), 5008),
                       (dict(elems_per_wave=32, waves=2, groups_per_cu=1, d_panels=5), 5000)):
        c = dict(zip(L.feature_names(), L.perf_features_count("dg", "f32", 5000, 64, 3, tile, 256)))
        assert c["gst_dg_out"] == 5000 * 3 * 64 * 4      # every output written once
        assert c["gld_dg_u"] == rows * 64 * 4
        assert c["mfma_f32"] >= 2 * 3 * 64 * 64 * 5000   # at least the algorithmic flops


# ------------------------------------------------------------------ adjoint, quantiser, batched


def _both(orc, L, kernel, dtype, n0, nunit, nmat, tile, num_cu=256, workgroups=0):
    """(library closed form, oracle walk); None where a side refuses the descriptor."""
    try:
        got = L.perf_features_count(kernel, dtype, n0, nunit, nmat, tile, num_cu, workgroups)
    except L.DGError:
        got = None
    try:
        ref = orc.features(kernel, dtype, n0, nunit, nmat, tile.get("elems_per_wave", 0), tile.get("waves", 0),
                           tile.get("groups_per_cu", 0), tile.get("d_panels", 0), tile.get("flags", 0), num_cu,
                           workgroups)
    except ValueError:
        ref = None
    return got, ref


def _bwd_u_cases():
    cases = []
    # the GEMM body: FP32 rows of 97 nodes or more, ragged element tiles and XCD groups
    for n in (97, 125, 128, 129, 216, 343, 512):
        for E in (1, 127, 128, 129, 1000, 128 * 9 + 5):
            for M in (1, 3):
                cases.append(("f32", n, M, E, dict(elems_per_wave=128, waves=4, groups_per_cu=2, flags=4)))
    # the contraction body: one launch with nmat segments, or one per operator
    rng = np.random.default_rng(5)
    for dtype in ("f32", "f64"):
        for n in (1, 5, 8, 27, 64, 96, 125, 216, 343, 512):
            if dtype == "f32" and n >= 97:
                continue
            for M in (1, 2, 3, 4):
                E = int(rng.choice([1, 17, 300, 4097]))
                per_cu = int(rng.choice([1, 2, 3]))
                ppg = int(rng.choice([1, 2, (n + 15) // 16]))
                cases.append((dtype, n, M, E, dict(elems_per_wave=16, waves=4, groups_per_cu=per_cu,
                                                   d_panels=ppg)))
    return cases


@pytest.mark.parametrize("case", _bwd_u_cases())
def test_bwd_u_counts_match_brute_force(orc, L, case):
    dtype, n, M, E, tile = case
    got, ref = _both(orc, L, "bwd_u", dtype, E, n, M, tile)
    assert (got is None) == (ref is None), (got is None, ref is None)
    if got is not None:
        np.testing.assert_array_equal(got, ref)


# shapes whose brute-force walk stays within the CPU suite's time (n^2 M E
# <= 2e9; the larger ones are covered by the same code paths at smaller E)
_BWD_D_CASES = [(dtype, n, M, E, per_cu) for dtype in ("f32", "f64")
                for n, M in ((1, 1), (8, 3), (27, 3), (64, 2), (125, 3), (129, 1), (216, 3), (512, 1))
                for E in (0, 1, 16, 255, 256, 4097, 70001) for per_cu in (1, 2, 4)
                if n * n * M * E <= 2e9]


@pytest.mark.parametrize("dtype,n,M,E,per_cu", _BWD_D_CASES)
def test_bwd_d_counts_match_brute_force(orc, L, dtype, n, M, E, per_cu):
    got, ref = _both(orc, L, "bwd_d", dtype, E, n, M, dict(groups_per_cu=per_cu))
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("to", ["bf16", "fp8"])
@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 5), (1000, 27), (4097, 64), (513, 125), (100, 216),
                                       (70, 257), (9, 512), (33, 513), (5, 1024), (3, 1025), (2, 3001),
                                       (1 << 18, 8), (300000, 4)])
@pytest.mark.parametrize("per_row", [0, 1])
def test_quant_counts_match_brute_force(orc, L, to, rows, cols, per_row):
    got, ref = _both(orc, L, "quant", to, rows, cols, per_row, {})
    np.testing.assert_array_equal(got, ref)


def _batched_cases():
    cases = []
    # one element per thread (order 1)
    for cnt in (1, 63, 64, 65, 256, 1000, 100003):
        for G in (8, 16, 64, 512):
            cases.append((cnt, 8, dict(elems_per_wave=256, waves=4), G))
    # resident panels: every order, column blocks, panel groups, shares
    rng = np.random.default_rng(11)
    for p in (1, 2, 3, 4, 5):
        n = (p + 1) ** 3
        panels = 3 * ((n + 15) // 16)
        for cb in (1, 2):
            for _ in range(4):
                ppg = int(rng.choice([1, 2, max(1, panels // 3), panels]))
                ng = -(-panels // ppg)
                G = 8 * ng * int(rng.choice([1, 2, 5]))
                cnt = int(rng.choice([1, 15, 64, 129, 3000]))
                cases.append((cnt, n, dict(elems_per_wave=16 * cb, waves=4, groups_per_cu=2, d_panels=ppg), G))
    # GEMM tiles (orders 6, 7 and forced lower orders)
    for p in (3, 5, 6, 7):
        for cnt in (1, 127, 128, 129, 1031, 2500):
            cases.append((cnt, (p + 1) ** 3, dict(elems_per_wave=128, waves=4, groups_per_cu=1, d_panels=8,
                                                  flags=4), 16))
    return cases


@pytest.mark.parametrize("case", _batched_cases())
def test_batched_counts_match_brute_force(orc, L, case):
    cnt, n, tile, G = case
    got, ref = _both(orc, L, "batched", "f32", cnt, n, 3, tile, 256, G)
    assert (got is None) == (ref is None), (got is None, ref is None)
    if got is not None:
        np.testing.assert_array_equal(got, ref)


def test_batched_pool_and_refusals(orc, L):
    for G in (1, 8, 777):
        np.testing.assert_array_equal(L.perf_features_count("batched_pool", "f32", G),
                                      orc.features("batched_pool", "f32", G))
    # a share that is not a whole number of streams per operator group, and
    # one element per thread for a row of 27 nodes, are refused by both sides
    for tile, n, G in ((dict(elems_per_wave=16, waves=4, groups_per_cu=2, d_panels=1), 64, 8),
                       (dict(elems_per_wave=256, waves=4), 27, 8)):
        got, ref = _both(orc, L, "batched", "f32", 100, n, 3, tile, 256, G)
        assert got is None and ref is None


def test_adjoint_quant_batched_invariants(L):
    """What the method fixes whatever the schedule: every output value
    written once, every input row read (at least) once, at least the
    algorithmic matrix flops."""
    names = L.feature_names()
    E, n, M = 3001, 125, 3
    cu = dict(zip(names, L.perf_features_count("bwd_u", "f32", E, n, M,
                                               dict(elems_per_wave=128, waves=4, groups_per_cu=2, flags=4),
                                               256)))
    assert cu["gst_dg_out"] + cu["gst_dg_out_unal"] == E * n * 4
    assert cu["gld_dg_u"] + cu["gld_dg_u_unal"] == M * E * n * 4
    assert cu["mfma_f32"] >= 2 * M * n * n * E
    cd = dict(zip(names, L.perf_features_count("bwd_d", "f32", E, n, M, dict(groups_per_cu=2), 256)))
    assert cd["gst_dg_out_unal"] == M * n * n * 4
    assert cd["mfma_f32"] >= 2 * M * n * n * E
    assert cd["gld_ws"] == cd["gst_ws"]      # every partial written is read back once
    for to, esz in (("bf16", 2), ("fp8", 1)):
        q = dict(zip(names, L.perf_features_count("quant", to, 1 << 16, 216, 1)))
        assert q["gst_dg_out"] == (1 << 16) * 216 * esz and q["gld_dg_u"] == (1 << 16) * 216 * 4
    for cnt, n, tile, G in ((1000, 8, dict(elems_per_wave=256, waves=4), 64),
                            (1000, 64, dict(elems_per_wave=16, waves=4, groups_per_cu=2, d_panels=12), 8),
                            (1000, 343, dict(elems_per_wave=128, waves=4, flags=4), 8)):
        b = dict(zip(names, L.perf_features_count("batched", "f32", cnt, n, 3, tile, 256, G)))
        assert b["gst_dg_out_unal"] == 3 * cnt * n * 4
        assert b["gld_dg_u_unal"] == cnt * n * 4
        assert b["mfma_f32"] + b["valu_f32"] >= 2 * 3 * n * n * cnt


# ------------------------------------------------------------------ measurement kernels

def _ub_cases():
    cases = [("stream", 1, 1, 0), ("stream", 1000, 3, 0), ("stream", 8192 * 256 + 5, 2, 0),
             ("stream", 3 * 8192 * 256, 4, 0), ("strided", 1, 1, 0), ("strided", 1000, 33, 0),
             ("fma", 3, 0, 0), ("fma", 2, 7, 0), ("mfma", 2, 5, 0), ("lds", 3, 0, 1), ("lds", 2, 9, 4),
             ("barrier", 5, 17, 0), ("overlap", 1, 3, 0), ("overlap", 257, 0, 0), ("overlap", 1000, 12, 0),
             ("twin_stencil", 1024, 1088, 1024), ("twin_stencil", 4100, 4160, 4100),
             ("twin_matmul", 1000, 0, 0), ("twin_matmul", 1024, 0, 0),
             ("tile_read", 16, 0, 0), ("tile_read", 96, 0, 0), ("tile_read", 96, 1, 0), ("tile_read", 160, 1, 0)]
    return cases


def test_tile_read_refusals(orc, L):
    """n not a multiple of 16, or a pattern other than a (0) or b (1): both
    sides refuse."""
    for n, a in ((100, 0), (64, 2)):
        with pytest.raises(L.DGError):
            L.perf_ubench_count("tile_read", n, a)
        with pytest.raises(ValueError):
            orc.ubench_features("tile_read", n, a)


@pytest.mark.parametrize("case", _ub_cases())
def test_ubench_counts_match_brute_force(orc, L, case):
    kind, n, a, b = case
    for dtype in (("f32", "bf16") if kind == "mfma" else ("f32",)):
        np.testing.assert_array_equal(L.perf_ubench_count(kind, n, a, b, dtype, num_cu=256),
                                      orc.ubench_features(kind, n, a, b, dtype, num_cu=256))


@pytest.mark.parametrize("nunit,E,tile", [
    (27, 100003, dict(elems_per_wave=32, waves=8, groups_per_cu=3, d_panels=6)),
    (64, 1 << 18, dict(elems_per_wave=16, waves=8, groups_per_cu=2, d_panels=12)),
    (64, 5001, dict(elems_per_wave=32, waves=4, groups_per_cu=3, d_panels=12)),
    (125, 70000, dict(elems_per_wave=32, waves=8, groups_per_cu=1, d_panels=12)),
    (216, 4097, dict(elems_per_wave=16, waves=8, groups_per_cu=1, d_panels=11)),
    (8, 999, dict(elems_per_wave=16, waves=4, groups_per_cu=4, d_panels=3))])
def test_dg_twin_counts(orc, L, nunit, E, tile):
    """The DG twin: the forward's global accesses and schedule exactly (walk
    == closed form), no on-chip work, one add per loaded value."""
    got = L.perf_ubench_count("twin_dg", E, nunit, 3, tile=tile, num_cu=256)
    ref = orc.ubench_features("twin_dg", E, nunit, 3, tile=tile, num_cu=256)
    np.testing.assert_array_equal(got, ref)
    fwd = dict(zip(L.feature_names(), L.perf_features_count("dg", "f32", E, nunit, 3, tile, 256)))
    tw = dict(zip(L.feature_names(), got))
    for k in fwd:
        if k.startswith("gld_") or k.startswith("gst_") or k in ("workgroups", "launch", "wave_tiles",
                                                                   "serial_steps"):
            assert tw[k] == fwd[k], k
    assert tw["lds_bytes"] == tw["mfma_f32"] == tw["barrier_x_wg"] == 0
    assert tw["valu_f32"] * 4 == sum(v for k, v in tw.items() if k.startswith("gld_"))


# ------------------------------------------------------------------ model fit


def test_fit_matches_oracle(L):
    from oracle import model as M
    rng = np.random.default_rng(7)
    F = rng.uniform(1, 10, size=(60, 8)) * np.logspace(-3, 9, 8)
    t = F @ rng.uniform(0.5, 2, 8) * np.logspace(-12, -6, 8)[None, :].sum() * rng.uniform(0.95, 1.05, 60)
    for rel in (True, False):
        a = L.perf_model_fit(F, t, relative=rel)
        b = M.fit(F, t, relative=rel)
        np.testing.assert_allclose(a["p"], b["p"], rtol=1e-9)
        assert a["rank"] == b["rank"] == 8
        assert abs(a["resid"] - b["resid"]) <= 1e-9 * max(1.0, b["resid"])
        np.testing.assert_allclose(L.perf_model_predict(F, a["p"]), M.predict(F, b["p"]), rtol=1e-12)


def test_fit_rank_deficient_and_errors(L):
    from oracle import model as M
    rng = np.random.default_rng(8)
    a = rng.uniform(1, 2, 30)
    F = np.stack([a, a, rng.uniform(1, 2, 30), np.zeros(30)], axis=1)
    t = F @ np.array([1.0, 3.0, 2.0, 0.0]) + 0.0
    got = L.perf_model_fit(F, t, relative=False)
    ref = M.fit(F, t, relative=False)
    assert got["rank"] == ref["rank"] == 2
    np.testing.assert_allclose(got["p"], ref["p"], rtol=1e-9, atol=1e-12)
    with pytest.raises(L.DGError):
        L.perf_model_fit(F, -t, relative=True)
    with pytest.raises(L.DGError):
        L.perf_model_fit(np.full((2, 2), np.nan), np.ones(2))


def test_overlap_fit_matches_oracle(L):
    """The library's Levenberg-Marquardt fit of the overlap model reaches the
    same minimiser as the oracle's library least-squares routine."""
    from oracle import model as M
    rng = np.random.default_rng(12)
    F = np.column_stack([np.ones(50), rng.integers(16, 4096, 50), rng.uniform(1e8, 1e10, 50),
                         rng.uniform(1e8, 1e10, 50), rng.uniform(1e11, 1e13, 50)])
    group = [0, 0, 1, 1, 2]
    p_true = np.array([5e-6, 2e-9, 2e-13, 1.5e-13, 7e-15])
    t = M.overlap_predict(F, group, p_true, 3e4) * rng.uniform(0.97, 1.03, 50)
    p0 = p_true * rng.uniform(0.7, 1.4, 5)
    a = L.perf_model_fit_overlap(F, t, group, p0=p0, edge0=2e4)
    b = M.overlap_fit(F, t, group, p0, 2e4)
    pa = L.perf_model_predict_overlap(F, group, a["p"], a["edge"])
    pb = M.overlap_predict(F, group, b["p"], b["edge"])
    assert abs(a["resid"] - b["resid"]) <= 1e-6 * b["resid"] + 1e-12
    np.testing.assert_allclose(pa, pb, rtol=1e-5)
    np.testing.assert_allclose(L.perf_model_predict_overlap(F, group, a["p"], a["edge"]),
                               M.overlap_predict(F, group, a["p"], a["edge"]), rtol=1e-12)


def _neg_linear_case(seed):
    """A law whose last feature nearly duplicates another and enters with a
    negative weight: the unconstrained fit goes below zero there."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(1.0, 10.0, size=(40, 5)) * np.array([1.0, 1e3, 1e6, 1e9, 1e6])
    F[:, 4] = 0.9 * F[:, 2] + rng.uniform(0, 3e5, 40)
    t = F[:, :4] @ np.array([5e-6, 1e-9, 2e-12, 3e-15]) - 5e-13 * F[:, 4]
    return F, t * rng.uniform(0.97, 1.03, 40)


@pytest.mark.parametrize("seed", [5, 6, 7, 10])
@pytest.mark.parametrize("rel", [True, False])
def test_nonneg_fit_matches_oracle(L, seed, rel):
    """Lawson-Hanson NNLS in the library against the oracle's library NNLS,
    on systems whose unconstrained fit has a negative weight."""
    from oracle import model as M
    F, t = _neg_linear_case(seed)
    assert M.fit(F, t, relative=rel)["negative"]
    a = L.perf_model_fit(F, t, relative=rel, nonneg=True)
    b = M.fit(F, t, relative=rel, nonneg=True)
    assert np.all(a["p"] >= 0) and not a["negative"]
    np.testing.assert_allclose(a["p"], b["p"], rtol=1e-8, atol=1e-12 * np.max(np.abs(b["p"])))
    assert abs(a["resid"] - b["resid"]) <= 1e-9 * max(1.0, b["resid"])
    # unconstrained entry point unchanged by the flag's existence
    np.testing.assert_allclose(L.perf_model_fit(F, t, relative=rel)["p"],
                               M.fit(F, t, relative=rel)["p"], rtol=1e-9)
    with pytest.raises(L.DGError):           # unknown flag bit
        f1 = np.ones(1)
        dp = ctypes.POINTER(ctypes.c_double)
        L.check(L.lib().perf_model_fit(1, 1, f1.ctypes.data_as(dp), f1.ctypes.data_as(dp), 8,
                                       np.zeros(1).ctypes.data_as(dp), None, None, None))


def test_overlap_fit_nonneg_matches_oracle(L):
    """Projected LM against the oracle's bounded trust-region fit when the
    data pull one cost parameter below zero: both stay in the orthant and
    reach the same residual."""
    from oracle import model as M
    rng = np.random.default_rng(14)
    F = np.column_stack([np.ones(50), rng.integers(16, 4096, 50), rng.uniform(1e8, 1e10, 50),
                         rng.uniform(1e8, 1e10, 50), rng.uniform(1e10, 1e12, 50)])
    group = [0, 0, 1, 1, 2]
    p_true = np.array([5e-6, 0.0, 2e-13, 1.5e-13, 7e-15])
    t = M.overlap_predict(F, group, p_true, 1e3) - 3e-10 * F[:, 1]
    t = np.abs(t * rng.uniform(0.97, 1.03, 50))
    p0 = np.array([5e-6, 1e-9, 2e-13, 1.5e-13, 7e-15]) * rng.uniform(0.7, 1.4, 5)
    un = L.perf_model_fit_overlap(F, t, group, p0=p0, edge0=2e3)
    assert np.any(un["p"] < 0)
    a = L.perf_model_fit_overlap(F, t, group, p0=p0, edge0=2e3, nonneg=True)
    b = M.overlap_fit(F, t, group, p0, 2e3, nonneg=True)
    assert np.all(a["p"] >= 0) and np.all(b["p"] >= 0)
    assert abs(a["resid"] - b["resid"]) <= 1e-8 * b["resid"]
    np.testing.assert_allclose(L.perf_model_predict_overlap(F, group, a["p"], a["edge"]),
                               M.overlap_predict(F, group, b["p"], b["edge"]), rtol=1e-6)
