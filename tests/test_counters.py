"""The counted features against hardware counters (CPU only: reads the
rocprofv3 --pmc counters committed in profiles/counters.json, taken on an
MI355X with paper_1904_09538_amd/counter_set.py).

This pins the oracle's brute-force walks (oracle/features_bf.c), and the
library's closed forms that must equal them, to what the GPU executed rather
than to a second reading of the same schedule:
  - matrix-core flops (MOPS x 512) equal the counted flops exactly;
  - LDS bytes ((LOAD + STORE bandwidth) x 64) equal the counted bytes exactly
    once the instructions that move under 64 bytes are set aside (the counter
    adds floor(active lanes x size / 64) per instruction): the batched pool's
    one-lane 8-byte claim store, the low-precision kernels' 8-lane operator
    scale staging, and the ragged last wave-tile of the slab path;
  - SQ_WAVES equals the waves of the counted work-groups;
  - HBM bytes written (WRITE_SIZE) equal the counted stores for rows of
    whole 16-byte vectors, and are never below them;
  - HBM bytes read (FETCH_SIZE x 2, the factor a plain copy reads at) match
    the counted loads of the streaming kernels.
Barriers have no counter on gfx950 and are not pinned here.
"""
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "profiles", "counters.json")


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


@pytest.fixture(scope="module")
def variants():
    with open(DATA) as fh:
        return {v["id"]: v for v in json.load(fh)["variants"]}


def _walk(orc, kind, dtype, n0, nunit=0, nmat=0, tile=None, num_cu=0, workgroups=0):
    t = tile or {}
    return orc.features(kind, dtype, n0, nunit, nmat, t.get("elems_per_wave", 0), t.get("waves", 0),
                        t.get("groups_per_cu", 0), t.get("d_panels", 0), t.get("flags", 0), num_cu, workgroups)


def counted(orc, L, v):
    """(library closed form, oracle walk) of one variant's call, int64 arrays."""
    k, p = v["kind"], v["params"]
    if k == "dg":
        args = ("dg", p["dtype"], p["E"], v["nunit"], p.get("nmat", 3), v["tile"], v["num_cu"])
        return L.perf_features_count(*args), _walk(orc, *args)
    if k == "stencil":
        return L.perf_features_count("stencil", "f32", p["n"]), _walk(orc, "stencil", "f32", p["n"])
    if k == "matmul":
        return (L.perf_features_count("matmul", "f32", p["n"], num_cu=v["num_cu"]),
                _walk(orc, "matmul", "f32", p["n"], num_cu=v["num_cu"]))
    if k == "empty":
        return L.perf_features_count("empty", "f32", p["wgs"]), _walk(orc, "empty", "f32", p["wgs"])
    if k == "quant":
        return (L.perf_features_count("quant", p["to"], p["rows"], p["cols"], 1),
                _walk(orc, "quant", p["to"], p["rows"], p["cols"], 1))
    if k == "adjoint":
        tu, td = v["tiles_bwd"]
        n = v["nunit"]
        lib = (L.perf_features_count("bwd_d", "f32", p["E"], n, 3, td, v["num_cu"]) +
               L.perf_features_count("bwd_u", "f32", p["E"], n, 3, tu, v["num_cu"]))
        orc_ = (_walk(orc, "bwd_d", "f32", p["E"], n, 3, td, v["num_cu"]) +
                _walk(orc, "bwd_u", "f32", p["E"], n, 3, tu, v["num_cu"]))
        return lib, orc_
    if k == "batched":
        plan = {int(q): i for q, i in v["plan"].items()}
        lib = L.batched_counts(plan, v["num_cu"])
        orc_ = None
        grid = 0
        chain = [L.feature_names().index(k) for k in L.CHAIN_FEATURES]
        for q, i in plan.items():
            if i["count"] == 0:
                continue
            grid += i["workgroups"]
            w = _walk(orc, "batched", "f32", i["count"], (q + 1) ** 3, 3, i["tile"], v["num_cu"], i["workgroups"])
            if orc_ is None:
                orc_ = w
            else:
                # orders side by side: work adds, the longest chain sets the launch's
                longest = np.maximum(orc_[chain], w[chain])
                orc_ = orc_ + w
                orc_[chain] = longest
        if any(i["tile"]["flags"] & 4 for i in plan.values() if i["count"]):
            orc_ = orc_ + _walk(orc, "batched_pool", "f32", grid)
        orc_[0] = 1
        return lib, orc_
    return None, None


IDS = ["dg_f32_p2_2e21", "dg_f32_p3_2e21", "dg_f32_p4_2e21", "dg_f32_p5_2e21", "dg_f32_p3_2e18_epw32_w4",
       "dg_f32_p4_2e18_panels8", "dg_f32_p2_100003", "dg_f64_p3_4096", "dg_bf16_p5_2e20", "dg_fp8_p5_2e20",
       "dg_bf16_p5_2e20_ldspanels", "dg_fp8_p5_2e20_ldspanels", "dg_bf16_p5_100003_split",
       "dg_fp8native_p5_2e20", "dg_bf16_p5_2e20_nmat1", "dg_bf16_p5_2e20_nmat2", "dg_fp8_p5_2e20_nmat1",
       "dg_fp8_p5_2e20_nmat2", "dg_bf16_p5_2e20_grid8", "dg_bf16_p5_2e20_grid24", "quant_fp8_rows_2e20x216", "quant_bf16_2e20x216", "batched_p1_7_2e20",
       "adjoint_p4_2e19", "stencil_16384", "stencil_1030", "matmul_8192", "matmul_1000", "empty_1024"]


def _names(L):
    return L.feature_names()


def _staged(v):
    """The low-precision call ran the staged body (rows of a multiple of 8
    nodes, neither the LDS-panel nor the native FP8 flag)."""
    return v["nunit"] % 8 == 0 and not v["tile"]["flags"] & (2 | 8)


def _lds_under_64(v, f):
    """Counted LDS bytes moved by instructions of under 64 bytes, which the
    counter does not see (see the module docstring); None for the ragged
    slab case, bounded separately."""
    if v["kind"] == "batched":
        plan = {int(q): i for q, i in v["plan"].items()}
        claims = 0
        grid = sum(i["workgroups"] for i in plan.values() if i["count"])
        for q, i in plan.items():
            if i["count"] and i["tile"]["flags"] & 4:
                n = (q + 1) ** 3
                claims += -(-3 * n // 128) * -(-i["count"] // 128)   # one claim per GEMM tile
        claims += 8 * grid                                            # each pool found drained
        return 8 * claims
    if v["kind"] == "dg" and v["params"]["dtype"] in ("bf16", "fp8") and not _staged(v):
        return 32 * f["workgroups"]
    if v["id"] in ("dg_f32_p2_100003", "dg_bf16_p5_100003_split"):
        return None
    return 0


@pytest.mark.parametrize("vid", IDS)
def test_walk_and_closed_form_match_counters(orc, L, variants, vid):
    v = variants[vid]
    lib, walk = counted(orc, L, v)
    np.testing.assert_array_equal(lib, walk)       # the walk reproduces the closed form ...
    f = dict(zip(_names(L), (int(x) for x in walk)))
    c = v["counters_per_call"]
    # ... and both reproduce the hardware's matrix-core work exactly
    mops = sum(c.get(k, 0.0) for k in ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64",
                                       "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F8"))
    assert mops * 512 == f["mfma_f32"] + f["mfma_f64"] + f["mfma_bf16"] + f["mfma_fp8"]
    assert c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0) * 512 == f["mfma_f64"]
    assert c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0) * 512 == f["mfma_bf16"]
    assert c.get("SQ_INSTS_VALU_MFMA_MOPS_F8", 0) * 512 == f["mfma_fp8"]
    # LDS bytes
    lds = (c.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0) + c.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0)) * 64
    small = _lds_under_64(v, f)
    if small is None and v["id"] == "dg_f32_p2_100003":
        # the slab path's last wave-tile holds 3 elements (100003 = 3125 x 32 + 3):
        # its scalar LDS accesses of 3 elements' lanes are under 64 bytes each
        gap = f["lds_bytes"] - lds
        assert 0 < gap <= 2 * 3 * 27 * 4 + 3 * 3 * 27 * 4 * 4, gap
    elif small is None:
        # staged body with split row groups (144- and 72-row result rows in
        # LDS): the LDS instruction count agrees exactly (SQ_INSTS_LDS), the
        # bytes fall short of the counted ones by 64 per work-group tile, a
        # counter effect not isolated further (0.07 % here)
        gap = f["lds_bytes"] - lds
        assert gap == 64 * f["wave_tiles"], (gap, f["wave_tiles"])
    else:
        assert lds == f["lds_bytes"] - small, (lds, f["lds_bytes"], small)
    if v["id"] == "dg_bf16_p5_100003_split":
        # LDS instructions per work-group tile: 2 result-row reads and a
        # chunk copy plus a scale per wave; per wave holding a row block 7 B
        # fragment reads, a scale read and a result write; per work-group
        # one more copy (tiles + 1) and the padding rows' zero fill
        n_tiles, groups, wgs = 6251, 6, f["workgroups"]
        active = (9 + 5) * 3          # waves holding a block: 9 in a slab's first 144 rows, 5 in its last 72
        per_group_tile = 9 * 2 + 9 * 2
        assert c["SQ_INSTS_LDS"] == (per_group_tile * groups + active * 9) * n_tiles + wgs * (18 + 1)
    # waves (work-groups of the staged body without tiles exit at once, and
    # are counted as launched)
    waves_per_wg = v["tile"]["waves"] if v["kind"] == "dg" else 4
    assert c["SQ_WAVES"] == f["workgroups"] * waves_per_wg


@pytest.mark.parametrize("vid", IDS)
def test_hbm_bytes_against_counted(L, orc, variants, vid):
    v = variants[vid]
    _, walk = counted(orc, L, v)
    f = dict(zip(_names(L), (int(x) for x in walk)))
    c = v["counters_per_call"]
    copy = variants["copy_1GiB"]["counters_per_call"]
    # the scale at which the counters read a plain copy of 1 GiB
    fscale = (1 << 30) / (copy["FETCH_SIZE"] * 1024)
    wscale = (1 << 30) / (copy["WRITE_SIZE"] * 1024)
    assert abs(fscale - 2.0) < 0.01 and abs(wscale - 1.0) < 0.01
    written = c.get("WRITE_SIZE", 0) * 1024 * wscale
    stored = sum(x for k, x in f.items() if k.startswith("gst_"))
    read = c.get("FETCH_SIZE", 0) * 1024 * fscale
    loaded = sum(x for k, x in f.items() if k.startswith("gld_") and not k.endswith("_l2"))
    if stored:
        assert written >= 0.999 * stored
    if vid in ("dg_f32_p2_2e21", "dg_f32_p3_2e21", "dg_f32_p3_2e18_epw32_w4", "dg_f64_p3_4096",
               "stencil_16384", "matmul_8192", "matmul_1000"):
        # whole 16-byte row vectors: every counted store byte, no more
        assert abs(written / stored - 1) < 1e-3, written / stored
    if vid in ("stencil_16384", "quant_fp8_rows_2e20x216", "quant_bf16_2e20x216", "dg_f32_p2_2e21",
               "dg_f32_p3_2e21"):
        # streaming kernels: each input read once from memory
        assert abs(read / loaded - 1) < 0.05, read / loaded
    if v["kind"] == "dg" and v["params"]["dtype"] in ("bf16", "fp8") and _staged(v):
        # the staged body writes whole output rows: every counted store byte
        assert abs(written / stored - 1) < 1e-3, written / stored
    if vid in ("dg_bf16_p5_2e20_nmat1", "dg_fp8_p5_2e20_nmat1", "dg_bf16_p5_2e20_grid24"):
        # one reader per element tile (one operator), or the readers of a
        # tile close together (work-groups of ~32 tiles): the element data
        # come from memory once; the fetch adds the operator rows and element
        # scales (L2-resident, a few MB)
        assert 0.95 <= read / f["gld_dg_u"] <= 1.10, read / f["gld_dg_u"]
