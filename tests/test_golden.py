"""Golden values the paper prints for its matrix-multiplication example
(tests/golden/matmul_prefetch_counts.txt, citations in the file): the
prefetching 16 x 16 variant performs 2 n^3 local loads and 2 n^3 / 16 local
stores that the non-prefetching variant does not, 16 times fewer global loads
(2 n^3 / 16 against 2 n^3), and n^3 multiply-adds.  Checked against the
oracle's brute-force walk of the variants' schedules and the library's closed
form (which must equal the walk).  Counts there are bytes of the lanes that
issue them (4 per value), a multiply-add being 2 flops; the tiled variant's
LDS feature holds its loads and stores together."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "matmul_prefetch_counts.txt")


def _golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


@pytest.mark.parametrize("n", [16, 48, 128, 1024])
def test_matmul_variant_counts_are_the_papers(orc, L, n):
    g = _golden()
    n3 = n ** 3
    names = orc.VARIANT_FEATURES
    pf = dict(zip(names, orc.variant_features("mm_pf", n, 0, 0, False, 0)))
    nopf = dict(zip(names, orc.variant_features("mm_nopf", n, 0, 0, False, 0)))
    # the library's closed form is the walk
    assert np.array_equal(L.perf_variant_count("mm_pf", n), [pf[k] for k in names])
    assert np.array_equal(L.perf_variant_count("mm_nopf", n), [nopf[k] for k in names])
    # local memory: loads and stores of the prefetching variant, none without
    assert pf["lds_sg"] == 4 * (g["lmem_loads_prefetch"] + g["lmem_stores_prefetch"]) * n3
    assert nopf["lds_sg"] == 0
    # global loads: 2 n^3 / 16 against 2 n^3, a factor of 16
    assert pf["gld_mm_pf_a"] + pf["gld_mm_pf_b"] == 4 * g["gmem_loads_prefetch"] * n3
    assert nopf["gld_mm_nopf_a"] + nopf["gld_mm_nopf_b"] == 4 * g["gmem_loads_noprefetch"] * n3
    # multiply-adds, 2 flops each, the same in both
    assert pf["valu_f32_sg"] == nopf["valu_f32_sg"] == 2 * g["madd"] * n3
    # one store of c per element
    assert pf["gst_mm_c"] == nopf["gst_mm_c"] == 4 * n * n


def _stencil_golden():
    path = os.path.join(os.path.dirname(GOLDEN), "stencil_workgroup_counts.txt")
    rows = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                v, *nums = line.split()
                rows[v] = dict(zip(("threads", "computing", "idle", "stride"), map(int, nums)))
    return rows


@pytest.mark.parametrize("kind", ["fd16", "fd18"])
def test_stencil_variant_work_groups_are_the_papers(orc, L, kind):
    from oracle import variants as OV
    g = _stencil_golden()[kind]
    assert g["computing"] + g["idle"] == g["threads"]
    # one work-group over exactly one stride of interior points: every
    # work-item fetches once, the computing ones store once
    n = g["stride"]
    gx, gy, T = OV.shape(kind, n)
    assert (gx, gy, T) == (1, 1, g["threads"])
    f = dict(zip(orc.VARIANT_FEATURES, orc.variant_features(kind, n, 0, 0, False, 0)))
    assert f["workgroups"] == 1
    assert f[f"gld_{kind}_u"] == 4 * g["threads"]
    assert f[f"gst_{kind}_res"] == 4 * g["computing"]
    # larger grids: work-groups start `stride` points apart in both directions
    for m in (3 * n, 3 * n + 1):
        gx, gy, _ = OV.shape(kind, m)
        assert gx == gy == -(-m // g["stride"])
        f = dict(zip(orc.VARIANT_FEATURES, orc.variant_features(kind, m, 0, 0, False, 0)))
        assert f["workgroups"] == gx * gy
        assert np.array_equal(L.perf_variant_count(kind, m, ld_u=m + 2, ld_res=m),
                              orc.variant_features(kind, m, 0, 0, False, 0))


def test_dg_variant_configuration_is_the_papers(orc, L):
    from oracle import variants as OV
    from paper_1904_09538_amd import variant_study as V
    g = {}
    with open(os.path.join(os.path.dirname(GOLDEN), "dg_variant_config.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                g[k] = int(v)
    assert (V.NUNIT, V.NMAT) == (g["nunit_nodes"], g["nmatrices"])
    for kind in ("dg_nopf", "dg_pfu", "dg_pfdm", "dg_pfdmt"):
        E = 5 * g["tile"] + 3
        gx, gy, T = OV.shape(kind, E, g["nunit_nodes"])
        assert T == g["workgroup"] == g["tile"] ** 2
        assert (gx, gy) == (-(-E // g["tile"]), g["nunit_nodes"] // g["tile"])
        f = dict(zip(orc.VARIANT_FEATURES, orc.variant_features(kind, E, g["nunit_nodes"], g["nmatrices"],
                                                                False, 0)))
        assert f["workgroups"] == gx * gy
        # every variant does the same 2 nmat nunit^2 flops per element slot of its grid
        assert f["valu_f32_sg"] == 2 * g["nmatrices"] * g["nunit_nodes"] ** 2 * g["tile"] * gx
