"""GPU parity of dgdiff_apply (FP32 / FP64) against the FP64 oracle.

Tolerances (normwise max relative error): 1e-12 for FP64, 1e-5 for FP32.
Inputs come from the seeded generators; FP32 runs feed the oracle the
FP32-rounded values widened to FP64, so the error measures the kernel.
"""
import numpy as np
import pytest
import torch

from paper_1904_09538_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def ops():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda:0", dtype=dtype)


def _run(ops, D, u, dtype, tile=None):
    out = ops.dgdiff_apply(_dev(D, dtype), _dev(u, dtype), tile=tile)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def _as(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x


def _epw64_unavailable(dtype, nunit):
    """The documented limit of an element tile of 64 per wave: nunit <= 128 in
    FP32, nunit <= 64 in FP64 (the wave's element fragments in registers)."""
    return nunit > (128 if dtype == torch.float32 else 64)


def _check_or_refused(orc, ops, D, u, dtype, tile):
    """Shapes the header documents as unavailable raise DGError; every other
    shape runs and matches the oracle."""
    if tile and tile.get("elems_per_wave") == 64 and _epw64_unavailable(dtype, u.shape[1]):
        with pytest.raises(ops.DGError):
            _run(ops, _as(D, dtype), _as(u, dtype), dtype, tile)
        return
    _check(orc, ops, D, u, dtype, tile=tile)


def _check(orc, ops, D, u, dtype, tile=None):
    D, u = _as(D, dtype), _as(u, dtype)
    got = _run(ops, D, u, dtype, tile)
    ref = orc.dg_forward(D, u)
    from oracle.metrics import normwise_rel
    err = normwise_rel(got, ref)
    assert err <= TOL[dtype], f"normwise error {err:.3e}"
    return err


@pytest.mark.parametrize("dkind", ["gll", "random"])
def test_fp64_hex_p3_4096_elements(orc, ops, dkind):
    D = I.gll_dmats(3) if dkind == "gll" else I.random_dmats(64)
    u = I.uniform_u(4096, 64)
    _check(orc, ops, D, u, torch.float64)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("nunit", [1, 5, 8, 17, 27, 64, 100, 125, 216, 343, 512])
def test_sweep_nunit_ragged(orc, ops, dtype, nunit):
    for nmat, nelem in ((3, 300), (1, 33), (2, 1)):
        D = I.random_dmats(nunit, nmat=nmat)
        u = I.uniform_u(nelem, nunit)
        _check(orc, ops, D, u, dtype)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_gll_operators_fp32(orc, ops, p):
    D = I.gll_dmats(p)
    u = I.uniform_u(1000, (p + 1) ** 3)
    _check(orc, ops, D, u, torch.float32)


@pytest.mark.parametrize("nunit", [64, 216])
@pytest.mark.parametrize("tile", [dict(elems_per_wave=16), dict(elems_per_wave=32),
                                  dict(waves=1), dict(waves=2, elems_per_wave=16),
                                  dict(d_panels=1), dict(d_panels=3, waves=3),
                                  dict(groups_per_cu=1), dict(elems_per_wave=64, flags=1),
                                  dict(flags=1)])
def test_tile_variants(orc, ops, nunit, tile):
    if tile.get("elems_per_wave") == 64 and nunit > 128:
        with pytest.raises(ops.DGError):
            ops.dgdiff_apply(_dev(I.random_dmats(nunit), torch.float32),
                             _dev(I.uniform_u(8, nunit), torch.float32), tile=tile)
        return
    D = I.random_dmats(nunit)
    u = I.uniform_u(777, nunit)
    _check(orc, ops, D, u, torch.float32, tile=tile)


@pytest.mark.parametrize("nunit", [27, 64, 216])
def test_grids_of_several_rounds_bitwise(orc, ops, nunit):
    """groups_per_cu above the occupancy gives a grid of several rounds of
    work-groups (each with fewer tiles): every element still gets the same
    schedule per tile, so the result equals the resident grid's bit for bit,
    and the oracle's."""
    D = I.random_dmats(nunit).astype(np.float32)
    u = I.uniform_u(50021, nunit).astype(np.float32)
    base = _run(ops, D, u, torch.float32)
    for g in (8, 24):
        assert np.array_equal(_run(ops, D, u, torch.float32, dict(groups_per_cu=g)), base), g
    _check(orc, ops, D.astype(np.float64), u.astype(np.float64), torch.float32, tile=dict(groups_per_cu=24))


@pytest.mark.parametrize("nunit,tile", [(216, dict(elems_per_wave=32, waves=8)),
                                        (216, dict(elems_per_wave=32, waves=8, d_panels=6, groups_per_cu=1))])
def test_resolve_refuses_what_launch_refuses(ops, nunit, tile):
    """A shape whose work-group exceeds the kernel's bound is refused by the
    resolver as by the launch (same message), not resolved then refused."""
    with pytest.raises(ops.DGError, match="fit 64 registers"):
        ops.resolve_tile("f32", 3, 1000, nunit, tile)
    with pytest.raises(ops.DGError, match="fit 64 registers"):
        ops.dgdiff_apply(_dev(I.random_dmats(nunit), torch.float32),
                         _dev(I.uniform_u(1000, nunit), torch.float32), tile=tile)


@pytest.mark.parametrize("nunit", [8, 27, 64, 125, 216, 512])
@pytest.mark.parametrize("nelem", [1, 777, 4099])
def test_streaming_stores_bitwise(orc, ops, nunit, nelem):
    """DG_TILE_NT_STORE changes only the stores' cache policy: every store path
    (paired, single-panel vectors, rows staged through the wave's slab) gives
    the same bits with and without it, and matches the oracle."""
    D = _dev(I.random_dmats(nunit), torch.float32)
    u = _dev(I.uniform_u(nelem, nunit), torch.float32)
    t0 = ops.resolve_tile("f32", 3, nelem, nunit, None)
    t1 = dict(t0, flags=t0["flags"] | 1)
    a = ops.dgdiff_apply(D, u, tile=t0)
    b = ops.dgdiff_apply(D, u, tile=t1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    _check(orc, ops, I.random_dmats(nunit), I.uniform_u(nelem, nunit), torch.float32, tile=t1)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("nunit", [5, 27, 125])
@pytest.mark.parametrize("tile", [dict(elems_per_wave=16, d_panels=1), dict(elems_per_wave=16, d_panels=3),
                                  dict(elems_per_wave=32, d_panels=5), dict(elems_per_wave=16, waves=3),
                                  dict(elems_per_wave=64, d_panels=2)])
def test_unaligned_rows_staged_stores(orc, ops, dtype, nunit, tile):
    """Rows that are not 16-byte multiples go through the wave's LDS slab in
    both directions; panel groups that hold only part of an operator's rows
    write partial rows.  Element counts with ragged last tiles."""
    D = I.random_dmats(nunit)
    for nelem in (1, 63, 1001):
        u = I.uniform_u(nelem, nunit)
        _check_or_refused(orc, ops, D, u, dtype, tile)


@pytest.mark.parametrize("nunit", [32, 64, 96, 512])
@pytest.mark.parametrize("tile", [None, dict(elems_per_wave=32), dict(elems_per_wave=64), dict(d_panels=2),
                                  dict(d_panels=3), dict(d_panels=4, waves=3)])
def test_paired_stores(orc, ops, nunit, tile):
    """FP32 rows of a multiple of 32 nodes take the paired-store variant (two
    panels per step, halves traded between lanes c and c^8), also with several
    panel groups; odd groups (d_panels=3) fall back to single panels.  Ragged
    element counts leave the second store of a pair partly or wholly empty."""
    D = I.random_dmats(nunit)
    for nelem in (1, 9, 23, 1001):
        u = I.uniform_u(nelem, nunit)
        _check_or_refused(orc, ops, D, u, torch.float32, tile)


@pytest.mark.parametrize("nunit", [64, 512])
def test_paired_matches_single_panels_bitwise(ops, nunit):
    """Pairing reorders stores only: an even panel group (paired) and an odd
    one (single panels) give bit-identical results."""
    D = _dev(I.random_dmats(nunit), torch.float32)
    u = _dev(I.uniform_u(1001, nunit), torch.float32)
    a = ops.dgdiff_apply(D, u, tile=dict(d_panels=4))
    b = ops.dgdiff_apply(D, u, tile=dict(d_panels=3))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("nunit,tile", [(32, None), (64, None), (64, dict(elems_per_wave=32)),
                                        (64, dict(waves=4)), (128, None)])
def test_pipelined_loads_many_tiles(orc, ops, nunit, tile):
    """Paired-store launches with small fragments load the next tile's element
    data ahead of the current tile's stores: many tiles per stream, a ragged
    end; equal to the oracle and bit-identical to a launch with an odd panel
    group (single panels, loads not pipelined)."""
    D = I.random_dmats(nunit)
    u = I.uniform_u(300007, nunit)
    _check(orc, ops, D, u, torch.float32, tile=tile)
    Dg, ug = _dev(D, torch.float32), _dev(u, torch.float32)
    a = ops.dgdiff_apply(Dg, ug, tile=tile)
    b = ops.dgdiff_apply(Dg, ug, tile=dict(tile or {}, d_panels=3))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_integer_data_bit_exact(orc, ops, dtype):
    rng = np.random.default_rng(12)
    for nunit in (27, 64, 125):
        D = rng.integers(-3, 4, size=(3, nunit, nunit)).astype(np.float64)
        u = rng.integers(-7, 8, size=(150, nunit)).astype(np.float64)
        got = _run(ops, D, u, dtype)
        np.testing.assert_array_equal(got, orc.dg_forward(D, u))


def test_deterministic_and_guard_band(ops):
    nunit, nelem = 125, 1500
    D = _dev(I.random_dmats(nunit), torch.float32)
    u = _dev(I.uniform_u(nelem, nunit), torch.float32)
    n = 3 * nelem * nunit
    buf = torch.full((n + 2048,), 12345.0, device="cuda:0")
    out = buf[1024:1024 + n].view(3, nelem, nunit)
    ops.dgdiff_apply(D, u, out=out)
    first = out.clone()
    ops.dgdiff_apply(D, u, out=out)
    torch.cuda.synchronize()
    assert torch.equal(first, out)
    assert torch.all(buf[:1024] == 12345.0) and torch.all(buf[1024 + n:] == 12345.0)


def test_unaligned_pointers(orc, ops):
    """Views that start one element into a buffer take the scalar path."""
    nunit, nelem = 64, 200
    D = I.random_dmats(nunit)
    u = _as(I.uniform_u(nelem, nunit), torch.float32)
    ub = torch.zeros(nelem * nunit + 1, device="cuda:0")
    ub[1:] = _dev(u, torch.float32).reshape(-1)
    uv = ub[1:].view(nelem, nunit)
    ob = torch.zeros(3 * nelem * nunit + 1, device="cuda:0")
    ov = ob[1:].view(3, nelem, nunit)
    ops.dgdiff_apply(_dev(_as(D, torch.float32), torch.float32), uv, out=ov)
    torch.cuda.synchronize()
    from oracle.metrics import normwise_rel
    assert normwise_rel(ov.double().cpu().numpy(), orc.dg_forward(_as(D, torch.float32), u)) <= 1e-5


@pytest.mark.parametrize("nunit,nelem", [(5, 1), (10, 4099), (26, 513), (27, 37), (27, 300007), (30, 65)])
def test_slab_rows_vector_and_scalar_loads_bitwise(orc, ops, nunit, nelem):
    """Rows off 16-byte boundaries reach the wave's slab as 16-byte vectors
    when the source is aligned and value by value when it starts one element
    into a buffer: both give bit-identical results, equal to the oracle, over
    many tiles and a run whose last values end inside a vector
    (nelem * nunit not a multiple of 4)."""
    D = _as(I.random_dmats(nunit), torch.float32)
    u = _as(I.uniform_u(nelem, nunit), torch.float32)
    Dg, ug = _dev(D, torch.float32), _dev(u, torch.float32)
    ub = torch.zeros(nelem * nunit + 4, device="cuda:0")
    uv = ub[1:1 + nelem * nunit].view(nelem, nunit)
    uv.copy_(ug)
    a = ops.dgdiff_apply(Dg, ug)
    b = ops.dgdiff_apply(Dg, uv)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    from oracle.metrics import normwise_rel
    assert normwise_rel(a.double().cpu().numpy(), orc.dg_forward(D, u)) <= 1e-5


def test_nan_propagates_to_its_element_only(orc, ops):
    nunit, nelem = 27, 64
    D = I.random_dmats(nunit)
    u = I.uniform_u(nelem, nunit)
    u[5, 3] = np.nan
    got = _run(ops, D, u, torch.float32)
    assert np.all(np.isnan(got[:, 5, :]))
    mask = np.ones(nelem, bool)
    mask[5] = False
    ref = orc.dg_forward(_as(D, torch.float32), _as(u, torch.float32))
    from oracle.metrics import normwise_rel
    assert normwise_rel(got[:, mask, :], ref[:, mask, :]) <= 1e-5


def test_empty_is_noop(ops):
    D = torch.zeros(3, 64, 64, device="cuda:0")
    u = torch.zeros(0, 64, device="cuda:0")
    out = ops.dgdiff_apply(D, u)
    assert out.shape == (3, 0, 64)


def test_full_size_p3_every_element(orc, ops):
    """The benchmark's headline launch (hex p=3, 2^21 elements, GLL operators,
    FP32): every output against the FP64 oracle."""
    nunit, nelem = 64, 1 << 21
    D = _as(I.gll_dmats(3), torch.float32)
    u32 = np.asarray(I.uniform_u(nelem, nunit), dtype=np.float32)
    print(f"full size: FP32 nunit={nunit} nelem={nelem}, all outputs", flush=True)
    out = ops.dgdiff_apply(_dev(D, torch.float32), torch.from_numpy(u32).cuda())
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    del out
    ref = orc.dg_forward(D, u32.astype(np.float64))
    from oracle.metrics import normwise_rel
    assert normwise_rel(got, ref) <= 1e-5


@pytest.mark.parametrize("p,nelem", [(2, 1 << 21), (4, 1 << 21), (5, 1 << 21), (5, 1 << 20)])
def test_full_size_every_wave_tile(orc, ops, p, nelem):
    """The benchmark's other FP32 launches at full size: one element from
    every 16-element wave-tile and the whole first and last 512 elements
    against the FP64 oracle."""
    from sample_sets import every_tile
    nunit = (p + 1) ** 3
    D = _as(I.gll_dmats(p), torch.float32)
    u32 = np.asarray(I.uniform_u(nelem, nunit), dtype=np.float32)
    print(f"full size: FP32 nunit={nunit} nelem={nelem}, every wave-tile", flush=True)
    out = ops.dgdiff_apply(_dev(D, torch.float32), torch.from_numpy(u32).cuda())
    torch.cuda.synchronize()
    sel = every_tile(nelem, seed=p)
    ref = orc.dg_forward_select(D, u32.astype(np.float64), sel)        # [nsel][3][n]
    got = out[:, torch.from_numpy(sel).cuda(), :].permute(1, 0, 2).double().cpu().numpy()
    from oracle.metrics import normwise_rel
    assert normwise_rel(got, ref) <= 1e-5
