"""GPU parity of the quantiser (bit-exact against the oracle's independent
encoders) and of the BF16 / FP8-E4M3 DG path.

Two error measures for the low-precision forward:
  (i)  normwise, against the FP64 oracle on the unquantised FP32 inputs: the
       accuracy of the method, bounded by 2e-2 (BF16) and 8e-2 (FP8);
  (ii) against the FP64 oracle on the oracle's own dequantised inputs: the
       kernel alone.  Products of BF16/FP8 values are exact in FP32, so what
       remains is the FP32 accumulation; it is bounded elementwise by the
       classical dot-product bound |y - y_ref| <= n 2^-23 sum_j |D_ij| |u_j|
       (n = nunit; 2^-23 rather than 2^-24 allows the matrix core's internal
       sums to truncate instead of rounding to nearest).
"""
import numpy as np
import pytest
import torch

from oracle.metrics import normwise_rel
from paper_1904_09538_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_METHOD = {"bf16": 2e-2, "e4m3": 8e-2}


@pytest.fixture(scope="module")
def ops():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _q_gpu(ops, x32, to, per_row):
    q, inv = ops.dgdiff_quantize(torch.from_numpy(x32).cuda(), to, per_row=per_row)
    torch.cuda.synchronize()
    codes = q.view(torch.int16 if to == "bf16" else torch.uint8).cpu().numpy()
    return codes.view(np.uint16) if to == "bf16" else codes, inv.cpu().numpy()


def _special_rows():
    vals = np.array([0.0, -0.0, 1.0, -1.0, 448.0, 449.0, 464.0, 480.0, 1e30, -1e30, np.inf, -np.inf,
                     np.nan, 2.0 ** -6, 2.0 ** -7, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 1.0625,
                     1.1875, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.4e38, 1e-38, 1e-45, 255.99, 0.1],
                    dtype=np.float32)
    return vals


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("per_row", [True, False])
def test_quantize_bit_exact(orc, ops, to, per_row):
    rng = np.random.default_rng(21)
    x = rng.uniform(-1, 1, size=(300, 216)).astype(np.float32)
    x[7] *= 1e-3
    x[8] *= 37.0
    x[9] = 0.0
    x[10, :len(_special_rows())] = _special_rows() if to == "bf16" else np.nan_to_num(_special_rows())
    q, inv = _q_gpu(ops, x, to, per_row)
    qo, invo = orc.quantize(x, to, per_row)
    np.testing.assert_array_equal(q, qo)
    if to == "e4m3" or per_row:
        np.testing.assert_array_equal(inv, invo)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("rows,cols,misalign", [(1, 5, 0), (7, 13, 0), (4097, 216, 0), (3, 3001, 0),
                                                (1 << 14, 343, 0), (7, 13, 1), (1000, 27, 1)])
def test_quantize_one_scale_grid_wide(orc, ops, to, rows, cols, misalign):
    """One scale for the whole array: the grid-wide maximum and encode passes
    over many work-groups, 16-byte vectors with a value-by-value tail, and an
    input 4 bytes off 16-byte alignment (value-by-value throughout)."""
    rng = np.random.default_rng(rows + cols)
    x = rng.uniform(-1, 1, size=(rows, cols)).astype(np.float32)
    x[rows // 2, cols // 2] = 300.0          # the array's maximum, anywhere in the grid
    base = torch.empty(rows * cols + misalign, device="cuda")
    xt = base[misalign:].view(rows, cols)
    xt.copy_(torch.from_numpy(x).cuda())
    assert (xt.data_ptr() % 16 == 0) == (misalign == 0)
    q, inv = ops.dgdiff_quantize(xt, to, per_row=False)
    torch.cuda.synchronize()
    codes = q.view(torch.int16 if to == "bf16" else torch.uint8).cpu().numpy()
    codes = codes.view(np.uint16) if to == "bf16" else codes
    qo, invo = orc.quantize(x, to, False)
    np.testing.assert_array_equal(codes, qo)
    if to == "e4m3":
        np.testing.assert_array_equal(inv.cpu().numpy(), invo)
    else:
        assert inv.cpu().numpy().tolist() == [1.0]


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("cols", [1, 2, 3, 4, 5, 8, 9, 13, 16, 17, 27, 32, 33, 63, 64, 65, 125, 128, 129, 200,
                                  216, 255, 256, 257])
@pytest.mark.parametrize("rows", [1, 37, 1001])
def test_quantize_packed_rows(orc, ops, to, cols, rows):
    """Rows of up to 256 values share a wave (64 / SW rows of SW lanes): every
    row width and ragged last slot, codes and scales bit-equal to the oracle;
    one row scaled far up and one holding specials, so that each row's scale
    is its own."""
    rng = np.random.default_rng(1000 * cols + rows)
    x = rng.uniform(-1, 1, size=(rows, cols)).astype(np.float32)
    x[rows // 2] *= 300.0
    sp = _special_rows()
    if rows > 2:
        k = min(cols, len(sp))
        x[1, :k] = sp[:k] if to == "bf16" else np.nan_to_num(sp[:k])
    q, inv = _q_gpu(ops, x, to, True)
    qo, invo = orc.quantize(x, to, True)
    np.testing.assert_array_equal(q, qo)
    np.testing.assert_array_equal(inv.view(np.uint32), invo.view(np.uint32))


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
def test_quantize_random_bit_patterns(orc, ops, to):
    """2^20 random FP32 bit patterns (all exponents, NaN, inf, subnormals)
    in rows of 64: codes and scales bit-equal to the oracle."""
    rng = np.random.default_rng(22)
    bits = rng.integers(0, 2 ** 32, size=(1 << 14, 64), dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    q, inv = _q_gpu(ops, x, to, True)
    qo, invo = orc.quantize(x, to, True)
    np.testing.assert_array_equal(q, qo)
    np.testing.assert_array_equal(inv.view(np.uint32), invo.view(np.uint32))


def _dot_scaled(orc, got, ref, Dd, ud):
    den = orc.dg_forward(np.abs(Dd), np.abs(ud))
    return float(np.max(np.abs(got - ref) / np.maximum(den, 1e-300)))


def _lowp_case(orc, ops, D64, u64, to):
    D32, u32 = D64.astype(np.float32), u64.astype(np.float32)
    nmat, n, _ = D32.shape
    per_matrix = D32.reshape(nmat, n * n)
    # GPU path: quantise on the GPU, multiply on the GPU
    qD, isD = ops.dgdiff_quantize(torch.from_numpy(per_matrix).cuda(), to, per_row=True)
    qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to, per_row=True)
    out = ops.dgdiff_apply(qD.view(nmat, n, n), qu, inv_sD=isD if to == "e4m3" else None,
                           inv_su=isu if to == "e4m3" else None)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    # oracle path: its own quantiser and decoder, FP64 contraction
    qDo, isDo = orc.quantize(per_matrix, to, True)
    quo, isuo = orc.quantize(u32, to, True)
    if to == "bf16":
        Dd = orc.bf16_decode_array(qDo).astype(np.float64).reshape(nmat, n, n)
        ud = orc.bf16_decode_array(quo).astype(np.float64)
    else:
        Dd = (orc.e4m3_decode_array(qDo) * isDo[:, None]).reshape(nmat, n, n)
        ud = orc.e4m3_decode_array(quo) * isuo[:, None]
    ref_kernel = orc.dg_forward(Dd, ud)
    ref_method = orc.dg_forward(D32.astype(np.float64), u32.astype(np.float64))
    return _dot_scaled(orc, got, ref_kernel, Dd, ud) / (n * 2.0 ** -23), normwise_rel(got, ref_method)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("nunit", [8, 27, 64, 100, 125, 216, 343])
def test_lowp_forward(orc, ops, to, nunit):
    p = round(nunit ** (1 / 3)) - 1
    D = I.gll_dmats(p) if (p + 1) ** 3 == nunit else I.random_dmats(nunit)
    u = I.uniform_u(300, nunit)
    k_err, m_err = _lowp_case(orc, ops, D, u, to)
    assert k_err <= 1.0, k_err          # fraction of the FP32 accumulation bound
    assert m_err <= TOL_METHOD[to], m_err


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
def test_lowp_random_operators(orc, ops, to):
    D = I.random_dmats(216)
    u = I.uniform_u(500, 216)
    k_err, m_err = _lowp_case(orc, ops, D, u, to)
    assert k_err <= 1.0 and m_err <= TOL_METHOD[to]


def _oracle_dequantised(orc, D32, u32, to):
    """The oracle's own quantisation and decoding of the FP32 inputs."""
    nmat, n, _ = D32.shape
    qDo, isDo = orc.quantize(D32.reshape(nmat, -1), to, True)
    quo, isuo = orc.quantize(u32, to, True)
    if to == "bf16":
        Dd = orc.bf16_decode_array(qDo).astype(np.float64).reshape(nmat, n, n)
        ud = orc.bf16_decode_array(quo).astype(np.float64)
    else:
        Dd = (orc.e4m3_decode_array(qDo) * isDo[:, None]).reshape(nmat, n, n)
        ud = orc.e4m3_decode_array(quo) * isuo[:, None]
    return Dd, ud


_LDS = 8   # DG_TILE_LP_LDS_PANELS: the body with operator panels in LDS
LDS_PANEL_TILES = [dict(elems_per_wave=16, flags=_LDS), dict(elems_per_wave=32, flags=_LDS),
                   dict(elems_per_wave=64, flags=_LDS), dict(d_panels=5, flags=_LDS),
                   dict(d_panels=1, flags=_LDS), dict(waves=2, flags=_LDS),
                   dict(waves=3, elems_per_wave=32, flags=_LDS), dict(groups_per_cu=1, flags=_LDS)]
# staged body: one or two row blocks per wave, whole-row and split row groups
# (ragged last group at nunit 216: 14 blocks in groups of 4, 6 or 8), waves
# with fewer valid blocks than they hold, one or two column blocks per tile
STAGED_TILES = [None, dict(elems_per_wave=32), dict(waves=8, d_panels=8), dict(waves=9, d_panels=9),
                dict(waves=12, d_panels=12), dict(waves=16, d_panels=16), dict(waves=7, d_panels=14),
                dict(waves=8, d_panels=16, elems_per_wave=32), dict(groups_per_cu=1), dict(waves=7, d_panels=7)]


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("nunit", [64, 216])
@pytest.mark.parametrize("tile", LDS_PANEL_TILES + STAGED_TILES)
def test_lowp_tiles(orc, ops, to, nunit, tile):
    """Launch shapes of both low-precision bodies against the FP64 oracle on
    the oracle's dequantised inputs (the FP32 accumulation bound), ragged
    element counts."""
    p = round(nunit ** (1 / 3)) - 1
    D32 = I.gll_dmats(p).astype(np.float32)
    for nelem in (1, 333):
        u32 = I.uniform_u(nelem, nunit).astype(np.float32)
        qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), to)
        qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to)
        sc = dict(inv_sD=isD, inv_su=isu) if to == "e4m3" else {}
        got = ops.dgdiff_apply(qD.view(3, nunit, nunit), qu, tile=tile, **sc)
        torch.cuda.synchronize()
        Dd, ud = _oracle_dequantised(orc, D32, u32, to)
        err = _dot_scaled(orc, got.double().cpu().numpy(), orc.dg_forward(Dd, ud), Dd, ud)
        assert err <= nunit * 2.0 ** -23, (nelem, err)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("nunit,tile", [(32, dict(flags=_LDS)), (64, dict(flags=_LDS)),
                                        (64, dict(d_panels=2, flags=_LDS)), (64, dict(d_panels=3, flags=_LDS)),
                                        (64, dict(elems_per_wave=64, flags=_LDS)),
                                        (512, dict(d_panels=8, flags=_LDS)), (512, dict(flags=_LDS))])
def test_lowp_paired_stores(orc, ops, to, nunit, tile):
    """LDS-panel body: rows of a multiple of 32 nodes take the paired-store
    variant when the panel groups are even (scales applied per element before
    the exchange); ragged element counts; odd groups fall back to single
    panels."""
    D = I.gll_dmats(3) if nunit == 64 else I.random_dmats(nunit)
    D32 = D.astype(np.float32)
    for nelem in (1, 9, 300):
        u32 = I.uniform_u(nelem, nunit).astype(np.float32)
        qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), to)
        qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to)
        sc = dict(inv_sD=isD, inv_su=isu) if to == "e4m3" else {}
        got = ops.dgdiff_apply(qD.view(3, nunit, nunit), qu, tile=tile, **sc)
        torch.cuda.synchronize()
        # the oracle on the oracle's own dequantised operands
        qDo, isDo = orc.quantize(D32.reshape(3, -1), to, True)
        quo, isuo = orc.quantize(u32, to, True)
        if to == "bf16":
            Dd = orc.bf16_decode_array(qDo).astype(np.float64).reshape(3, nunit, nunit)
            ud = orc.bf16_decode_array(quo).astype(np.float64)
        else:
            Dd = (orc.e4m3_decode_array(qDo) * isDo[:, None]).reshape(3, nunit, nunit)
            ud = orc.e4m3_decode_array(quo) * isuo[:, None]
        ref = orc.dg_forward(Dd, ud)
        err = _dot_scaled(orc, got.double().cpu().numpy(), ref, Dd, ud) / (nunit * 2.0 ** -23)
        assert err <= 1.0, (nelem, err)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
def test_lowp_paired_matches_single_panels_bitwise(ops, to):
    D32 = I.gll_dmats(3).astype(np.float32)
    u32 = I.uniform_u(1001, 64).astype(np.float32)
    qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), to)
    qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to)
    sc = dict(inv_sD=isD, inv_su=isu) if to == "e4m3" else {}
    a = ops.dgdiff_apply(qD.view(3, 64, 64), qu, tile=dict(d_panels=4, flags=_LDS), **sc)
    b = ops.dgdiff_apply(qD.view(3, 64, 64), qu, tile=dict(d_panels=3, flags=_LDS), **sc)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _quantised(ops, D32, u32, to):
    nmat, n, _ = D32.shape
    qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(nmat, -1)).cuda(), to)
    qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to)
    sc = dict(inv_sD=isD, inv_su=isu) if to == "e4m3" else {}
    return qD.view(nmat, n, n), qu, sc


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("nunit,nmat,nelem,tile", [
    (8, 3, 1, None), (8, 3, 4097, None), (40, 3, 300, None), (40, 2, 300, dict(waves=3, d_panels=3)),
    (64, 3, 1001, None), (64, 1, 17, dict(elems_per_wave=32)), (216, 3, 5001, None),
    (216, 3, 5001, dict(waves=9, d_panels=9)), (216, 5, 333, dict(elems_per_wave=32, waves=7)),
    (512, 3, 700, None), (512, 3, 700, dict(waves=16, d_panels=16, elems_per_wave=32)),
    (256, 8, 200, dict(waves=8, d_panels=8))])
def test_lowp_staged_equals_lds_panels_bitwise(ops, to, nunit, nmat, nelem, tile):
    """The staged body runs the LDS-panel body's products in the same order
    (same fragments, same k-steps, same de-scaling): bit-identical outputs,
    whatever the row groups, tile and ragged end."""
    D32 = I.random_dmats(nunit, nmat).astype(np.float32)
    u32 = I.uniform_u(nelem, nunit).astype(np.float32)
    qD, qu, sc = _quantised(ops, D32, u32, to)
    dt = "bf16" if to == "bf16" else "fp8"
    t = ops.resolve_tile(dt, nmat, nelem, nunit, tile)
    ref = ops.dgdiff_apply(qD, qu, tile=dict(flags=_LDS), **sc)
    got = ops.dgdiff_apply(qD, qu, tile=t, **sc)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), (t, (got - ref).abs().max().item())


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
def test_lowp_misaligned_falls_back(orc, ops, to):
    """Element data that do not start on a 16-byte boundary take the LDS-panel
    body: the same values as the aligned call."""
    n, E = 64, 250
    D32 = I.gll_dmats(3).astype(np.float32)
    u32 = I.uniform_u(E, n).astype(np.float32)
    qD, qu, sc = _quantised(ops, D32, u32, to)
    buf = torch.empty(E * n + 8, dtype=qu.dtype, device="cuda")
    mis = buf[1:1 + E * n].view(E, n)            # one value (1 or 2 bytes) past alignment
    mis.copy_(qu)
    a = ops.dgdiff_apply(qD, qu, **sc)
    b = ops.dgdiff_apply(qD, mis, **sc)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_lowp_staged_refusals(ops):
    """Shapes the staged body cannot run are refused before any launch."""
    for nunit, tile in ((512, dict(waves=8, d_panels=16)),      # two blocks per wave past nunit 256
                        (512, dict(waves=2)),                    # too few threads to stage a tile
                        (64, dict(elems_per_wave=64)),           # tiles are 16 or 32 elements
                        (64, dict(waves=3, d_panels=7)),         # d_panels not a multiple of waves
                        (216, dict(waves=4, d_panels=8))):       # fewer than nunit / 32 waves
        with pytest.raises(ops.DGError):
            ops.resolve_tile("bf16", 3, 1000, nunit, tile)


_QU = 16   # DG_TILE_QUANT_U


@pytest.mark.parametrize("nunit", [8, 40, 64, 216, 256, 512])
@pytest.mark.parametrize("nelem", [1, 17, 4099])
def test_fused_bf16_rounding_is_quantise_then_apply(orc, ops, nunit, nelem):
    """FP32 element data rounded to BF16 inside the staged body: bit for bit
    the two-step path (dgdiff_quantize to BF16, then dgdiff_apply), specials
    included, and within the kernel bound of the oracle on the rounded data."""
    rng = np.random.default_rng(nunit * 7 + nelem)
    D32 = (rng.standard_normal((3, nunit, nunit)) / np.sqrt(nunit)).astype(np.float32)
    u32 = rng.uniform(-1, 1, (nelem, nunit)).astype(np.float32)
    u32[0, :min(nunit, 6)] = np.array([np.nan, np.inf, -np.inf, 3.0e38, 1e-40, -0.0], np.float32)[:min(nunit, 6)]
    if nelem > 2:
        u32[2] *= 1e5
    qD, _ = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), "bf16", per_row=True)
    qD = qD.view(3, nunit, nunit)
    ug = torch.from_numpy(u32).cuda()
    qu, _ = ops.dgdiff_quantize(ug, "bf16", per_row=True)
    two = ops.dgdiff_apply(qD, qu)
    one = ops.dgdiff_apply(qD, ug, tile=dict(flags=_QU))
    torch.cuda.synchronize()
    assert torch.equal(one.view(torch.int32), two.view(torch.int32))
    # the oracle on the rounded data (rows free of specials: all but 0 and 2)
    rows = np.array([r for r in range(nelem) if r not in (0, 2)], dtype=np.int64)
    if rows.size:
        quo, _ = orc.quantize(u32[rows], "bf16", True)
        qDo, _ = orc.quantize(D32.reshape(3, -1), "bf16", True)
        Dd = orc.bf16_decode_array(qDo).astype(np.float64).reshape(3, nunit, nunit)
        ud = orc.bf16_decode_array(quo).astype(np.float64)
        got = one.double().cpu().numpy()[:, rows, :]
        assert _dot_scaled(orc, got, orc.dg_forward(Dd, ud), Dd, ud) <= nunit * 2.0 ** -23


def test_fused_bf16_refusals(ops):
    """The fused rounding runs in the staged body only."""
    qD = torch.zeros(3, 27, 27, dtype=torch.bfloat16, device="cuda:0")
    u = torch.zeros(10, 27, device="cuda:0")
    with pytest.raises(ops.DGError):                      # rows off a multiple of 8
        ops.dgdiff_apply(qD, u, tile=dict(flags=_QU))
    qD = torch.zeros(3, 64, 64, dtype=torch.bfloat16, device="cuda:0")
    u = torch.zeros(10, 64, device="cuda:0")
    for tile in (dict(flags=_QU | 8), dict(flags=_QU, elems_per_wave=32)):
        with pytest.raises(ops.DGError):
            ops.dgdiff_apply(qD, u, tile=tile)
    with pytest.raises(TypeError):                        # u must be FP32
        ops.dgdiff_apply(qD, u.bfloat16(), tile=dict(flags=_QU))


def test_fused_bf16_full_size(ops):
    """p = 5, 2^20 elements (the low-precision workload): fused equals two-step."""
    from paper_1904_09538_amd import inputs as I
    n, E = 216, 1 << 20
    D = torch.from_numpy(I.gll_dmats(5).astype(np.float32)).cuda()
    u = torch.from_numpy(I.uniform_u(E, n).astype(np.float32)).cuda()
    qD, _ = ops.dgdiff_quantize(D.reshape(3, -1), "bf16", per_row=True)
    qD = qD.view(3, n, n)
    qu, _ = ops.dgdiff_quantize(u, "bf16", per_row=True)
    two = ops.dgdiff_apply(qD, qu)
    one = ops.dgdiff_apply(qD, u, tile=dict(flags=_QU))
    torch.cuda.synchronize()
    assert torch.equal(one, two)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("nunit", [64, 216])
def test_lowp_grids_of_several_rounds_bitwise(ops, to, nunit):
    """groups_per_cu above the occupancy (several rounds of work-groups on
    the staged body) equals the resident grid bit for bit."""
    p = round(nunit ** (1 / 3)) - 1
    D32 = I.gll_dmats(p).astype(np.float32)
    u32 = I.uniform_u(50021, nunit).astype(np.float32)
    qD, qu, sc = _quantised(ops, D32, u32, to)
    base = ops.dgdiff_apply(qD, qu, **sc)
    for g in (8, 24):
        got = ops.dgdiff_apply(qD, qu, tile=dict(groups_per_cu=g), **sc)
        torch.cuda.synchronize()
        assert torch.equal(got, base), g


def test_fp8_requires_scales(ops):
    q = torch.zeros(3, 64, 64, dtype=torch.float8_e4m3fn, device="cuda:0")
    u = torch.zeros(10, 64, dtype=torch.float8_e4m3fn, device="cuda:0")
    with pytest.raises(ops.DGError):
        ops.dgdiff_apply(q, u)


@pytest.mark.parametrize("to", ["bf16", "e4m3"])
@pytest.mark.parametrize("p,E", [(5, 1 << 20), (3, 1 << 21)])
def test_lowp_full_size_sampled(orc, ops, to, p, E):
    """Hex p=5, 2^20 elements (the low-precision benchmark configuration) and
    hex p=3, 2^21 (paired stores): one element of every 16-element wave-tile
    and the whole first and last 512, and the sampled rows' quantiser codes
    and scales bit-equal to the oracle's."""
    print(f"full size: {to} p={p} nelem={E}", flush=True)
    n = (p + 1) ** 3
    D32 = I.gll_dmats(p).astype(np.float32)
    u32 = np.asarray(I.uniform_u(E, n), dtype=np.float32)
    qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), to)
    qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), to)
    out = ops.dgdiff_apply(qD.view(3, n, n), qu, inv_sD=isD if to == "e4m3" else None,
                           inv_su=isu if to == "e4m3" else None)
    torch.cuda.synchronize()
    from sample_sets import every_tile
    sel = every_tile(E, seed=31)
    got = out[:, torch.from_numpy(sel).cuda(), :].permute(1, 0, 2).double().cpu().numpy()
    us = u32[sel]
    qDo, isDo = orc.quantize(D32.reshape(3, -1), to, True)
    quo, isuo = orc.quantize(us, to, True)
    codes = qu[torch.from_numpy(sel).cuda()].view(torch.int16 if to == "bf16" else torch.uint8).cpu().numpy()
    np.testing.assert_array_equal(codes.view(np.uint16) if to == "bf16" else codes, quo)
    if to == "e4m3":
        np.testing.assert_array_equal(isu[torch.from_numpy(sel).cuda()].cpu().numpy(), isuo)
    if to == "bf16":
        Dd = orc.bf16_decode_array(qDo).astype(np.float64).reshape(3, n, n)
        ud = orc.bf16_decode_array(quo).astype(np.float64)
    else:
        Dd = (orc.e4m3_decode_array(qDo) * isDo[:, None]).reshape(3, n, n)
        ud = orc.e4m3_decode_array(quo) * isuo[:, None]
    ref_k = orc.dg_forward(Dd, ud).transpose(1, 0, 2)
    den = orc.dg_forward(np.abs(Dd), np.abs(ud)).transpose(1, 0, 2)
    ref_m = orc.dg_forward(D32.astype(np.float64), us.astype(np.float64)).transpose(1, 0, 2)
    assert np.max(np.abs(got - ref_k) / den) <= n * 2.0 ** -23
    assert normwise_rel(got, ref_m) <= TOL_METHOD[to]


def test_fp8_native_instruction_flag(orc, ops):
    """The opt-in native FP8 matrix instruction: same method accuracy bound;
    its internal 32-product sums are coarser than FP32, bounded here by
    2^-12 of sum_j |D_ij| |u_j| (measured worst about 2^-12.8)."""
    n = 216
    D32 = I.gll_dmats(5).astype(np.float32)
    u32 = I.uniform_u(400, n).astype(np.float32)
    qD, isD = ops.dgdiff_quantize(torch.from_numpy(D32.reshape(3, -1)).cuda(), "e4m3")
    qu, isu = ops.dgdiff_quantize(torch.from_numpy(u32).cuda(), "e4m3")
    got = ops.dgdiff_apply(qD.view(3, n, n), qu, inv_sD=isD, inv_su=isu,
                           tile=dict(flags=ops.DG_TILE_FP8_NATIVE))
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    qDo, isDo = orc.quantize(D32.reshape(3, -1), "e4m3", True)
    quo, isuo = orc.quantize(u32, "e4m3", True)
    Dd = (orc.e4m3_decode_array(qDo) * isDo[:, None]).reshape(3, n, n)
    ud = orc.e4m3_decode_array(quo) * isuo[:, None]
    assert _dot_scaled(orc, got, orc.dg_forward(Dd, ud), Dd, ud) <= 2.0 ** -12
    ref_m = orc.dg_forward(D32.astype(np.float64), u32.astype(np.float64))
    assert normwise_rel(got, ref_m) <= TOL_METHOD["e4m3"]
