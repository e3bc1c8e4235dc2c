"""GPU parity of the program variants (dg_variant_run) against the FP64
oracle: the full variants against the plain operations (dg_forward,
stencil5, matmul; FP32 tolerance 1e-5 normwise, exact on small-integer
data), their work-removed twins bit for bit against oracle/variants.py on
small-integer inputs, including the untouched (NaN-filled) part of a result
array; and the variant-study sizes on sampled outputs."""
import numpy as np
import pytest
import torch

from oracle import variants as OV
from oracle.metrics import normwise_rel
from paper_1904_09538_amd import inputs as I

pytestmark = pytest.mark.gpu

DG = ("dg_nopf", "dg_pfu", "dg_pfdm", "dg_pfdmt")


@pytest.fixture(scope="module")
def ops():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _ints(shape, seed, lo=-4, hi=5):
    return np.random.default_rng(seed).integers(lo, hi, shape).astype(np.float64)


def _dg(ops, kind, D, u, nmat):
    """Run a DG variant on element-major u [E][nunit]; returns [nmat][E][nunit]."""
    E, nu = u.shape
    tr = kind == "dg_pfdmt"
    ug = _dev(u.T if tr else u)
    out = torch.full((nmat, nu, E) if tr else (nmat, E, nu), float("nan"), device="cuda")
    ops.dg_variant_run(kind, E, ug, _dev(D), out, nunit=nu, nmat=nmat)
    torch.cuda.synchronize()
    r = out.double().cpu().numpy()
    return np.transpose(r, (0, 2, 1)) if tr else r


@pytest.mark.parametrize("kind", DG)
@pytest.mark.parametrize("E,nu,M", [(1, 64, 3), (17, 64, 3), (300, 64, 3), (40, 16, 1), (70, 32, 8),
                                    (33, 48, 5)])
def test_dg_variant_parity(orc, ops, kind, E, nu, M):
    D = I.as_f32(I.random_dmats(nu, M)).astype(np.float64)
    u = I.as_f32(I.uniform_u(E, nu)).astype(np.float64)
    got = _dg(ops, kind, D, u, M)
    assert np.all(np.isfinite(got))
    assert normwise_rel(got, orc.dg_forward(D, u)) <= 1e-5


@pytest.mark.parametrize("kind", DG)
def test_dg_variant_integer_exact(orc, ops, kind):
    D, u = _ints((3, 64, 64), 1), _ints((45, 64), 2)
    assert np.array_equal(_dg(ops, kind, D, u, 3), orc.dg_forward(D, u))


@pytest.mark.parametrize("kind", ["mm_pf", "mm_nopf"])
@pytest.mark.parametrize("n", [16, 48, 128])
def test_matmul_variant_parity(orc, ops, kind, n):
    a, b = (I.as_f32(x).astype(np.float64) for x in I.matmul_operands(n))
    c = torch.full((n, n), float("nan"), device="cuda")
    ops.dg_variant_run(kind, n, _dev(a), _dev(b), c)
    torch.cuda.synchronize()
    assert normwise_rel(c.double().cpu().numpy(), orc.matmul(a, b)) <= 1e-5
    ai, bi = _ints((n, n), 3), _ints((n, n), 4)
    ops.dg_variant_run(kind, n, _dev(ai), _dev(bi), c)
    torch.cuda.synchronize()
    assert np.array_equal(c.double().cpu().numpy(), orc.matmul(ai, bi))


def _fd(ops, kind, u, n, ld_u, ld_res):
    ug = torch.full((n + 2, ld_u), float("nan"), device="cuda")
    ug[:, :n + 2] = _dev(u)
    res = torch.full((max(n, 1), ld_res), -7.0, device="cuda")
    ops.dg_variant_run(kind, n, ug, None, res, ld_u=ld_u, ld_res=ld_res)
    torch.cuda.synchronize()
    return res.double().cpu().numpy()


@pytest.mark.parametrize("kind", ["fd16", "fd18"])
@pytest.mark.parametrize("n,pad", [(1, 0), (13, 3), (14, 0), (15, 1), (16, 0), (17, 5), (100, 28), (255, 1)])
def test_stencil_variant_parity(orc, ops, kind, n, pad):
    u = I.as_f32(I.stencil_grid(n)).astype(np.float64)
    got = _fd(ops, kind, u, n, n + 2 + pad, n + pad)
    assert normwise_rel(got[:n, :n], orc.stencil5(u)) <= 1e-5
    assert np.all(got[:n, n:] == -7.0)                 # pitch padding untouched
    ui = _ints((n + 2, n + 2), 5, -50, 50)
    got = _fd(ops, kind, ui, n, n + 2 + pad, n + pad)
    assert np.array_equal(got[:n, :n], orc.stencil5(ui))


def _twin_case(ops, kind, keep, n, nunit=0, nmat=0):
    """Run a twin on small-integer inputs; returns (got, want) arrays."""
    gx, gy, T = OV.shape(kind, n, nunit)
    if kind.startswith("mm"):
        a, b = _ints((n, n), 11), _ints((n, n), 12)
        res_shape, ld_u, ld_res = (n, n), 0, 0
    elif kind.startswith("dg"):
        a = _ints((nunit, n) if kind == "dg_pfdmt" else (n, nunit), 13)
        b = _ints((nmat, nunit, nunit), 14)
        res_shape = (nmat, nunit, n) if kind == "dg_pfdmt" else (nmat, n, nunit)
        ld_u = ld_res = 0
    else:
        a, b = _ints((n + 2, n + 2), 15), None
        ld_u, ld_res = n + 2, n + 1
        res_shape = (n, ld_res)
    ag = _dev(a) if keep & 1 else None
    bg = _dev(b) if (keep & 2 and b is not None) else None
    if keep & 4:
        out = torch.full(res_shape, float("nan"), device="cuda")
    else:
        out = torch.full((gx * gy * T,), float("nan"), device="cuda")
    ops.dg_variant_run(kind, n, ag, bg, out, nunit=nunit, nmat=nmat, ld_u=ld_u, ld_res=ld_res,
                       work_removed=True, keep=keep)
    torch.cuda.synchronize()
    dest, res = OV.twin(kind, keep, n, a, b, nunit, nmat, ld_res)
    return out.double().cpu().numpy(), (dest if res is None else res)


@pytest.mark.parametrize("kind,n,nunit,nmat", [
    ("mm_pf", 48, 0, 0), ("mm_nopf", 32, 0, 0), ("dg_nopf", 37, 32, 3), ("dg_pfu", 37, 32, 3),
    ("dg_pfdm", 37, 32, 3), ("dg_pfdmt", 37, 32, 3), ("dg_pfu", 16, 64, 8), ("fd16", 31, 0, 0),
    ("fd18", 33, 0, 0)])
def test_twins_exact(ops, kind, n, nunit, nmat):
    for keep in range(8):
        if kind.startswith("fd") and keep & 2:
            continue
        got, want = _twin_case(ops, kind, keep, n, nunit, nmat)
        np.testing.assert_array_equal(got, want, err_msg=f"{kind} keep={keep}")


def test_study_size_dg_sampled(orc, ops):
    """The largest DG size of the variant study (2^19 elements, nunit 64,
    nmat 3) on a sample of elements."""
    E, nu, M = 1 << 19, 64, 3
    D = I.as_f32(I.random_dmats(nu, M)).astype(np.float64)
    u = I.as_f32(I.uniform_u(E, nu)).astype(np.float64)
    sel = np.unique(np.concatenate([np.arange(16), E - 1 - np.arange(16),
                                    np.random.default_rng(7).integers(0, E, 200)]))
    want = np.transpose(orc.dg_forward_select(D, u, sel), (1, 0, 2))     # [m][sel][i]
    for kind in DG:
        got = _dg(ops, kind, D, u, M)
        assert normwise_rel(got[:, sel, :], want) <= 1e-5, kind


def test_study_size_matmul_and_stencil_sampled(orc, ops):
    n = 2048
    a, b = (I.as_f32(x).astype(np.float64) for x in I.matmul_operands(n))
    rng = np.random.default_rng(8)
    ii, jj = rng.integers(0, n, 300), rng.integers(0, n, 300)
    want = orc.matmul_select(a, b, ii, jj)
    for kind in ("mm_pf", "mm_nopf"):
        c = torch.empty((n, n), device="cuda")
        ops.dg_variant_run(kind, n, _dev(a), _dev(b), c)
        torch.cuda.synchronize()
        assert normwise_rel(c.double().cpu().numpy()[ii, jj], want) <= 1e-5, kind
    n = 8190
    u = I.as_f32(I.stencil_grid(n)).astype(np.float64)
    ii, jj = rng.integers(0, n, 500), rng.integers(0, n, 500)
    want = orc.stencil5_select(u, ii, jj)
    for kind in ("fd16", "fd18"):
        res = _fd(ops, kind, u, n, n + 2, n)
        assert normwise_rel(res[ii, jj], want) <= 1e-5, kind


def test_refused_on_gpu(ops):
    u = torch.zeros(64, device="cuda")
    with pytest.raises(ops.DGError):
        ops.dg_variant_run("dg_pfu", 1, u, u, u, nunit=64, nmat=3)              # output overlaps
    with pytest.raises(ops.DGError):
        ops.dg_variant_run("mm_pf", 16, None, u, u)                              # NULL input
