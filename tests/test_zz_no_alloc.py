"""dgdiff_backward_noalloc, the backward entry point that allocates nothing,
against dgdiff_backward (which takes a caller workspace) and the FP64 oracle.

Two calls in a row on the same GPU, the second with a smaller input, so the
second reads the fixed scratch the first left behind.  grad_u runs the same
kernels in both entry points (bit-equal); grad_D may be split into fewer
element ranges when the partials would not fit the fixed scratch, so it is
compared at the parity tolerance (FP32 1e-5, FP64 1e-12 normwise).
"""
import numpy as np
import pytest
import torch

from oracle.metrics import normwise_rel
from paper_1904_09538_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _t(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dtype)


def _as(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x


def _inputs(p, nelem, dtype, random_D):
    n = I.nunit_of_order(p)
    D = I.random_dmats(n, nmat=3) if random_D else I.gll_dmats(p)
    return _as(D, dtype), _as(I.uniform_u(nelem, n), dtype), _as(I.normal_g(3, nelem, n), dtype)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_two_calls_match_backward(orc, ops, dtype):
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    # (order, elements): a large call whose grad_D partials fill the scratch,
    # then a smaller one with a ragged element count
    for p, nelem, random_D in ((4, 1 << 17, False), (3, 3001, True)):
        print(f"noalloc: dtype={dtype} p={p} nelem={nelem}", flush=True)
        D, u, g = _inputs(p, nelem, dtype, random_D)
        Dt, ut, gt = _t(D, dtype), _t(u, dtype), _t(g, dtype)
        gu_ref, gD_ref = ops.dgdiff_backward(Dt, ut, gt)
        gu, gD = ops.dgdiff_backward_noalloc(Dt, ut, gt)
        torch.cuda.synchronize()
        assert torch.equal(gu, gu_ref)
        assert normwise_rel(gD.double().cpu().numpy(), gD_ref.double().cpu().numpy()) <= tol
        if nelem <= 4096:
            ru, rD = orc.dg_adjoint(D, u, g)
            assert normwise_rel(gu.double().cpu().numpy(), ru) <= tol
            assert normwise_rel(gD.double().cpu().numpy(), rD) <= tol
        del Dt, ut, gt, gu_ref, gD_ref, gu, gD


def test_noalloc_grad_D_only_and_empty(orc, ops):
    D, u, g = _inputs(2, 517, torch.float32, True)
    _, gD = ops.dgdiff_backward_noalloc(_t(D, torch.float32), _t(u, torch.float32), _t(g, torch.float32),
                                        want_u=False)
    torch.cuda.synchronize()
    _, rD = orc.dg_adjoint(D, u, g, want_u=False)
    assert normwise_rel(gD.double().cpu().numpy(), rD) <= 1e-5
    # no elements: grad_D is the empty sum
    D0 = _t(D, torch.float32)
    u0 = torch.empty((0, D.shape[1]), device="cuda:0")
    g0 = torch.empty((3, 0, D.shape[1]), device="cuda:0")
    gu0, gD0 = ops.dgdiff_backward_noalloc(D0, u0, g0)
    torch.cuda.synchronize()
    assert gu0.numel() == 0 and torch.count_nonzero(gD0).item() == 0


def test_noalloc_rejects_beyond_scratch(ops):
    # FP64, 8 operators of 512 nodes: 2 * 8 * 512^2 * 8 bytes = 32 MiB > 24 MiB
    nmat, n, nelem = 8, 512, 16
    D = torch.zeros((nmat, n, n), dtype=torch.float64, device="cuda:0")
    u = torch.zeros((nelem, n), dtype=torch.float64, device="cuda:0")
    g = torch.zeros((nmat, nelem, n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ops.DGError) as ei:
        ops.dgdiff_backward_noalloc(D, u, g, want_u=False)
    assert ei.value.status == ops.DG_EUNSUPPORTED
    assert "fixed scratch" in str(ei.value)
