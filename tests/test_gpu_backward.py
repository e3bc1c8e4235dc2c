"""GPU parity of the adjoint (dgdiff_backward) and of the autograd Function.

Checks: the FP64 oracle adjoint (FP64 <= 1e-12, FP32 <= 1e-5 normwise); the
dot-product identity <g, out> = <grad_u, u> = <grad_D, D>; FP64 central finite
differences (h = 1e-6) on a 64-element slice; torch.autograd.gradcheck;
full-size sampled parity; bit-identical reruns.
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


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nunit", [8, 27, 64, 125, 216, 343, 512])
def test_backward_vs_oracle(orc, ops, dtype, nunit):
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for nmat, nelem in ((3, 300), (1, 33), (2, 1), (4, 70)):
        D = _as(I.random_dmats(nunit, nmat=nmat), dtype)
        u = _as(I.uniform_u(nelem, nunit), dtype)
        g = _as(I.normal_g(nmat, nelem, nunit), dtype)
        gu, gD = ops.dgdiff_backward(_t(D, dtype), _t(u, dtype), _t(g, dtype))
        torch.cuda.synchronize()
        ru, rD = orc.dg_adjoint(D, u, g)
        assert normwise_rel(gu.double().cpu().numpy(), ru) <= tol
        assert normwise_rel(gD.double().cpu().numpy(), rD) <= tol


@pytest.mark.parametrize("nunit", [97, 128, 129, 256])
def test_grad_u_gemm_edges(orc, ops, nunit):
    """FP32 grad_u from 97 nodes on runs as a 128 x 128-tile GEMM: node counts
    at and across the tile edge, element counts around the 128-element tile
    and around the grouping of tiles by XCD (8 tiles)."""
    for nmat, nelem in ((3, 127), (3, 129), (1, 128 * 9 + 5), (2, 1)):
        D = _as(I.random_dmats(nunit, nmat=nmat), torch.float32)
        u = _as(I.uniform_u(nelem, nunit), torch.float32)
        g = _as(I.normal_g(nmat, nelem, nunit), torch.float32)
        gu, _ = ops.dgdiff_backward(_t(D, torch.float32), _t(u, torch.float32), _t(g, torch.float32),
                                    want_D=False)
        torch.cuda.synchronize()
        ru, _ = orc.dg_adjoint(D, u, g, want_D=False)
        assert normwise_rel(gu.double().cpu().numpy(), ru) <= 1e-5, (nmat, nelem)


def test_backward_partial_outputs_and_empty(orc, ops):
    D = I.random_dmats(64)
    u = I.uniform_u(100, 64)
    g = I.normal_g(3, 100, 64)
    gu, gD = ops.dgdiff_backward(_t(D, torch.float64), _t(u, torch.float64), _t(g, torch.float64),
                                 want_D=False)
    assert gD is None
    ru, rD = orc.dg_adjoint(D, u, g)
    assert normwise_rel(gu.cpu().numpy(), ru) <= 1e-12
    gu, gD = ops.dgdiff_backward(_t(D, torch.float64), _t(u, torch.float64), _t(g, torch.float64),
                                 want_u=False)
    assert gu is None and normwise_rel(gD.cpu().numpy(), rD) <= 1e-12
    # empty batch: grad_D is the empty sum, 0
    gu, gD = ops.dgdiff_backward(_t(D, torch.float32), torch.zeros(0, 64, device="cuda:0"),
                                 torch.zeros(3, 0, 64, device="cuda:0"))
    torch.cuda.synchronize()
    assert gu.shape == (0, 64) and torch.all(gD == 0)


def test_dot_product_identity(ops):
    D = _t(I.gll_dmats(4), torch.float64)
    u = _t(I.uniform_u(500, 125), torch.float64)
    g = _t(I.normal_g(3, 500, 125), torch.float64)
    out = ops.dgdiff_apply(D, u)
    gu, gD = ops.dgdiff_backward(D, u, g)
    L = float((g * out).sum())
    assert abs(float((gu * u).sum()) - L) <= 1e-12 * abs(L)
    assert abs(float((gD * D).sum()) - L) <= 1e-12 * abs(L)


def test_central_differences_64_element_slice(orc, ops):
    """Hex p=4, elements 0..63 of the seeded inputs, FP64: every entry of u and
    D.  L = <g, out> is linear in each argument, so a central difference has no
    truncation error; only the rounding of L enters (about eps*|L|/h)."""
    n, E, h = 125, 64, 1e-6
    D = I.gll_dmats(4)
    u = I.uniform_u(1 << 19, n)[:E]
    g = I.normal_g(3, 1 << 19, n)[:, :E, :]
    gu, gD = ops.dgdiff_backward(_t(D, torch.float64), _t(u, torch.float64), _t(g, torch.float64))
    torch.cuda.synchronize()
    gu, gD = gu.cpu().numpy(), gD.cpu().numpy()
    # u entries: only element e's outputs move, evaluate L on that element
    fd_u = np.empty_like(u)
    for e in range(E):
        for j in range(n):
            up, um = u[e:e + 1].copy(), u[e:e + 1].copy()
            up[0, j] += h
            um[0, j] -= h
            Lp = np.sum(g[:, e:e + 1, :] * orc.dg_forward(D, up))
            Lm = np.sum(g[:, e:e + 1, :] * orc.dg_forward(D, um))
            fd_u[e, j] = (Lp - Lm) / (2 * h)
    assert normwise_rel(gu, fd_u) <= 1e-7
    # D entries: only output row (m, i) moves
    fd_D = np.empty_like(D)
    for m in range(3):
        for i in range(n):
            row = D[m, i].copy()
            gi = g[m, :, i]
            for j in range(n):
                rp, rm = row.copy(), row.copy()
                rp[j] += h
                rm[j] -= h
                fd_D[m, i, j] = (np.dot(gi, u @ rp) - np.dot(gi, u @ rm)) / (2 * h)
    assert normwise_rel(gD, fd_D) <= 1e-7


def test_autograd_function_and_gradcheck(orc, ops):
    from paper_1904_09538_amd.autograd import DGDiffFn
    D = _t(I.random_dmats(8), torch.float64).requires_grad_(True)
    u = _t(I.uniform_u(5, 8), torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(DGDiffFn.apply, (D, u), eps=1e-6, atol=1e-8)
    # needs_input_grad honoured
    u2 = _t(I.uniform_u(7, 8), torch.float64).requires_grad_(True)
    D2 = _t(I.random_dmats(8), torch.float64)
    DGDiffFn.apply(D2, u2).sum().backward()
    ru, _ = orc.dg_adjoint(D2.cpu().numpy(), u2.detach().cpu().numpy(), np.ones((3, 7, 8)))
    assert normwise_rel(u2.grad.cpu().numpy(), ru) <= 1e-12


def test_full_size_fp32_p4(orc, ops):
    """Forward + backward through the autograd Function at hex p=4, 2^19
    elements, FP32, g ~ N(0,1): all of grad_u and all 46,875 entries of
    grad_D against the FP64 oracle adjoint."""
    from paper_1904_09538_amd.autograd import DGDiffFn
    n, E = 125, 1 << 19
    D32 = I.gll_dmats(4).astype(np.float32)
    u32 = np.asarray(I.uniform_u(E, n), dtype=np.float32)
    g32 = np.asarray(I.normal_g(3, E, n), dtype=np.float32)
    D = torch.from_numpy(D32).cuda().requires_grad_(True)
    u = torch.from_numpy(u32).cuda().requires_grad_(True)
    out = DGDiffFn.apply(D, u)
    out.backward(torch.from_numpy(g32).cuda())
    torch.cuda.synchronize()
    # every entry of grad_u and of grad_D against the oracle adjoint
    ru, rD = orc.dg_adjoint(D32.astype(np.float64), u32.astype(np.float64), g32.astype(np.float64))
    assert normwise_rel(u.grad.double().cpu().numpy(), ru) <= 1e-5
    assert normwise_rel(D.grad.double().cpu().numpy(), rD) <= 1e-5


def test_backward_deterministic(ops):
    D = _t(I.random_dmats(125), torch.float32)
    u = _t(I.uniform_u(20000, 125), torch.float32)
    g = _t(I.normal_g(3, 20000, 125), torch.float32)
    a = ops.dgdiff_backward(D, u, g)
    b = ops.dgdiff_backward(D, u, g)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
