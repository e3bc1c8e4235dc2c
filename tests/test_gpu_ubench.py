"""GPU parity of the measurement kernels (dg_ubench_run) against their
definitions in the oracle (oracle/ubench.py), exact on small-integer and
dyadic inputs; the work-removed twins write every element their original
kernel writes (NaN-filled outputs, zero inputs: every written element is 0)."""
import numpy as np
import pytest
import torch

from oracle import ubench as U
from paper_1904_09538_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    from paper_1904_09538_amd import _lib
    _lib.lib()
    return _lib


def _ints(n, seed, lo=-8, hi=8):
    return torch.from_numpy(np.random.default_rng(seed).integers(lo, hi, n).astype(np.float32)).cuda()


@pytest.mark.parametrize("nin", [1, 2, 3, 4])
@pytest.mark.parametrize("n4", [1, 1000, 8192 * 256 + 5])
def test_stream(ops, nin, n4):
    ins = [_ints(4 * n4, k) for k in range(nin)]
    out = torch.full((4 * n4,), float("nan"), device="cuda")
    ops.dg_ubench_run("stream", n4, ins, out, a=nin)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.stream([x.cpu().numpy() for x in ins]))


@pytest.mark.parametrize("n,S", [(1, 1), (1000, 1), (1000, 33), (70000, 32)])
def test_strided(ops, n, S):
    x = _ints(n * S, 3)
    out = torch.empty(n, device="cuda")
    ops.dg_ubench_run("strided", n, [x], out, a=S)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.strided(x.cpu().numpy(), n, S))


@pytest.mark.parametrize("iters", [0, 1, 2, 3])
def test_fma(ops, iters):
    out = torch.empty(256 * 2, device="cuda")
    ops.dg_ubench_run("fma", 2, [], out, a=iters)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.fma(2, iters))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("iters", [0, 1, 3])
def test_mfma(ops, dtype, iters):
    out = torch.empty(256 * 3 * 4, device="cuda")
    ops.dg_ubench_run("mfma", 3, [], out, a=iters, dtype=dtype)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.mfma(3, iters, dtype))


@pytest.mark.parametrize("width", [1, 4])
@pytest.mark.parametrize("iters", [0, 1, 5, 64, 65])
def test_lds(ops, width, iters):
    x = _ints(2 * 256 * width, 5, -1000, 1000)
    out = torch.empty_like(x)
    ops.dg_ubench_run("lds", 2, [x], out, a=iters, b=width)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.lds(x.cpu().numpy(), 2, iters, width))


def test_barrier(ops):
    out = torch.empty(256 * 3, device="cuda")
    ops.dg_ubench_run("barrier", 3, [], out, a=10)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.barrier(3, 10))


@pytest.mark.parametrize("n4,m", [(300, 0), (300, 1), (1000, 5), (1000, 64), (4096, 7)])
def test_overlap(ops, n4, m):
    x = _ints(4 * n4, 9, -100, 100)
    out = torch.full((4 * n4,), float("nan"), device="cuda")
    ops.dg_ubench_run("overlap", n4, [x], out, a=m)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.overlap(x.cpu().numpy(), n4, m))


@pytest.mark.parametrize("p,E,tile", [
    (2, 100003, None), (3, 1 << 16, None), (3, 5001, dict(elems_per_wave=32, waves=4)),
    (4, 70000, None), (5, 4097, None), (1, 999, None), (4, 3000, dict(d_panels=8))])
def test_dg_twin_writes_every_output(ops, p, E, tile):
    n = I.nunit_of_order(p)
    t = ops.resolve_tile("f32", 3, E, n, tile)
    D = torch.zeros((3, n, n), device="cuda")
    u = torch.zeros((E, n), device="cuda")
    out = torch.full((3, E, n), float("nan"), device="cuda")
    ops.dg_ubench_run("twin_dg", E, [D, u], out, a=n, b=3, tile=t)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0      # NaN != 0: every element was written


@pytest.mark.parametrize("n", [1024, 4100])
def test_stencil_twin_writes_every_output(ops, n):
    ld = ((n + 2 + 63) // 64) * 64
    u = torch.zeros((n + 2, ld), device="cuda")
    res = torch.full((n, n), float("nan"), device="cuda")
    ops.dg_ubench_run("twin_stencil", n, [u], res, a=ld, b=n)
    torch.cuda.synchronize()
    assert torch.count_nonzero(res).item() == 0


@pytest.mark.parametrize("n", [1000, 1024])
def test_matmul_twin_writes_every_output(ops, n):
    a = torch.zeros((n, n), device="cuda")
    b = torch.zeros((n, n), device="cuda")
    c = torch.full((n, n), float("nan"), device="cuda")
    ops.dg_ubench_run("twin_matmul", n, [a, b], c)
    torch.cuda.synchronize()
    assert torch.count_nonzero(c).item() == 0


@pytest.mark.parametrize("pattern", [0, 1])
@pytest.mark.parametrize("n", [16, 64, 96])
def test_tile_read(ops, n, pattern):
    x = _ints(n * n, 11, -50, 50)
    out = torch.full((n * n,), float("nan"), device="cuda")
    ops.dg_ubench_run("tile_read", n, [x], out, a=pattern)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), U.tile_read(x.cpu().numpy(), n, pattern))
