"""ctypes binding of libdgdiff.so (argument marshalling only).

Every computation behind these functions runs in the library's HIP kernels;
this module only turns torch tensors into device pointers and sizes, passes
torch's current HIP stream, and raises on a non-OK status.  If the built
library is missing the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgdiff.so")

DG_OK, DG_EINVAL, DG_EUNSUPPORTED, DG_EHIP, DG_ENOMEM = range(5)
DG_F64, DG_F32, DG_BF16, DG_FP8E4M3 = range(4)
_STATUS = {0: "DG_OK", 1: "DG_EINVAL", 2: "DG_EUNSUPPORTED", 3: "DG_EHIP", 4: "DG_ENOMEM"}


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class dg_tile(ctypes.Structure):
    _fields_ = [("elems_per_wave", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("d_panels", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


DG_TILE_NT_STORE = 1
DG_TILE_FP8_NATIVE = 2
DG_TILE_BATCH_GEMM = 4
DG_TILE_LP_LDS_PANELS = 8
DG_TILE_QUANT_U = 16

(DG_K_DGDIFF, DG_K_STENCIL5, DG_K_MATMUL, DG_K_EMPTY, DG_K_BWD_U, DG_K_BWD_D, DG_K_QUANT,
 DG_K_BATCHED, DG_K_BATCHED_POOL) = range(9)
_KERNELS = {"dg": DG_K_DGDIFF, "stencil": DG_K_STENCIL5, "matmul": DG_K_MATMUL, "empty": DG_K_EMPTY,
            "bwd_u": DG_K_BWD_U, "bwd_d": DG_K_BWD_D, "quant": DG_K_QUANT, "batched": DG_K_BATCHED,
            "batched_pool": DG_K_BATCHED_POOL}


class perf_kernel_desc(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n0", ctypes.c_int64),
                ("nunit", ctypes.c_int32), ("nmat", ctypes.c_int32), ("tile", dg_tile),
                ("num_cu", ctypes.c_int32), ("workgroups", ctypes.c_int64)]


class dg_ubench_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64),
                ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("tile", dg_tile), ("num_cu", ctypes.c_int32)]


UBENCH = {"stream": 0, "strided": 1, "fma": 2, "mfma": 3, "lds": 4, "barrier": 5, "overlap": 6,
          "twin_dg": 7, "twin_stencil": 8, "twin_matmul": 9, "tile_read": 10}

class dg_variant_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int64), ("nunit", ctypes.c_int32),
                ("nmat", ctypes.c_int32), ("ld_u", ctypes.c_int64), ("ld_res", ctypes.c_int64),
                ("work_removed", ctypes.c_int32), ("keep", ctypes.c_int32)]


VARIANTS = {"mm_pf": 0, "mm_nopf": 1, "dg_nopf": 2, "dg_pfu": 3, "dg_pfdm": 4, "dg_pfdmt": 5,
            "fd16": 6, "fd18": 7}
DG_V_KEEP_IN0, DG_V_KEEP_IN1, DG_V_KEEP_OUT = 1, 2, 4

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def _declare(L):
    L.dg_last_error.restype = ctypes.c_char_p
    L.dg_last_error.argtypes = []
    L.dgdiff_apply.restype = _i32
    L.dgdiff_apply.argtypes = [_i32, _i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(dg_tile), _vp]
    L.dgdiff_backward_workspace.restype = ctypes.c_size_t
    L.dgdiff_backward_workspace.argtypes = [_i32, _i32, _i64, _i32]
    L.dgdiff_backward.restype = _i32
    L.dgdiff_backward.argtypes = [_i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                  ctypes.c_size_t, _vp]
    L.dgdiff_backward_noalloc.restype = _i32
    L.dgdiff_backward_noalloc.argtypes = [_i32, _i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
    L.dgdiff_quantize.restype = _i32
    L.dgdiff_quantize.argtypes = [_i32, _i64, _i64, _i32, _vp, _vp, _vp, _vp]
    L.dgdiff_plan_create.restype = _i32
    L.dgdiff_plan_create.argtypes = [_i64, _vp, _i32, _vp, _vp, _vp, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_void_p)]
    L.dgdiff_plan_total_nodes.restype = _i64
    L.dgdiff_plan_total_nodes.argtypes = [_vp]
    L.dgdiff_plan_info.restype = _i32
    L.dgdiff_plan_info.argtypes = [_vp, _i32, ctypes.POINTER(dg_tile), ctypes.POINTER(_i64),
                                   ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]
    L.dgdiff_apply_batched.restype = _i32
    L.dgdiff_apply_batched.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.dgdiff_plan_destroy.restype = None
    L.dgdiff_plan_destroy.argtypes = [_vp]
    L.dg_empty_launch.restype = _i32
    L.dg_empty_launch.argtypes = [_i64, _vp]
    L.perf_feature_count.restype = _i32
    L.perf_feature_name.restype = ctypes.c_char_p
    L.perf_feature_name.argtypes = [_i32]
    L.perf_features_count.restype = _i32
    L.perf_features_count.argtypes = [ctypes.POINTER(perf_kernel_desc), ctypes.POINTER(ctypes.c_int64)]
    L.dgdiff_resolve_tile.restype = _i32
    L.dgdiff_resolve_tile.argtypes = [_i32, _i32, _i64, _i32, ctypes.POINTER(dg_tile)]
    L.dg_ubench_run.restype = _i32
    L.dg_ubench_run.argtypes = [ctypes.POINTER(dg_ubench_desc), ctypes.POINTER(ctypes.c_void_p), _vp, _vp]
    L.perf_ubench_count.restype = _i32
    L.dg_variant_shape.restype = _i32
    L.dg_variant_shape.argtypes = [ctypes.POINTER(dg_variant_desc), ctypes.POINTER(_i64), ctypes.POINTER(_i32)]
    L.dg_variant_run.restype = _i32
    L.dg_variant_run.argtypes = [ctypes.POINTER(dg_variant_desc), _vp, _vp, _vp, _vp]
    L.perf_variant_feature_count.restype = _i32
    L.perf_variant_feature_count.argtypes = []
    L.perf_variant_feature_name.restype = ctypes.c_char_p
    L.perf_variant_feature_name.argtypes = [_i32]
    L.perf_variant_count.restype = _i32
    L.perf_variant_count.argtypes = [ctypes.POINTER(dg_variant_desc), ctypes.POINTER(ctypes.c_int64)]
    L.perf_ubench_count.argtypes = [ctypes.POINTER(dg_ubench_desc), ctypes.POINTER(ctypes.c_int64)]
    L.dgdiff_resolve_backward.restype = _i32
    L.dgdiff_resolve_backward.argtypes = [_i32, _i32, _i64, _i32, ctypes.POINTER(dg_tile),
                                          ctypes.POINTER(dg_tile)]
    _dp = ctypes.POINTER(ctypes.c_double)
    L.perf_model_fit.restype = _i32
    L.perf_model_fit.argtypes = [_i32, _i32, _dp, _dp, _i32, _dp, _dp, ctypes.POINTER(_i32), _dp]
    L.perf_model_fit_overlap.restype = _i32
    L.perf_model_fit_overlap.argtypes = [_i32, _i32, _dp, ctypes.POINTER(_i32), _dp, _i32, _dp, _dp,
                                         _dp, ctypes.POINTER(_i32)]
    L.perf_model_predict_overlap.restype = _i32
    L.perf_model_predict_overlap.argtypes = [_i32, _i32, _dp, ctypes.POINTER(_i32), _dp,
                                             ctypes.c_double, _dp]
    L.perf_model_predict.restype = _i32
    L.perf_model_predict.argtypes = [_i32, _i32, _dp, _dp, _dp]
    L.stencil5_apply.restype = _i32
    L.stencil5_apply.argtypes = [_i32, _i64, _vp, _i64, _vp, _i64, _vp]
    L.matmul_apply.restype = _i32
    L.matmul_apply.argtypes = [_i32, _i64, _vp, _vp, _vp, _vp]


def check(status: int):
    if status != DG_OK:
        raise DGError(status, lib().dg_last_error().decode())


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return DG_F64
    if t == torch.float32:
        return DG_F32
    if t == torch.bfloat16:
        return DG_BF16
    if t == torch.float8_e4m3fn:
        return DG_FP8E4M3
    raise TypeError(f"unsupported dtype {t}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_tile(tile):
    if tile is None:
        return None
    if isinstance(tile, dg_tile):
        return ctypes.byref(tile)
    t = dg_tile(*[int(tile.get(k, 0)) for k in ("elems_per_wave", "waves", "groups_per_cu",
                                                 "d_panels", "flags")])
    return ctypes.byref(t)


def dgdiff_apply(D, u, out=None, inv_sD=None, inv_su=None, tile=None, out_dtype=None, stream=None):
    """out[m][e][i] = inv_sD[m] inv_su[e] sum_j D[m][i][j] u[e][j] on the GPU.

    D: [nmat][nunit][nunit], u: [nelem][nunit] (same dtype, except that with
    DG_TILE_QUANT_U in tile's flags D is BF16 and u FP32, rounded to BF16 in
    the kernel); returns out [nmat][nelem][nunit] (FP32 for BF16/FP8 inputs)."""
    nmat, nunit, nunit2 = D.shape
    nelem = u.shape[0]
    if nunit2 != nunit or u.shape[1:] != (nunit,):
        raise ValueError("shape mismatch")
    flags = tile.flags if isinstance(tile, dg_tile) else int((tile or {}).get("flags", 0))
    if flags & DG_TILE_QUANT_U:
        if D.dtype != torch.bfloat16 or u.dtype != torch.float32:
            raise TypeError("DG_TILE_QUANT_U: D BF16, u FP32")
    elif D.dtype != u.dtype:
        raise TypeError("D and u must share a dtype")
    in_t = _dtype_code(D.dtype)
    if out_dtype is None:
        out_dtype = D.dtype if D.dtype in (torch.float32, torch.float64) else torch.float32
    if out is None:
        out = torch.empty((nmat, nelem, nunit), dtype=out_dtype, device=u.device)
    check(lib().dgdiff_apply(in_t, _dtype_code(out.dtype), nmat, nelem, nunit, _ptr(D), _ptr(u),
                             _ptr(out), _ptr(inv_sD), _ptr(inv_su), make_tile(tile), _stream(stream)))
    return out


def stencil5_apply(u, res=None, n=None, stream=None):
    """Five-point stencil of an (n+2) x ld_u grid (leading dimension = u.stride(0));
    returns res [n][ld_res] (a fresh [n][n] tensor unless res is given)."""
    if u.dim() != 2 or u.stride(1) != 1:
        raise ValueError("u must be 2-D with unit column stride")
    if n is None:
        n = u.shape[0] - 2
    if u.shape[0] < n + 2 or u.shape[1] < n + 2:
        raise ValueError("u must hold (n+2) x (n+2) values")
    if res is None:
        res = torch.empty((n, n), dtype=u.dtype, device=u.device)
    if res.dim() != 2 or res.stride(1) != 1 or res.shape[0] < n or res.shape[1] < n:
        raise ValueError("res must be 2-D [>=n][>=n] with unit column stride")
    check(lib().stencil5_apply(_dtype_code(u.dtype), n, ctypes.c_void_p(u.data_ptr()), u.stride(0),
                               ctypes.c_void_p(res.data_ptr()), res.stride(0), _stream(stream)))
    return res


def matmul_apply(a, b, c=None, stream=None):
    """c = a @ b for square FP32 matrices on the GPU."""
    n = a.shape[0]
    if a.shape != (n, n) or b.shape != (n, n):
        raise ValueError("square matrices expected")
    if c is None:
        c = torch.empty((n, n), dtype=a.dtype, device=a.device)
    check(lib().matmul_apply(_dtype_code(a.dtype), n, _ptr(a), _ptr(b), _ptr(c), _stream(stream)))
    return c


def dgdiff_quantize(x, to, per_row=True, stream=None):
    """Quantise an FP32 [rows][cols] tensor to BF16 (torch.bfloat16) or FP8
    E4M3FN (torch.float8_e4m3fn) with power-of-two scales; returns (q, inv_scale)."""
    if x.dtype != torch.float32 or x.dim() != 2:
        raise TypeError("x must be a 2-D float32 tensor")
    rows, cols = x.shape
    if to in ("bf16", torch.bfloat16):
        q = torch.empty((rows, cols), dtype=torch.bfloat16, device=x.device)
        code = DG_BF16
    elif to in ("e4m3", "fp8", torch.float8_e4m3fn):
        q = torch.empty((rows, cols), dtype=torch.float8_e4m3fn, device=x.device)
        code = DG_FP8E4M3
    else:
        raise ValueError(to)
    inv = torch.empty(rows if per_row else 1, dtype=torch.float32, device=x.device)
    check(lib().dgdiff_quantize(code, rows, cols, int(per_row), _ptr(x), _ptr(q), _ptr(inv),
                                _stream(stream)))
    return q, inv


def dgdiff_backward(D, u, g, want_u=True, want_D=True, stream=None):
    """(grad_u, grad_D) of L with dL/dout = g, on the GPU (FP32 or FP64)."""
    nmat, nunit, _ = D.shape
    nelem = u.shape[0]
    if g.shape != (nmat, nelem, nunit):
        raise ValueError("g must be [nmat][nelem][nunit]")
    if not (D.dtype == u.dtype == g.dtype):
        raise TypeError("D, u, g must share a dtype")
    t = _dtype_code(u.dtype)
    gu = torch.empty_like(u) if want_u else None
    gD = torch.empty_like(D) if want_D else None
    nbytes = lib().dgdiff_backward_workspace(t, nmat, nelem, nunit) if want_D else 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device=u.device) if nbytes else None
    check(lib().dgdiff_backward(t, nmat, nelem, nunit, _ptr(D), _ptr(u), _ptr(g), _ptr(gu), _ptr(gD),
                                _ptr(ws), nbytes, _stream(stream)))
    return gu, gD


def dgdiff_backward_noalloc(D, u, g, want_u=True, want_D=True, stream=None):
    """dgdiff_backward through the entry point that allocates nothing (its
    grad_D partials use the library's fixed per-device scratch)."""
    nmat, nunit, _ = D.shape
    nelem = u.shape[0]
    if g.shape != (nmat, nelem, nunit):
        raise ValueError("g must be [nmat][nelem][nunit]")
    if not (D.dtype == u.dtype == g.dtype):
        raise TypeError("D, u, g must share a dtype")
    t = _dtype_code(u.dtype)
    gu = torch.empty_like(u) if want_u else None
    gD = torch.empty_like(D) if want_D else None
    check(lib().dgdiff_backward_noalloc(t, nmat, nelem, nunit, _ptr(D), _ptr(u), _ptr(g), _ptr(gu),
                                        _ptr(gD), _stream(stream)))
    return gu, gD


# ------------------------------------------------------------------ performance model

_DT = {"f64": DG_F64, "f32": DG_F32, "bf16": DG_BF16, "fp8": DG_FP8E4M3}


def feature_names():
    L = lib()
    return [L.perf_feature_name(k).decode() for k in range(L.perf_feature_count())]


def perf_features_count(kernel, dtype, n0, nunit=0, nmat=0, tile=None, num_cu=0, workgroups=0):
    """Exact operation counts of one launch (numpy int64 array, feature_names() order).
    kernel: dg, stencil, matmul, empty, bwd_u, bwd_d, quant, batched, batched_pool."""
    import numpy as np
    L = lib()
    d = perf_kernel_desc()
    d.kernel = _KERNELS[kernel]
    d.dtype = _DT[dtype]
    d.n0 = int(n0)
    d.nunit = int(nunit)
    d.nmat = int(nmat)
    if tile is not None:
        t = tile if isinstance(tile, dg_tile) else dg_tile(
            *[int(tile.get(k, 0)) for k in ("elems_per_wave", "waves", "groups_per_cu", "d_panels", "flags")])
        d.tile = t
    d.num_cu = int(num_cu)
    d.workgroups = int(workgroups)
    out = np.zeros(L.perf_feature_count(), dtype=np.int64)
    check(L.perf_features_count(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def _ub_desc(kind, n, a=0, b=0, dtype="f32", tile=None, num_cu=0):
    d = dg_ubench_desc()
    d.kind = UBENCH[kind]
    d.dtype = _DT[dtype]
    d.n = int(n)
    d.a = int(a)
    d.b = int(b)
    if tile is not None:
        d.tile = dg_tile(*[int(tile.get(k, 0)) for k in ("elems_per_wave", "waves", "groups_per_cu", "d_panels",
                                                       "flags")])
    d.num_cu = int(num_cu)
    return d


def dg_ubench_run(kind, n, inputs, out, a=0, b=0, dtype="f32", tile=None, stream=None):
    """Launch a measurement kernel (dg_ubench_run): inputs a list of device
    tensors, out a device tensor."""
    d = _ub_desc(kind, n, a, b, dtype, tile)
    arr = (ctypes.c_void_p * max(1, len(inputs)))(*[t.data_ptr() for t in inputs])
    check(lib().dg_ubench_run(ctypes.byref(d), arr, _ptr(out), _stream(stream)))
    return out


def perf_ubench_count(kind, n, a=0, b=0, dtype="f32", tile=None, num_cu=0):
    """Counted features of one measurement-kernel launch (feature_names() order)."""
    import numpy as np
    d = _ub_desc(kind, n, a, b, dtype, tile, num_cu)
    out = np.zeros(lib().perf_feature_count(), dtype=np.int64)
    check(lib().perf_ubench_count(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def _v_desc(kind, n, nunit=0, nmat=0, ld_u=0, ld_res=0, work_removed=False, keep=0):
    return dg_variant_desc(VARIANTS[kind], int(n), int(nunit), int(nmat), int(ld_u), int(ld_res),
                           int(bool(work_removed)), int(keep))


def variant_feature_names():
    L = lib()
    return [L.perf_variant_feature_name(k).decode() for k in range(L.perf_variant_feature_count())]


def variant_shape(kind, n, nunit=0, nmat=0, ld_u=0, ld_res=0, work_removed=False, keep=0):
    """(work-groups, work-items per work-group) of a program-variant launch."""
    d = _v_desc(kind, n, nunit, nmat, ld_u, ld_res, work_removed, keep)
    wg, th = _i64(), _i32()
    check(lib().dg_variant_shape(ctypes.byref(d), ctypes.byref(wg), ctypes.byref(th)))
    return wg.value, th.value


def dg_variant_run(kind, n, in0, in1, out, nunit=0, nmat=0, ld_u=0, ld_res=0, work_removed=False, keep=0,
                   stream=None):
    """Launch a program variant (or its work-removed twin) on device tensors;
    in0 / in1 may be None where the twin does not read them."""
    d = _v_desc(kind, n, nunit, nmat, ld_u, ld_res, work_removed, keep)
    p0 = in0.data_ptr() if in0 is not None else None
    p1 = in1.data_ptr() if in1 is not None else None
    check(lib().dg_variant_run(ctypes.byref(d), p0, p1, _ptr(out), _stream(stream)))
    return out


def perf_variant_count(kind, n, nunit=0, nmat=0, ld_u=0, ld_res=0, work_removed=False, keep=0):
    """Counted features of one program-variant launch (variant_feature_names() order)."""
    import numpy as np
    d = _v_desc(kind, n, nunit, nmat, ld_u, ld_res, work_removed, keep)
    out = np.zeros(lib().perf_variant_feature_count(), dtype=np.int64)
    check(lib().perf_variant_count(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def _tile_dict(t):
    return {k: getattr(t, k) for k in ("elems_per_wave", "waves", "groups_per_cu", "d_panels", "flags")}


def resolve_backward(dtype, nmat, nelem, nunit):
    """Launch shapes of dgdiff_backward's grad_u and grad_D steps (GPU)."""
    tu, td = dg_tile(), dg_tile()
    check(lib().dgdiff_resolve_backward(_DT[dtype], nmat, nelem, nunit, ctypes.byref(tu), ctypes.byref(td)))
    return _tile_dict(tu), _tile_dict(td)


# features that measure a chain of dependent steps rather than an amount of work
CHAIN_FEATURES = ("serial_steps", "lat_steps", "stage_chain")


def batched_counts(plan_info, num_cu=0):
    """Counted features of a whole batched launch from dgdiff_plan_info's
    per-order report ({p: info}), one launch.  The orders' shares run side by
    side on the GPU, so their amounts of work (bytes, flops, work-groups,
    barriers) add, while the launch's chain of dependent steps is the longest
    of the orders' chains; the GEMM pool's fixed cost is added when an order
    runs GEMM tiles."""
    import numpy as np
    names = feature_names()
    chain = [names.index(k) for k in CHAIN_FEATURES]
    tot = None
    grid = sum(int(i["workgroups"]) for i in plan_info.values() if int(i["count"]) > 0)
    pool = False
    for p, i in plan_info.items():
        if int(i["count"]) == 0:
            continue
        c = np.asarray(perf_features_count("batched", "f32", int(i["count"]), (int(p) + 1) ** 3, 3, i["tile"],
                                           num_cu, int(i["workgroups"])))
        pool = pool or bool(int(i["tile"]["flags"]) & DG_TILE_BATCH_GEMM)
        if tot is None:
            tot = c.copy()
        else:
            longest = np.maximum(tot[chain], c[chain])
            tot = tot + c
            tot[chain] = longest
    if tot is None:
        return None
    if pool:
        tot = tot + np.asarray(perf_features_count("batched_pool", "f32", grid))
    tot[0] = 1
    return tot


def resolve_tile(dtype, nmat, nelem, nunit, tile=None):
    """Fill the open fields of a DG launch shape as dgdiff_apply would (GPU)."""
    t = dg_tile(*[int((tile or {}).get(k, 0)) for k in
                  ("elems_per_wave", "waves", "groups_per_cu", "d_panels", "flags")])
    check(lib().dgdiff_resolve_tile(_DT[dtype], nmat, nelem, nunit, ctypes.byref(t)))
    return {k: getattr(t, k) for k in ("elems_per_wave", "waves", "groups_per_cu", "d_panels", "flags")}


DG_FIT_RELATIVE = 1
DG_FIT_NONNEG = 2


def _fit_flags(relative, nonneg):
    return (DG_FIT_RELATIVE if relative else 0) | (DG_FIT_NONNEG if nonneg else 0)


def perf_model_fit(F, t, relative=True, nonneg=False):
    """FP64 least-squares fit (non-negative with nonneg=True); returns
    dict(p, resid, rank, cond, negative)."""
    import numpy as np
    F = np.ascontiguousarray(F, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    rows, cols = F.shape
    p = np.zeros(cols)
    resid = ctypes.c_double()
    rank = ctypes.c_int32()
    cond = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().perf_model_fit(rows, cols, F.ctypes.data_as(dp), t.ctypes.data_as(dp),
                               _fit_flags(relative, nonneg),
                               p.ctypes.data_as(dp), ctypes.byref(resid), ctypes.byref(rank),
                               ctypes.byref(cond)))
    return {"p": p, "resid": resid.value, "rank": rank.value, "cond": cond.value,
            "negative": [int(k) for k in np.nonzero(p < 0)[0]]}


def perf_model_predict(F, p):
    import numpy as np
    F = np.ascontiguousarray(F, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(F.shape[0])
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().perf_model_predict(F.shape[0], F.shape[1], F.ctypes.data_as(dp), p.ctypes.data_as(dp),
                                   out.ctypes.data_as(dp)))
    return out


def perf_model_fit_overlap(F, t, group, relative=True, p0=None, edge0=0.0, nonneg=False):
    """Nonlinear overlap model fit (LM, FP64; p >= 0 with nonneg=True);
    returns dict(p, edge, resid, iters)."""
    import numpy as np
    F = np.ascontiguousarray(F, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    g = np.ascontiguousarray(group, dtype=np.int32)
    rows, cols = F.shape
    p = np.zeros(cols) if p0 is None else np.array(p0, dtype=np.float64)
    edge = ctypes.c_double(edge0)
    resid = ctypes.c_double()
    iters = ctypes.c_int32()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().perf_model_fit_overlap(rows, cols, F.ctypes.data_as(dp),
                                       g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       t.ctypes.data_as(dp), _fit_flags(relative, nonneg),
                                       p.ctypes.data_as(dp),
                                       ctypes.byref(edge), ctypes.byref(resid), ctypes.byref(iters)))
    return {"p": p, "edge": edge.value, "resid": resid.value, "iters": iters.value}


def perf_model_predict_overlap(F, group, p, edge):
    import numpy as np
    F = np.ascontiguousarray(F, dtype=np.float64)
    g = np.ascontiguousarray(group, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(F.shape[0])
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().perf_model_predict_overlap(F.shape[0], F.shape[1], F.ctypes.data_as(dp),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           p.ctypes.data_as(dp), float(edge), out.ctypes.data_as(dp)))
    return out


def dg_empty_launch(workgroups, stream=None):
    check(lib().dg_empty_launch(int(workgroups), _stream(stream)))


class BatchedPlan:
    """Plan of the mixed-order persistent launch (owns device memory)."""

    def __init__(self, order, tiles=None, model=None, nmat=3):
        import numpy as np
        order = np.ascontiguousarray(order, dtype=np.int8)
        self.nelem = len(order)
        tarr = None
        if tiles is not None:
            tarr = (dg_tile * 8)()
            for p, t in tiles.items():
                tarr[p] = dg_tile(*[int(t.get(k, 0)) for k in
                                    ("elems_per_wave", "waves", "groups_per_cu", "d_panels", "flags")])
        cost = group = None
        edge = 0.0
        if model is not None:
            cost = np.ascontiguousarray(model["cost"], dtype=np.float64)
            if model.get("group") is not None:
                group = np.ascontiguousarray(model["group"], dtype=np.int32)
                edge = float(model.get("edge", 0.0))
        h = ctypes.c_void_p()
        check(lib().dgdiff_plan_create(self.nelem, order.ctypes.data_as(ctypes.c_void_p), nmat,
                                       ctypes.cast(tarr, ctypes.c_void_p) if tarr is not None else None,
                                       cost.ctypes.data_as(ctypes.c_void_p) if cost is not None else None,
                                       group.ctypes.data_as(ctypes.c_void_p) if group is not None else None,
                                       edge, ctypes.byref(h)))
        self._h = h
        self.total = lib().dgdiff_plan_total_nodes(h)

    def info(self, p):
        t = dg_tile()
        cnt = ctypes.c_int64()
        wgs = ctypes.c_int64()
        pred = ctypes.c_double()
        check(lib().dgdiff_plan_info(self._h, p, ctypes.byref(t), ctypes.byref(cnt), ctypes.byref(wgs),
                                     ctypes.byref(pred)))
        return {"tile": {k: getattr(t, k) for k in ("elems_per_wave", "waves", "groups_per_cu",
                                                    "d_panels", "flags")},
                "count": cnt.value, "workgroups": wgs.value, "predicted_s": pred.value}

    def apply(self, D_sets, u_packed, out=None, stream=None):
        """D_sets: dict p -> [3][n][n] float32 device tensor."""
        if out is None:
            out = torch.empty((3, self.total), dtype=torch.float32, device=u_packed.device)
        ptrs = (ctypes.c_void_p * 8)()
        for p, D in D_sets.items():
            ptrs[p] = D.data_ptr()
        check(lib().dgdiff_apply_batched(self._h, ctypes.cast(ptrs, ctypes.c_void_p), _ptr(u_packed),
                                         _ptr(out), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dgdiff_plan_destroy(h)
            self._h = None
