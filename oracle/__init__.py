"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path; the two meet only in
the seeded input generators, which hold none of the method's arithmetic.

Contents
  * ctypes wrappers over ``liboracle.so`` (plain C, FP64, single-threaded):
    DG differentiation and its adjoint, the mixed-order form, the five-point
    stencil, square matmul, BF16 / FP8-E4M3FN encoders and decoders, the
    quantiser with power-of-two scales, and the brute-force feature enumerator.
  * ``model``: the least-squares calibration and prediction of the paper's
    Sections "Computing Model Parameters" and "Predicting Cost", in FP64.
  * ``metrics``: error measures used by the parity tests.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = ctypes.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i8p = ctypes.POINTER(ctypes.c_int8)
_i64 = ctypes.c_int64
_i32 = ctypes.c_int


def _declare(L):
    L.orc_dg_forward.argtypes = [_i32, _i64, _i32, _dp, _dp, _dp]
    L.orc_dg_forward_select.argtypes = [_i32, _i32, _dp, _dp, _i64, _i64p, _dp]
    L.orc_dg_batched.argtypes = [_i32, _i64, _i8p, _i64p, _dp, _i64p, _dp, _dp]
    L.orc_dg_adjoint.argtypes = [_i32, _i64, _i32, _dp, _dp, _dp, ctypes.c_void_p, ctypes.c_void_p]
    L.orc_dg_adjoint_D_select.argtypes = [_i32, _i64, _i32, _dp, _dp, _i64, _i64p, _i64p, _i64p, _dp]
    L.orc_stencil5.argtypes = [_i64, _dp, _i64, _dp, _i64]
    L.orc_stencil5_select.argtypes = [_i64, _dp, _i64, _i64, _i64p, _i64p, _dp]
    L.orc_matmul.argtypes = [_i64, _dp, _dp, _dp]
    L.orc_matmul_select.argtypes = [_i64, _dp, _dp, _i64, _i64p, _i64p, _dp]
    L.orc_bf16_encode.argtypes = [ctypes.c_float]
    L.orc_bf16_encode.restype = ctypes.c_uint16
    L.orc_bf16_decode.argtypes = [ctypes.c_uint16]
    L.orc_bf16_decode.restype = ctypes.c_float
    L.orc_e4m3_encode.argtypes = [ctypes.c_double]
    L.orc_e4m3_encode.restype = ctypes.c_uint8
    L.orc_e4m3_decode.argtypes = [ctypes.c_uint8]
    L.orc_e4m3_decode.restype = ctypes.c_double
    L.orc_pow2_scale.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_pow2_scale.restype = ctypes.c_double
    L.orc_quantize.argtypes = [_i32, _i64, _i64, _i32, _fp, ctypes.c_void_p, _fp]
    L.orc_features.argtypes = [_i32, _i32, _i64, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i64, _i64p]
    L.orc_features.restype = _i32
    L.orc_ubench_features.argtypes = [_i32, _i32, _i64, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i64p]
    L.orc_ubench_features.restype = _i32
    L.orc_variant_features.argtypes = [_i32, _i64, _i32, _i32, _i32, _i32, _i64p]
    L.orc_variant_features.restype = _i32
    L.orc_count_triangle.argtypes = [_i64, _i64]
    L.orc_count_triangle.restype = _i64


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ DG family

def dg_forward(D, u):
    """out[m][e][i] = sum_j D[m][i][j] u[e][j]  (FP64)."""
    D, u = _f64(D), _f64(u)
    nmat, nunit, _ = D.shape
    nelem = u.shape[0]
    assert u.shape == (nelem, nunit)
    out = np.empty((nmat, nelem, nunit), dtype=np.float64)
    lib().orc_dg_forward(nmat, nelem, nunit, _ptr(D), _ptr(u), _ptr(out))
    return out


def dg_forward_select(D, u, elems):
    """Forward for the listed elements only; returns [nsel][nmat][nunit]."""
    D, u = _f64(D), _f64(u)
    nmat, nunit, _ = D.shape
    el = np.ascontiguousarray(elems, dtype=np.int64)
    assert el.min(initial=0) >= 0 and el.max(initial=0) < u.shape[0]
    out = np.empty((len(el), nmat, nunit), dtype=np.float64)
    lib().orc_dg_forward_select(nmat, nunit, _ptr(D), _ptr(u), len(el), _ptr(el, _i64p), _ptr(out))
    return out


def dg_batched(order, offsets, D_sets, u_packed, nmat=3):
    """Mixed-order forward.  D_sets: dict p -> [nmat][(p+1)^3][(p+1)^3]."""
    order = np.ascontiguousarray(order, dtype=np.int8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nelem = len(order)
    flat, doff = [], np.zeros(9, dtype=np.int64)
    pos = 0
    for p in range(0, 9):
        doff[p] = pos
        if p in D_sets:
            a = _f64(D_sets[p]).ravel()
            flat.append(a)
            pos += a.size
    flat = np.ascontiguousarray(np.concatenate(flat)) if flat else np.zeros(1)
    u = _f64(u_packed)
    out = np.empty(nmat * int(off[-1]), dtype=np.float64)
    lib().orc_dg_batched(nmat, nelem, _ptr(order, _i8p), _ptr(off, _i64p), _ptr(flat),
                         _ptr(doff, _i64p), _ptr(u), _ptr(out))
    return out.reshape(nmat, -1)


def dg_adjoint(D, u, g, want_u=True, want_D=True):
    """(grad_u, grad_D) of L = <g, dg_forward(D, u)>  (FP64)."""
    D, u, g = _f64(D), _f64(u), _f64(g)
    nmat, nunit, _ = D.shape
    nelem = u.shape[0]
    assert g.shape == (nmat, nelem, nunit)
    gu = np.empty((nelem, nunit)) if want_u else None
    gD = np.empty((nmat, nunit, nunit)) if want_D else None
    lib().orc_dg_adjoint(nmat, nelem, nunit, _ptr(D), _ptr(u), _ptr(g),
                         gu.ctypes.data if gu is not None else None,
                         gD.ctypes.data if gD is not None else None)
    return gu, gD


def dg_adjoint_D_select(u, g, mm, ii, jj):
    """Listed entries of grad_D = sum_e g[m][e][i] u[e][j]."""
    u, g = _f64(u), _f64(g)
    nmat, nelem, nunit = g.shape
    mm, ii, jj = (np.ascontiguousarray(x, dtype=np.int64) for x in (mm, ii, jj))
    out = np.empty(len(mm))
    lib().orc_dg_adjoint_D_select(nmat, nelem, nunit, _ptr(u), _ptr(g), len(mm), _ptr(mm, _i64p),
                                  _ptr(ii, _i64p), _ptr(jj, _i64p), _ptr(out))
    return out


# ------------------------------------------------------------------ companions

def stencil5(u):
    """res[i][j] of the five-point stencil for an (n+2)x(n+2) input."""
    u = _f64(u)
    n = u.shape[0] - 2
    assert u.shape[1] >= n + 2
    res = np.empty((n, n))
    lib().orc_stencil5(n, _ptr(u), u.shape[1], _ptr(res), n)
    return res


def stencil5_select(u, ii, jj):
    u = _f64(u)
    n = u.shape[0] - 2
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    assert len(ii) == len(jj) and (ii.size == 0 or (ii.max() < n and jj.max() < n and min(ii.min(), jj.min()) >= 0))
    out = np.empty(len(ii))
    lib().orc_stencil5_select(n, _ptr(u), u.shape[1], len(ii), _ptr(ii, _i64p), _ptr(jj, _i64p), _ptr(out))
    return out


def matmul(a, b):
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    assert a.shape == (n, n) and b.shape == (n, n)
    c = np.empty((n, n))
    lib().orc_matmul(n, _ptr(a), _ptr(b), _ptr(c))
    return c


def matmul_select(a, b, ii, jj):
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    out = np.empty(len(ii))
    lib().orc_matmul_select(n, _ptr(a), _ptr(b), len(ii), _ptr(ii, _i64p), _ptr(jj, _i64p), _ptr(out))
    return out


# ------------------------------------------------------------------ feature counts

FEATURES = ["launch", "workgroups", "barrier_x_wg", "gld_dg_u", "gld_dg_u_l2", "gld_dg_d",
            "gst_dg_out", "gld_st_u", "gst_st_res", "gld_mm_ab", "gst_mm_c", "lds_bytes",
            "mfma_f64", "mfma_f32", "mfma_bf16", "mfma_fp8", "valu_f32", "valu_f64",
            "gld_dg_u_unal", "gst_dg_out_unal", "wave_tiles", "serial_steps", "lat_steps",
            "gld_ws", "gst_ws", "gld_idx", "gld_ub", "gst_ub", "gld_ub_strided", "dg_out_w32", "dg_out_w64",
            "stage_chain"]
KERNELS = {"dg": 0, "stencil": 1, "matmul": 2, "empty": 3, "bwd_u": 4, "bwd_d": 5, "quant": 6,
           "batched": 7, "batched_pool": 8}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}


def features(kernel, dtype, n0, nunit=0, nmat=0, elems_per_wave=0, waves=0, groups_per_cu=0,
             d_panels=0, flags=0, num_cu=0, workgroups=0):
    """Brute-force enumeration of one launch's operation counts (int64 array).
    quant: nunit = cols, nmat = per-row scales (0/1); batched: one order's
    share of workgroups work-groups."""
    out = np.zeros(len(FEATURES), dtype=np.int64)
    rc = lib().orc_features(KERNELS[kernel], DTYPES[dtype], int(n0), nunit, nmat, elems_per_wave,
                            waves, groups_per_cu, d_panels, flags, num_cu, int(workgroups),
                            _ptr(out, _i64p))
    if rc != 0:
        raise ValueError("unsupported descriptor")
    return out


UBENCH = {"stream": 0, "strided": 1, "fma": 2, "mfma": 3, "lds": 4, "barrier": 5, "overlap": 6,
          "twin_dg": 7, "twin_stencil": 8, "twin_matmul": 9, "tile_read": 10}


def ubench_features(kind, n, a=0, b=0, dtype="f32", tile=None, num_cu=0):
    """Brute-force enumeration of one measurement-kernel launch's counts."""
    t = tile or {}
    out = np.zeros(len(FEATURES), dtype=np.int64)
    rc = lib().orc_ubench_features(UBENCH[kind], DTYPES[dtype], int(n), int(a), int(b),
                                   t.get("elems_per_wave", 0), t.get("waves", 0), t.get("groups_per_cu", 0),
                                   t.get("d_panels", 0), t.get("flags", 0), int(num_cu), _ptr(out, _i64p))
    if rc != 0:
        raise ValueError("unsupported descriptor")
    return out


VARIANT_FEATURES = ["launch", "workgroups", "barrier_x_wg", "valu_f32_sg", "lds_sg", "gld_ub", "gst_ub",
                    "gld_ub_strided", "gld_mm_pf_a", "gld_mm_pf_b", "gld_mm_nopf_a", "gld_mm_nopf_b",
                    "gst_mm_c", "gld_dg_nopf_u", "gld_dg_dm", "gld_dg_upf_u", "gld_dg_dmpf_u",
                    "gld_dg_dmpf_dm", "gld_dg_dmpft_u", "gst_dg_nopf_res", "gst_dg_upf_res",
                    "gst_dg_dmpf_res", "gst_dg_dmpft_res", "gld_fd16_u", "gst_fd16_res", "gld_fd18_u",
                    "gst_fd18_res"]
VARIANTS = {"mm_pf": 0, "mm_nopf": 1, "dg_nopf": 2, "dg_pfu": 3, "dg_pfdm": 4, "dg_pfdmt": 5,
            "fd16": 6, "fd18": 7}


def variant_features(kind, n, nunit=0, nmat=0, work_removed=False, keep=0):
    """Brute-force walk of one program-variant launch's counts (int64 array,
    VARIANT_FEATURES order)."""
    out = np.zeros(len(VARIANT_FEATURES), dtype=np.int64)
    rc = lib().orc_variant_features(VARIANTS[kind], int(n), int(nunit), int(nmat), int(bool(work_removed)),
                                    int(keep), _ptr(out, _i64p))
    if rc != 0:
        raise ValueError("unsupported descriptor")
    return out


def count_triangle(p, n):
    """#{(i, j): p <= i < n, p <= j < i + 1} by enumeration."""
    return int(lib().orc_count_triangle(p, n))


# ------------------------------------------------------------------ encodings

def bf16_encode(x: float) -> int:
    return int(lib().orc_bf16_encode(float(x)))


def bf16_decode(h: int) -> float:
    return float(lib().orc_bf16_decode(int(h)))


def e4m3_encode(x: float) -> int:
    return int(lib().orc_e4m3_encode(float(x)))


def e4m3_decode(c: int) -> float:
    return float(lib().orc_e4m3_decode(int(c)))


def pow2_scale(amax: float, fmax: float = 448.0) -> float:
    return float(lib().orc_pow2_scale(float(amax), float(fmax)))


def quantize(x, to: str, per_row: bool):
    """Quantise an FP32 [rows][cols] matrix to 'bf16' or 'e4m3'.
    Returns (codes, inv_scale) with inv_scale of length rows (per_row) or 1."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = x.shape
    if to == "bf16":
        q = np.empty((rows, cols), dtype=np.uint16)
        t = 0
    elif to == "e4m3":
        q = np.empty((rows, cols), dtype=np.uint8)
        t = 1
    else:
        raise ValueError(to)
    inv = np.empty(rows if per_row else 1, dtype=np.float32)
    lib().orc_quantize(t, rows, cols, int(per_row), _ptr(x, _fp), q.ctypes.data, _ptr(inv, _fp))
    return q, inv


def bf16_decode_array(q):
    q = np.ascontiguousarray(q, dtype=np.uint16)
    return (q.astype(np.uint32) << 16).view(np.float32)


def e4m3_decode_array(q):
    table = np.array([e4m3_decode(c) for c in range(256)], dtype=np.float64)
    return table[np.asarray(q, dtype=np.uint8)]
