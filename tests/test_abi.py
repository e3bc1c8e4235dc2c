"""Host-side checks of the C ABI (no GPU needed): every symbol the public
headers declare is exported, and argument validation fails before any launch."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"^\s*#[^\n]*", "", text, flags=re.M)   # preprocessor lines
        text = re.sub(r"typedef[^;]*;", "", text, flags=re.S)
        for m in re.finditer(r"\b([A-Za-z_]\w*)\s*\(", text):
            name = m.group(1)
            if name in ("if", "sizeof", "defined", "return"):
                continue
            names.add(name)
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_1904_09538_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.lib()


def test_headers_declare_something():
    names = _declared_functions()
    assert "dgdiff_apply" in names and "dg_last_error" in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _apply(L, in_t=1, out_t=1, nmat=3, nelem=10, nunit=64, D=1, u=2, out=3, sD=None, su=None):
    vp = ctypes.c_void_p
    return L.dgdiff_apply(in_t, out_t, nmat, nelem, nunit, vp(D) if D else None, vp(u) if u else None,
                          vp(out) if out else None, vp(sD) if sD else None, vp(su) if su else None,
                          None, None)


def test_validation_before_launch(L):
    from paper_1904_09538_amd import _lib as B
    assert _apply(L, nunit=0) == B.DG_EINVAL
    assert _apply(L, nelem=-1) == B.DG_EINVAL
    assert _apply(L, nmat=0) == B.DG_EINVAL
    assert _apply(L, nunit=513) == B.DG_EUNSUPPORTED
    assert _apply(L, nmat=9) == B.DG_EUNSUPPORTED
    assert _apply(L, in_t=2, out_t=0) == B.DG_EUNSUPPORTED
    assert _apply(L, in_t=7) == B.DG_EINVAL
    assert _apply(L, sD=16) == B.DG_EINVAL            # scales with FP32 input
    assert _apply(L, nelem=0, D=None, u=None, out=None) == B.DG_OK
    assert _apply(L, D=None) == B.DG_EINVAL
    # out overlapping u
    assert _apply(L, u=0x10000, out=0x10000 + 64) == B.DG_EINVAL
    assert b"overlap" in L.dg_last_error()


def test_fused_rounding_flag_validation(L):
    """DG_TILE_QUANT_U is refused for input other than BF16, before any launch."""
    from paper_1904_09538_amd import _lib as B
    t = B.dg_tile(0, 0, 0, 0, 16)
    vp = ctypes.c_void_p
    st = L.dgdiff_apply(B.DG_FP8E4M3, B.DG_F32, 3, 10, 64, vp(1), vp(2), vp(3), vp(4), vp(5),
                        ctypes.byref(t), None)
    assert st == B.DG_EINVAL
    st = L.dgdiff_apply(B.DG_F32, B.DG_F32, 3, 10, 64, vp(1), vp(2), vp(3), None, None, ctypes.byref(t), None)
    assert st == B.DG_EINVAL
