"""MI355X-native DG differentiation kernel family and black-box performance
model (after Stevens & Kloeckner, arXiv 1904.09538).

The compute path lives in libdgdiff.so (hand-written HIP for gfx950, C ABI in
include/dgdiff.h).  ``ops`` re-exports its thin Python binding; importing it
fails loudly when the library has not been built.
"""

__all__ = ["inputs", "ops"]


def __getattr__(name):
    if name == "ops":
        from . import _lib as ops
        return ops
    raise AttributeError(name)
