"""Error measures for parity tests (test infrastructure only).

The tolerances for the DG family are stated as maximum relative errors.  The
reading adopted is normwise over the whole output: max|y - y_ref| / max|y_ref|,
because elementwise relative error is unbounded where a derivative of random
data passes near zero.
"""
from __future__ import annotations

import numpy as np


def normwise_rel(y, ref) -> float:
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(y - ref))) if ref.size else 0.0
    if den == 0.0:
        return num
    return num / den


def elementwise_rel(y, ref, floor_frac: float = 1e-3) -> float:
    """Max elementwise relative error where |ref| >= floor_frac * max|ref|."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    thr = floor_frac * float(np.max(np.abs(ref)))
    m = np.abs(ref) >= thr
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(y[m] - ref[m]) / np.abs(ref[m])))
