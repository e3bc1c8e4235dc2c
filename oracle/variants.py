"""Outputs of the program variants' work-removed twins — TEST INFRASTRUCTURE ONLY.

The work-removal transformation (Section "Measurement Workload Synthesis by
Work Removal Transformation", Algorithm "remove work") keeps a kernel's loops
and its global accesses to a chosen set of arrays, adds every kept load to one
per-work-item sum, and stores that sum where the kernel stored its result (if
that store is kept) or into a destination of one value per work-item.  What a
twin writes therefore follows from which elements each work-item of the
variant loads; this module writes that down per variant from the variants'
documented schedules (work-item (l0, l1) of work-group (g0, g1); loads past
the last element or grid point read the last one).  On small-integer inputs
every such sum is exact in FP32, so the GPU must match bit for bit.

keep bits: 1 = first input (u, or a), 2 = second input (D, or b), 4 = result.
The full variants compute the plain operations of the oracle (dg_forward,
stencil5, matmul) and are checked against those.
"""
from __future__ import annotations

import numpy as np

KEEP_IN0, KEEP_IN1, KEEP_OUT = 1, 2, 4


def shape(kind, n, nunit=0):
    """(gx, gy, threads) of a variant launch."""
    if kind in ("mm_pf", "mm_nopf"):
        return n // 16, n // 16, 256
    if kind.startswith("dg_"):
        return -(-n // 16), nunit // 16, 256
    if kind == "fd16":
        g = -(-n // 14)
        return g, g, 256
    g = -(-n // 16)
    return g, g, 324


def _dest(kind, n, nunit, per_item):
    """Scatter per-work-item sums per_item(g0, g1, l0, l1) into the destination."""
    gx, gy, T = shape(kind, n, nunit)
    L = 18 if kind == "fd18" else 16
    t = np.arange(T)
    l0, l1 = t % L, t // L
    out = np.empty(gx * gy * T, dtype=np.float64)
    for g1 in range(gy):
        for g0 in range(gx):
            w = g1 * gx + g0
            out[w * T:(w + 1) * T] = per_item(g0, g1, l0, l1)
    return out


def twin(kind, keep, n, in0=None, in1=None, nunit=0, nmat=0, ld_res=0):
    """What the twin of `kind` keeping `keep` writes.  Returns (dest, result):
    dest the per-work-item array (None when the result store is kept), result
    the result array with NaN where nothing is written (None otherwise).  DG
    inputs in the variant's own layout (u [nelem][nunit], or [nunit][nelem]
    for dg_pfdmt); stencil u [n+2][ld_u]."""
    k0, k1, ko = bool(keep & KEEP_IN0), bool(keep & KEEP_IN1), bool(keep & KEEP_OUT)
    a = None if in0 is None else np.asarray(in0, dtype=np.float64)
    b = None if in1 is None else np.asarray(in1, dtype=np.float64)
    if kind in ("mm_pf", "mm_nopf"):
        idx = np.arange(n)
        if kind == "mm_pf":
            # a[i][16 ko + l0] with l0 = j % 16; b[16 ko + l1][j] with l1 = i % 16
            sa = np.stack([a[:, idx % 16 == r].sum(axis=1) for r in range(16)], axis=1) if k0 else None
            sb = np.stack([b[idx % 16 == r, :].sum(axis=0) for r in range(16)], axis=0) if k1 else None
            val = np.zeros((n, n))
            if k0:
                val += sa[:, idx % 16]
            if k1:
                val += sb[idx % 16, :]
        else:
            val = np.zeros((n, n))
            if k0:
                val += a.sum(axis=1)[:, None]
            if k1:
                val += b.sum(axis=0)[None, :]
        if ko:
            return None, val
        return _dest(kind, n, 0, lambda g0, g1, l0, l1: val[16 * g1 + l1, 16 * g0 + l0]), None
    if kind.startswith("dg_"):
        E, nu, M = n, nunit, nmat
        tr = kind == "dg_pfdmt"
        U = None if a is None else (a.T if tr else a)          # U[k][j]
        kc = lambda k: np.minimum(k, E - 1)
        rowD = None if b is None else b.sum(axis=2)              # [m][i]
        if kind in ("dg_nopf", "dg_pfdm", "dg_pfdmt"):
            # per operator m the sum gains the u row of the work-item's element
            # (all j) and, from D, the row i (untiled) or the columns j = l0
            # mod 16 of row i (the D tile loads of the staged variants)
            def per_m(k, i):
                s = np.zeros((M,) + np.shape(k))
                for m in range(M):
                    if k0:
                        s[m] += U[kc(k)].sum(axis=-1)
                    if k1:
                        if kind == "dg_nopf":
                            s[m] += rowD[m][i]
                        else:
                            l0 = np.asarray(k) % 16
                            s[m] += np.array([b[m, ii, jj::16].sum() for ii, jj in
                                              zip(np.ravel(i), np.ravel(np.broadcast_to(l0, np.shape(i))))]
                                             ).reshape(np.shape(i))
                return np.cumsum(s, axis=0)
            if ko:
                kk, ii = np.meshgrid(np.arange(E), np.arange(nu), indexing="ij")
                s = per_m(kk, ii)                                 # [m][k][i]
                return None, (np.transpose(s, (0, 2, 1)) if tr else s)
            return _dest(kind, n, nu, lambda g0, g1, l0, l1: per_m(16 * g0 + l0, 16 * g1 + l1)[-1]), None
        # dg_pfu: u tile loads u[min(16 g0 + l1, E - 1)][16 jo + l0] over jo,
        # D loads D[m][i][j] over all j and m; the final sum is stored per m
        def final(g0, g1, l0, l1):
            s = np.zeros(np.shape(l0), dtype=np.float64)
            if k0:
                kf = kc(16 * g0 + l1)
                s += np.array([U[kk, ll::16].sum() for kk, ll in zip(np.ravel(kf), np.ravel(l0))]
                              ).reshape(np.shape(l0))
            if k1:
                s += rowD.sum(axis=0)[16 * g1 + l1]
            return s
        if ko:
            res = np.empty((M, E, nu))
            kk, ii = np.meshgrid(np.arange(E), np.arange(nu), indexing="ij")
            v = final(kk // 16, ii // 16, kk % 16, ii % 16)
            res[:] = v[None]
            return None, res
        return _dest(kind, n, nu, final), None
    # stencils: each work-item loads u[min(B g1 + l1, n + 1)][min(B g0 + l0, n + 1)]
    B = 16 if kind == "fd18" else 14
    if ko:
        res = np.full((n, ld_res), np.nan)
        res[:, :n] = a[:n, :n] if k0 else 0.0
        return None, res
    def item(g0, g1, l0, l1):
        if not k0:
            return np.zeros(np.shape(l0))
        return a[np.minimum(B * g1 + l1, n + 1), np.minimum(B * g0 + l0, n + 1)]
    return _dest(kind, n, 0, item), None
