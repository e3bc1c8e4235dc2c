"""Seeded synthetic inputs for the DG differentiation family and its companion
kernels.

This module only *generates data*: it holds none of the arithmetic of the
operations being computed or modelled (the DG contraction, the stencil, the
matmul, quantisation, feature counting, the model fit).  Both the HIP path and
the FP64 CPU oracle are fed from here, so parity tests compare the two on the
very same arrays.

Seeds (fixed by convention so that every result can name its input):
  0 -> u (element data, U(-1,1))      1 -> random differentiation matrices
  2 -> batched element orders          3 -> upstream gradient g ~ N(0,1)
  4 -> held-out split of calibration   5 -> calibration measurement order
  6 -> stencil grid                    7 -> matmul operands

The differentiation matrices are the nodal DG operator on the hexahedron: the
1-D Gauss-Lobatto-Legendre (GLL) differentiation matrix placed into one slot of
a three-fold Kronecker product with identities (the paper's DG application,
Section "DG Differentiation", uses nmatrices = 3 such operators).  GLL nodes are
x_0 = -1, x_p = 1 and the interior roots of P_p'; the 1-D matrix is the
classical Lagrange-derivative closed form
    D1[i][j] = P_p(x_i) / (P_p(x_j) (x_i - x_j))   (i != j)
    D1[0][0] = -p(p+1)/4,  D1[p][p] = +p(p+1)/4,  other diagonal entries 0.
"""
from __future__ import annotations

import numpy as np

SEED_U = 0
SEED_RANDOM_D = 1
SEED_ORDERS = 2
SEED_G = 3
SEED_SPLIT = 4
SEED_MEASURE_ORDER = 5
SEED_STENCIL = 6
SEED_MATMUL = 7

MAX_ORDER = 7


def nunit_of_order(p: int) -> int:
    """Nodes of a hexahedral element of polynomial order p: (p+1)^3."""
    return (p + 1) ** 3


def _legendre_and_derivs(p: int, x: np.ndarray):
    """P_p(x) and P_p'(x) via Bonnet's three-term recurrence (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if p == 0:
        return p_prev, np.zeros_like(x)
    p_cur = x.copy()
    for k in range(1, p):
        p_next = ((2 * k + 1) * x * p_cur - k * p_prev) / (k + 1)
        p_prev, p_cur = p_cur, p_next
    # P_p' from (x^2 - 1) P_p' = p (x P_p - P_{p-1}); only used off the endpoints
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = p * (x * p_cur - p_prev) / (x * x - 1.0)
    return p_cur, dp


def gll_nodes(p: int) -> np.ndarray:
    """The p+1 Gauss-Lobatto-Legendre nodes on [-1, 1], ascending, FP64."""
    if p < 1:
        raise ValueError("GLL nodes need p >= 1")
    x = np.empty(p + 1, dtype=np.float64)
    x[0], x[p] = -1.0, 1.0
    if p >= 2:
        # Newton on P_p' for the interior nodes, started at Chebyshev-Lobatto points.
        t = -np.cos(np.pi * np.arange(1, p) / p)
        for _ in range(100):
            pp, dp = _legendre_and_derivs(p, t)
            # P_p'' from the Legendre ODE: (1-x^2) P'' = 2x P' - p(p+1) P
            d2p = (2.0 * t * dp - p * (p + 1) * pp) / (1.0 - t * t)
            step = dp / d2p
            t = t - step
            if np.max(np.abs(step)) < 1e-16:
                break
        x[1:p] = t
        # exact centro-symmetry of the node set
        x[:] = 0.5 * (x - x[::-1])
    return x


def gll_diff_1d(p: int) -> np.ndarray:
    """(p+1)x(p+1) GLL differentiation matrix, FP64 (closed form above)."""
    x = gll_nodes(p)
    pp, _ = _legendre_and_derivs(p, x)
    n = p + 1
    d = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            if i != j:
                d[i, j] = pp[i] / (pp[j] * (x[i] - x[j]))
    d[0, 0] = -p * (p + 1) / 4.0
    d[p, p] = p * (p + 1) / 4.0
    return d


def gll_dmats(p: int, nmat: int = 3) -> np.ndarray:
    """[nmat][n_u][n_u] FP64 operators D_m = kron with D1 in slot m (numpy kron
    convention: node j = (a*(p+1) + b)*(p+1) + c, a = axis 0 slowest)."""
    if not 1 <= nmat <= 3:
        raise ValueError("GLL Kronecker operators exist for nmat in 1..3")
    d1 = gll_diff_1d(p)
    eye = np.eye(p + 1)
    out = []
    for m in range(nmat):
        factors = [eye, eye, eye]
        factors[m] = d1
        out.append(np.kron(np.kron(factors[0], factors[1]), factors[2]))
    return np.ascontiguousarray(np.stack(out))


def random_dmats(nunit: int, nmat: int = 3, seed: int = SEED_RANDOM_D) -> np.ndarray:
    """[nmat][n_u][n_u] FP64 entries N(0, variance 1/n_u)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0 / np.sqrt(nunit), size=(nmat, nunit, nunit))


def uniform_u(nelem: int, nunit: int, seed: int = SEED_U) -> np.ndarray:
    """[nelem][n_u] FP64 element data U(-1,1)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(nelem, nunit))


def normal_g(nmat: int, nelem: int, nunit: int, seed: int = SEED_G) -> np.ndarray:
    """[nmat][nelem][n_u] FP64 upstream gradient N(0,1)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, size=(nmat, nelem, nunit))


def batched_orders(nelem: int, seed: int = SEED_ORDERS, max_order: int = MAX_ORDER) -> np.ndarray:
    """int8 [nelem] element orders p in 1..max_order drawn with P(p) ∝ 1/(p+1)."""
    ps = np.arange(1, max_order + 1)
    w = 1.0 / (ps + 1.0)
    rng = np.random.default_rng(seed)
    return rng.choice(ps, size=nelem, p=w / w.sum()).astype(np.int8)


def batched_offsets(order: np.ndarray) -> np.ndarray:
    """int64 [nelem+1] exclusive prefix sum of (p_e+1)^3 (ragged element-major layout)."""
    nu = (order.astype(np.int64) + 1) ** 3
    off = np.zeros(len(order) + 1, dtype=np.int64)
    np.cumsum(nu, out=off[1:])
    return off


def stencil_grid(n: int, seed: int = SEED_STENCIL) -> np.ndarray:
    """[(n+2)][(n+2)] FP64 U(-1,1) input of the five-point stencil."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n + 2, n + 2))


def matmul_operands(n: int, seed: int = SEED_MATMUL):
    """Two [n][n] FP64 N(0,1) matrices."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, n)), rng.normal(size=(n, n))


def as_f32(x: np.ndarray) -> np.ndarray:
    """Round once to FP32 (RNE).  Parity runs feed the FP64 oracle these FP32
    values widened back to FP64, so the error measures the kernel only."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))
