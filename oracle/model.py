"""Oracle for the paper's calibration and prediction steps (FP64, test only).

Calibration (Section "Computing Model Parameters"): with feature rows f_k and
measured times t_k, the parameters minimise the Euclidean norm of the residual
t - g(p).  For the linear model g_k(p) = f_k . p the least-squares minimiser is
reached exactly by a direct solve (the paper's Levenberg-Marquardt iteration
converges to the same point for a linear g).  With relative scaling
(the paper's ``scale_features_by_output``) every row is first divided by its
t_k and the right-hand side becomes 1.

Reading adopted where the paper is silent: the columns are equilibrated to unit
2-norm before the solve, singular values below 1e-12 * sigma_max are treated as
zero, and the minimum-norm solution is taken in the equilibrated coordinates;
the parameters are then un-scaled.  A library SVD least-squares routine
(numpy.linalg.lstsq) is the solve step.

Non-negative fit (``nonneg=True``): the paper's interpretability criterion
(Section "Assumptions and Limitations") rejects models whose fit needs negative
weights, since extra work never lowers cost.  Then, if the unconstrained
minimiser has a negative entry, the parameters are the non-negative
least-squares minimiser of the same row-scaled, equilibrated system, with a
library NNLS routine (scipy.optimize.nnls) as the solve step; the overlap fit
passes the bounds p >= 0 to its library nonlinear solver.

Prediction (Section "Predicting Cost"): t_hat = f . p for new feature rows.
Error statistics: the mean absolute percentage error and the geometric mean of
relative error (Section "Results").
"""
from __future__ import annotations

import numpy as np

RCOND = 1e-12


def fit(F, t, relative: bool = True, nonneg: bool = False):
    """Returns dict(p, resid, rank, cond, negative)."""
    F = np.array(F, dtype=np.float64, copy=True)
    t = np.array(t, dtype=np.float64, copy=True)
    if F.ndim != 2 or F.shape[0] == 0 or F.shape[0] != t.shape[0]:
        raise ValueError("bad shapes")
    if not (np.all(np.isfinite(F)) and np.all(np.isfinite(t))):
        raise ValueError("non-finite input")
    if relative:
        if np.any(t <= 0):
            raise ValueError("relative fit needs t > 0")
        A = F / t[:, None]
        b = np.ones_like(t)
    else:
        A, b = F, t
    norms = np.linalg.norm(A, axis=0)
    scale = np.where(norms > 0, 1.0 / np.where(norms > 0, norms, 1.0), 0.0)
    As = A * scale[None, :]
    y, _, rank, sv = np.linalg.lstsq(As, b, rcond=RCOND)
    if nonneg and np.any(y < 0):
        from scipy.optimize import nnls
        y = nnls(As, b, maxiter=50 * As.shape[1])[0]
    p = y * scale
    r = b - A @ p
    nz = sv[sv > RCOND * sv[0]] if sv.size and sv[0] > 0 else sv[:0]
    cond = float(nz[0] / nz[-1]) if nz.size else float("inf")
    return {"p": p, "resid": float(np.linalg.norm(r)), "rank": int(rank), "cond": cond,
            "negative": [int(k) for k in np.nonzero(p < 0)[0]]}


def predict(F, p):
    return np.asarray(F, dtype=np.float64) @ np.asarray(p, dtype=np.float64)


def mape(pred, meas):
    pred, meas = np.asarray(pred, np.float64), np.asarray(meas, np.float64)
    return float(np.mean(np.abs(pred - meas) / meas))


def geomean_rel_err(pred, meas, floor: float = 1e-6):
    pred, meas = np.asarray(pred, np.float64), np.asarray(meas, np.float64)
    r = np.maximum(np.abs(pred - meas) / meas, floor)
    return float(np.exp(np.mean(np.log(r))))


# ---------------------------------------------------------------- overlap model

def overlap_predict(F, group, p, edge):
    """Section "Modeling Operation Overlap": with c_x the cost of group x
    (0 overhead, 1 global memory, 2 on-chip),
    t = c_0 + c_1 s(c_1 - c_2) + c_2 s(c_2 - c_1),  s(x) = (tanh(edge x) + 1)/2."""
    F = np.asarray(F, dtype=np.float64)
    group = np.asarray(group)
    p = np.asarray(p, dtype=np.float64)
    c = [F[:, group == k] @ p[group == k] for k in (0, 1, 2)]

    def s(x):
        return (np.tanh(edge * x) + 1.0) / 2.0
    return c[0] + c[1] * s(c[1] - c[2]) + c[2] * s(c[2] - c[1])


def overlap_fit(F, t, group, p0, edge0, nonneg: bool = False):
    """Relative least squares of the overlap model with a library nonlinear
    least-squares routine (scipy.optimize.least_squares, trust region),
    unknowns scaled by their starting magnitudes; with nonneg the cost
    parameters are bounded below by zero."""
    from scipy.optimize import least_squares
    F = np.asarray(F, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    x0 = np.concatenate([np.abs(np.asarray(p0, dtype=np.float64)) if nonneg
                         else np.asarray(p0, dtype=np.float64), [edge0]])
    scale = np.where(np.abs(x0) > 0, np.abs(x0), 1.0)

    def res(z):
        x = z * scale
        return 1.0 - overlap_predict(F, group, x[:-1], x[-1]) / t
    lo = np.concatenate([np.zeros(x0.size - 1), [0.0]]) if nonneg else -np.inf
    sol = least_squares(res, np.ones_like(x0), bounds=(lo, np.inf), xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, max_nfev=20000)
    x = sol.x * scale
    return {"p": x[:-1], "edge": float(x[-1]), "resid": float(np.linalg.norm(sol.fun))}
