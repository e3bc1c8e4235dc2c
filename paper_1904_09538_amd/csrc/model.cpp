// Calibration and prediction of the black-box linear performance model
// (paper, Sections "Computing Model Parameters" and "Predicting Cost"), FP64.
//
// Fit.  Given feature rows f_k and measured times t_k, find p minimising the
// Euclidean norm of the residual t - F p.  With relative scaling (the paper's
// scale_features_by_output, used in all of its examples) row k is divided by
// t_k and the target becomes 1, so the fit minimises relative error.  The
// paper hands the (possibly nonlinear) problem to Levenberg-Marquardt; for the
// linear model the minimiser is reached directly:
//   1. equilibrate columns to unit 2-norm (features span ~20 orders of
//      magnitude: launches vs. bytes),
//   2. one-sided Jacobi SVD of the scaled matrix (never the normal equations,
//      whose condition number is the square),
//   3. minimum-norm solution over singular values > 1e-12 * sigma_max,
//   4. undo the column scaling.
// Reported: the residual norm at the solution (logged by the paper as a model
// adequacy signal), numerical rank and condition number of the kept part.
//
// Non-negative fit (DG_FIT_NONNEG).  The paper judges a model whose fit needs
// negative weights inconsistent with the notion of cost (Section
// "Assumptions and Limitations": interpretability).  With this flag the linear fit is the
// non-negative least-squares minimiser, by the active-set method of Lawson and
// Hanson (Solving Least Squares Problems, 1974, ch. 23) on the same row-scaled,
// column-equilibrated system; the overlap fit keeps its cost parameters in the
// non-negative orthant by an active-set projected Levenberg-Marquardt step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace dg {
namespace {

constexpr double kRcond = 1e-12;

// One-sided Jacobi: A (m x n, row-major, m >= n or not) is orthogonalised in
// place by column rotations; V accumulates them.  On exit the columns of A are
// U*Sigma.
void jacobi_svd(std::vector<double>& A, int m, int n, std::vector<double>& V,
                std::vector<double>& sv) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double app = 0, aqq = 0, apq = 0;
                for (int k = 0; k < m; ++k) {
                    const double x = A[(size_t)k * n + p], y = A[(size_t)k * n + q];
                    app += x * x;
                    aqq += y * y;
                    apq += x * y;
                }
                if (app == 0.0 || aqq == 0.0) continue;
                const double c_ = std::fabs(apq) / std::sqrt(app * aqq);
                if (c_ > off) off = c_;
                if (c_ < 1e-15) continue;
                const double zeta = (aqq - app) / (2.0 * apq);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int k = 0; k < m; ++k) {
                    const double x = A[(size_t)k * n + p], y = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * x - sn * y;
                    A[(size_t)k * n + q] = sn * x + cs * y;
                }
                for (int k = 0; k < n; ++k) {
                    const double x = V[(size_t)k * n + p], y = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * x - sn * y;
                    V[(size_t)k * n + q] = sn * x + cs * y;
                }
            }
        if (off < 1e-15) break;
    }
    sv.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int k = 0; k < m; ++k) s += A[(size_t)k * n + j] * A[(size_t)k * n + j];
        sv[j] = std::sqrt(s);
    }
}

// Minimum-norm least-squares solve of A x = b (A m x n) by the Jacobi SVD
// above, with column equilibration; returns the numerical rank.
int lstsq(std::vector<double> A, int m, int n, const std::vector<double>& b, std::vector<double>& x) {
    std::vector<double> cs(n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int k = 0; k < m; ++k) s += A[(size_t)k * n + j] * A[(size_t)k * n + j];
        cs[j] = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
        for (int k = 0; k < m; ++k) A[(size_t)k * n + j] *= cs[j];
    }
    std::vector<double> V, sv;
    jacobi_svd(A, m, n, V, sv);
    double smax = 0;
    for (double v : sv) smax = std::max(smax, v);
    x.assign(n, 0.0);
    int r = 0;
    for (int j = 0; j < n; ++j) {
        if (!(sv[j] > kRcond * smax) || smax == 0) continue;
        ++r;
        double utb = 0;
        for (int k = 0; k < m; ++k) utb += A[(size_t)k * n + j] * b[k];
        const double coef = utb / (sv[j] * sv[j]);
        for (int i = 0; i < n; ++i) x[i] += V[(size_t)i * n + j] * coef;
    }
    for (int j = 0; j < n; ++j) x[j] *= cs[j];
    return r;
}

// Non-negative least squares min ||A x - b||, x >= 0 (A m x n, columns
// already equilibrated), by Lawson-Hanson: grow the passive set by the
// variable of largest positive dual w = A^T (b - A x); solve the unconstrained
// problem on the passive columns; if that leaves the orthant, step back to its
// boundary along the segment and drop the variables that reached zero.
void nnls(const std::vector<double>& A, int m, int n, const std::vector<double>& b,
          std::vector<double>& x) {
    x.assign(n, 0.0);
    std::vector<char> passive(n, 0);
    std::vector<double> w(n), s(n);
    double anorm = 0;
    for (double v : A) anorm = std::max(anorm, std::fabs(v));
    double bnorm = 0;
    for (double v : b) bnorm += v * v;
    const double tol = 1e-13 * std::max(m, n) * std::max(anorm, 1.0) * std::sqrt(std::max(bnorm, 1.0));
    auto dual = [&]() {
        std::vector<double> r(b);
        for (int k = 0; k < m; ++k)
            for (int j = 0; j < n; ++j) r[k] -= A[(size_t)k * n + j] * x[j];
        for (int j = 0; j < n; ++j) {
            double v = 0;
            for (int k = 0; k < m; ++k) v += A[(size_t)k * n + j] * r[k];
            w[j] = v;
        }
    };
    // solve on the passive columns (the rest held at zero)
    auto solve_passive = [&]() {
        std::vector<int> cols;
        for (int j = 0; j < n; ++j)
            if (passive[j]) cols.push_back(j);
        const int c = (int)cols.size();
        std::vector<double> Ap((size_t)m * c), y;
        for (int k = 0; k < m; ++k)
            for (int q = 0; q < c; ++q) Ap[(size_t)k * c + q] = A[(size_t)k * n + cols[q]];
        lstsq(Ap, m, c, b, y);
        std::fill(s.begin(), s.end(), 0.0);
        for (int q = 0; q < c; ++q) s[cols[q]] = y[q];
    };
    for (int outer = 0; outer < 3 * n + 10; ++outer) {
        dual();
        int t = -1;
        double wmax = tol;
        for (int j = 0; j < n; ++j)
            if (!passive[j] && w[j] > wmax) {
                wmax = w[j];
                t = j;
            }
        if (t < 0) break;
        passive[t] = 1;
        for (int inner = 0; inner < 3 * n + 10; ++inner) {
            solve_passive();
            bool feasible = true;
            for (int j = 0; j < n; ++j)
                if (passive[j] && s[j] <= 0) feasible = false;
            if (feasible) {
                x = s;
                break;
            }
            double alpha = 1.0;
            int hit = -1;
            for (int j = 0; j < n; ++j)
                if (passive[j] && s[j] <= 0) {
                    const double a = x[j] / (x[j] - s[j]);
                    if (hit < 0 || a < alpha) {
                        alpha = a;
                        hit = j;
                    }
                }
            for (int j = 0; j < n; ++j) x[j] += alpha * (s[j] - x[j]);
            x[hit] = 0.0;  // the blocking variable lands on the boundary exactly
            for (int j = 0; j < n; ++j)
                if (passive[j] && x[j] <= 0.0) {
                    passive[j] = 0;
                    x[j] = 0.0;
                }
        }
    }
}

// Overlap model (paper, Sections "Modeling Operation Overlap" and "Models
// Demonstrated"): features are split into overhead (group 0), global memory
// (group 1) and on-chip (group 2) costs,
//     g = c_ovh + c_g s(c_g - c_o) + c_o s(c_o - c_g),   s(x) = (tanh(e x) + 1)/2,
// which, with s(-x) = 1 - s(x), equals c_ovh + c_o + (c_g - c_o) s(c_g - c_o).
struct Overlap {
    int rows, cols;
    const double* F;
    const int32_t* group;
    void costs(const double* p, int k, double* co, double* cg, double* cc) const {
        double a = 0, b = 0, c = 0;
        for (int j = 0; j < cols; ++j) {
            const double v = p[j] * F[(size_t)k * cols + j];
            if (group[j] == 0) a += v;
            else if (group[j] == 1) b += v;
            else c += v;
        }
        *co = a;
        *cg = b;
        *cc = c;
    }
    double eval(const double* p, double edge, int k) const {
        double co, cg, cc;
        costs(p, k, &co, &cg, &cc);
        const double d = cg - cc;
        return co + cc + d * 0.5 * (std::tanh(edge * d) + 1.0);
    }
};

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" {

dg_status perf_model_fit(int32_t rows, int32_t cols, const double* F, const double* t,
                         int32_t flags, double* p, double* resid, int32_t* rank, double* cond) {
    set_error("");
    const bool relative = flags & DG_FIT_RELATIVE, nonneg = flags & DG_FIT_NONNEG;
    if (flags & ~(DG_FIT_RELATIVE | DG_FIT_NONNEG)) return fail(DG_EINVAL, "perf_model_fit: unknown flags");
    if (rows <= 0 || cols <= 0 || !F || !t || !p) return fail(DG_EINVAL, "perf_model_fit: bad arguments");
    for (int64_t k = 0; k < (int64_t)rows * cols; ++k)
        if (!std::isfinite(F[k])) return fail(DG_EINVAL, "perf_model_fit: non-finite feature");
    for (int k = 0; k < rows; ++k) {
        if (!std::isfinite(t[k])) return fail(DG_EINVAL, "perf_model_fit: non-finite time");
        if (relative && !(t[k] > 0)) return fail(DG_EINVAL, "perf_model_fit: relative fit needs t > 0");
    }
    // row-scaled system A p = b
    std::vector<double> A((size_t)rows * cols), b(rows);
    for (int k = 0; k < rows; ++k) {
        const double w = relative ? 1.0 / t[k] : 1.0;
        for (int j = 0; j < cols; ++j) A[(size_t)k * cols + j] = F[(size_t)k * cols + j] * w;
        b[k] = relative ? 1.0 : t[k];
    }
    const std::vector<double> A0 = A;
    // column equilibration
    std::vector<double> cs(cols, 0.0);
    for (int j = 0; j < cols; ++j) {
        double s = 0;
        for (int k = 0; k < rows; ++k) s += A[(size_t)k * cols + j] * A[(size_t)k * cols + j];
        cs[j] = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
        for (int k = 0; k < rows; ++k) A[(size_t)k * cols + j] *= cs[j];
    }
    std::vector<double> V, sv;
    jacobi_svd(A, rows, cols, V, sv);
    double smax = 0;
    for (double s : sv) smax = std::max(smax, s);
    // y = V * diag(1/s) * U^T b, with U^T b = (A_rot^T b) / s for kept columns
    std::vector<double> y(cols, 0.0);
    int r = 0;
    double smin_kept = 0;
    for (int j = 0; j < cols; ++j) {
        if (!(sv[j] > kRcond * smax) || smax == 0) continue;
        ++r;
        smin_kept = (r == 1) ? sv[j] : std::min(smin_kept, sv[j]);
        double utb = 0;
        for (int k = 0; k < rows; ++k) utb += A[(size_t)k * cols + j] * b[k];
        utb /= sv[j];  // column j of A_rot is u_j * s_j
        const double coef = utb / sv[j];
        for (int i = 0; i < cols; ++i) y[i] += V[(size_t)i * cols + j] * coef;
    }
    bool any_negative = false;
    for (int j = 0; j < cols; ++j) any_negative |= y[j] < 0;
    if (nonneg && any_negative) {
        // A still holds the rotated columns; rebuild the equilibrated matrix
        std::vector<double> Ae((size_t)rows * cols);
        for (int k = 0; k < rows; ++k)
            for (int j = 0; j < cols; ++j) Ae[(size_t)k * cols + j] = A0[(size_t)k * cols + j] * cs[j];
        nnls(Ae, rows, cols, b, y);
    }
    for (int j = 0; j < cols; ++j) p[j] = y[j] * cs[j];
    if (resid) {
        double s = 0;
        for (int k = 0; k < rows; ++k) {
            double fp = 0;
            for (int j = 0; j < cols; ++j) fp += A0[(size_t)k * cols + j] * p[j];
            s += (b[k] - fp) * (b[k] - fp);
        }
        *resid = std::sqrt(s);
    }
    if (rank) *rank = r;
    if (cond) *cond = r ? smax / smin_kept : INFINITY;
    return DG_OK;
}

dg_status perf_model_predict_overlap(int32_t rows, int32_t cols, const double* F,
                                     const int32_t* group, const double* p, double edge,
                                     double* t_out) {
    set_error("");
    if (rows < 0 || cols <= 0 || (rows > 0 && (!F || !group || !p || !t_out)))
        return fail(DG_EINVAL, "perf_model_predict_overlap: bad arguments");
    Overlap M{rows, cols, F, group};
    for (int k = 0; k < rows; ++k) t_out[k] = M.eval(p, edge, k);
    return DG_OK;
}

dg_status perf_model_fit_overlap(int32_t rows, int32_t cols, const double* F, const int32_t* group,
                                 const double* t, int32_t flags, double* p, double* edge,
                                 double* resid, int32_t* iters) {
    set_error("");
    const bool relative = flags & DG_FIT_RELATIVE, nonneg = flags & DG_FIT_NONNEG;
    if (flags & ~(DG_FIT_RELATIVE | DG_FIT_NONNEG))
        return fail(DG_EINVAL, "perf_model_fit_overlap: unknown flags");
    if (rows <= 0 || cols <= 0 || !F || !group || !t || !p || !edge)
        return fail(DG_EINVAL, "perf_model_fit_overlap: bad arguments");
    for (int j = 0; j < cols; ++j)
        if (group[j] < 0 || group[j] > 2) return fail(DG_EINVAL, "perf_model_fit_overlap: group");
    for (int64_t k = 0; k < (int64_t)rows * cols; ++k)
        if (!std::isfinite(F[k])) return fail(DG_EINVAL, "perf_model_fit_overlap: non-finite feature");
    double tmed = 0;
    {
        std::vector<double> ts(t, t + rows);
        for (double v : ts)
            if (!(v > 0) || !std::isfinite(v)) return fail(DG_EINVAL, "perf_model_fit_overlap: t must be > 0");
        std::nth_element(ts.begin(), ts.begin() + rows / 2, ts.end());
        tmed = ts[rows / 2];
    }
    Overlap M{rows, cols, F, group};
    const int np = cols + 1;  // parameters + edge
    // Unknowns are scaled so that every one is O(1): p_j = q_j * sc_j with
    // sc_j = 1 / ||f_j / t||, edge = q_e / tmed.
    std::vector<double> sc(np);
    for (int j = 0; j < cols; ++j) {
        double s = 0;
        for (int k = 0; k < rows; ++k) {
            const double a = F[(size_t)k * cols + j] / (relative ? t[k] : 1.0);
            s += a * a;
        }
        sc[j] = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
    }
    sc[cols] = 1.0 / tmed;
    std::vector<double> q(np);
    // start: the caller's p if any entry is non-zero (e.g. a linear fit,
    // magnitudes taken), else equal shares; edge = 5 / median(t)
    bool given = false;
    for (int j = 0; j < cols; ++j) given |= p[j] != 0.0;
    for (int j = 0; j < cols; ++j)
        q[j] = (given && sc[j] > 0) ? std::fabs(p[j]) / sc[j] : 1.0 / std::sqrt((double)cols);
    q[cols] = (*edge > 0) ? *edge * tmed : 5.0;

    auto residuals = [&](const std::vector<double>& qq, std::vector<double>& r) {
        std::vector<double> pp(cols);
        for (int j = 0; j < cols; ++j) pp[j] = qq[j] * sc[j];
        const double e = qq[cols] * sc[cols];
        double ss = 0;
        for (int k = 0; k < rows; ++k) {
            const double g = M.eval(pp.data(), e, k);
            r[k] = relative ? 1.0 - g / t[k] : t[k] - g;
            ss += r[k] * r[k];
        }
        return ss;
    };
    std::vector<double> r(rows), rn(rows), J((size_t)rows * np);
    double cost = residuals(q, r);
    double lambda = 1e-3;
    int it = 0;
    bool converged = false;
    for (; it < 500; ++it) {
        // Jacobian of the residual in the scaled unknowns
        std::vector<double> pp(cols);
        for (int j = 0; j < cols; ++j) pp[j] = q[j] * sc[j];
        const double e = q[cols] * sc[cols];
        for (int k = 0; k < rows; ++k) {
            double co, cg, cc;
            M.costs(pp.data(), k, &co, &cg, &cc);
            const double d = cg - cc;
            const double th = std::tanh(e * d);
            const double s1 = 0.5 * (th + 1.0);
            const double ds = 0.5 * e * (1.0 - th * th);  // s'(d)
            const double dg_dcg = s1 + d * ds, dg_dcc = 1.0 - s1 - d * ds;
            const double w = relative ? -1.0 / t[k] : -1.0;
            for (int j = 0; j < cols; ++j) {
                const double f = F[(size_t)k * cols + j];
                const double dg = group[j] == 0 ? f : group[j] == 1 ? f * dg_dcg : f * dg_dcc;
                J[(size_t)k * np + j] = w * dg * sc[j];
            }
            J[(size_t)k * np + cols] = w * (0.5 * d * d * (1.0 - th * th)) * sc[cols];
        }
        // Marquardt step: min || [J; sqrt(lambda) diag(|J_j|)] dq + [r; 0] ||
        std::vector<double> dn(np);
        for (int j = 0; j < np; ++j) {
            double s = 0;
            for (int k = 0; k < rows; ++k) s += J[(size_t)k * np + j] * J[(size_t)k * np + j];
            dn[j] = std::sqrt(s);
        }
        if (nonneg) {
            // a cost parameter at zero whose descent direction points out of
            // the orthant (gradient J^T r > 0 there) is held: its column is
            // cleared, so the damping row alone fixes its step to zero
            for (int j = 0; j < cols; ++j) {
                if (q[j] > 0) continue;
                double gj = 0;
                for (int k = 0; k < rows; ++k) gj += J[(size_t)k * np + j] * r[k];
                if (gj >= 0)
                    for (int k = 0; k < rows; ++k) J[(size_t)k * np + j] = 0.0;
            }
        }
        bool improved = false;
        for (int tries = 0; tries < 30 && !improved; ++tries) {
            std::vector<double> A((size_t)(rows + np) * np, 0.0), b(rows + np, 0.0);
            for (int k = 0; k < rows; ++k) {
                for (int j = 0; j < np; ++j) A[(size_t)k * np + j] = J[(size_t)k * np + j];
                b[k] = -r[k];
            }
            for (int j = 0; j < np; ++j) A[(size_t)(rows + j) * np + j] = std::sqrt(lambda) * (dn[j] > 0 ? dn[j] : 1.0);
            std::vector<double> dq;
            lstsq(A, rows + np, np, b, dq);
            std::vector<double> qn(np);
            for (int j = 0; j < np; ++j) qn[j] = q[j] + dq[j];
            if (qn[cols] <= 0) qn[cols] = q[cols] * 0.5;  // the edge stays positive
            if (nonneg)
                for (int j = 0; j < cols; ++j) qn[j] = std::max(qn[j], 0.0);
            const double cn = residuals(qn, rn);
            if (std::isfinite(cn) && cn < cost) {
                const double rel = (cost - cn) / std::max(cost, 1e-300);
                q = qn;
                r = rn;
                cost = cn;
                lambda = std::max(lambda / 3.0, 1e-12);
                improved = true;
                if (rel < 1e-12) converged = true;
            } else {
                lambda *= 4.0;
            }
        }
        if (!improved || converged) {
            ++it;
            break;
        }
    }
    for (int j = 0; j < cols; ++j) p[j] = q[j] * sc[j];
    *edge = q[cols] * sc[cols];
    if (resid) *resid = std::sqrt(cost);
    if (iters) *iters = it;
    return DG_OK;
}

dg_status perf_model_predict(int32_t rows, int32_t cols, const double* F, const double* p,
                             double* t_out) {
    set_error("");
    if (rows < 0 || cols <= 0 || (rows > 0 && (!F || !p || !t_out)))
        return fail(DG_EINVAL, "perf_model_predict: bad arguments");
    for (int k = 0; k < rows; ++k) {
        double s = 0;
        for (int j = 0; j < cols; ++j) s += F[(size_t)k * cols + j] * p[j];
        t_out[k] = s;
    }
    return DG_OK;
}

}  // extern "C"
