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

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" {

dg_status perf_model_fit(int32_t rows, int32_t cols, const double* F, const double* t,
                         int32_t relative, double* p, double* resid, int32_t* rank, double* cond) {
    set_error("");
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
