/*
 * FP64 CPU oracle for the DG differentiation kernel family, its companion
 * calibration kernels and the low-precision encodings.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source with the HIP path.
 *
 * Every routine is the plain definition of what it computes, written as
 * straight loops, single-threaded, in FP64 with ascending-index summation, so
 * that it can be checked against the paper by eye:
 *   - DG differentiation: the kernel of the paper's DG evaluation case
 *     (Section "DG Differentiation"): res[m,k,i] = sum_j diff_mat[m,i,j] u[k,j].
 *   - Its adjoint (both partial derivatives of <g, res>).
 *   - The five-point stencil of Section "Finite Differences":
 *     res[i,j] = u[i,j+1] + u[i+1,j] - 4 u[i+1,j+1] + u[i+1,j+2] + u[i+2,j+1].
 *   - Square matrix multiplication c[i,j] = sum_k a[i,k] b[k,j]
 *     (Section "Kernel Creation and Transformation").
 *   - BF16 and OCP FP8-E4M3FN round-to-nearest-even encodings written from
 *     the format definitions (sign, exponent, mantissa, bias), not from any
 *     bit trick, so that the GPU encoder's bit manipulation is checked against
 *     an independent derivation.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <fenv.h>

/* ---------------------------------------------------------------- DG forward */

/* out[m][e][i] = sum_{j=0}^{nunit-1} D[m][i][j] * u[e][j]
   D: [nmat][nunit][nunit], u: [nelem][nunit], out: [nmat][nelem][nunit]. */
void orc_dg_forward(int nmat, int64_t nelem, int nunit,
                    const double* D, const double* u, double* out) {
    for (int m = 0; m < nmat; ++m)
        for (int64_t e = 0; e < nelem; ++e)
            for (int i = 0; i < nunit; ++i) {
                double acc = 0.0;
                for (int j = 0; j < nunit; ++j)
                    acc += D[((int64_t)m * nunit + i) * nunit + j] * u[e * nunit + j];
                out[((int64_t)m * nelem + e) * nunit + i] = acc;
            }
}

/* Same definition evaluated only for the listed elements (for sampled parity at
   full size).  out: [nsel][nmat][nunit]. */
void orc_dg_forward_select(int nmat, int nunit, const double* D, const double* u,
                           int64_t nsel, const int64_t* elems, double* out) {
    for (int64_t s = 0; s < nsel; ++s) {
        const double* ue = u + elems[s] * nunit;
        for (int m = 0; m < nmat; ++m)
            for (int i = 0; i < nunit; ++i) {
                double acc = 0.0;
                for (int j = 0; j < nunit; ++j)
                    acc += D[((int64_t)m * nunit + i) * nunit + j] * ue[j];
                out[(s * nmat + m) * nunit + i] = acc;
            }
    }
}

/* Mixed-order form: element e has order[e] (1..7), n_e = (order+1)^3 nodes,
   node data at u_packed[off[e] .. off[e]+n_e); its own operator set
   D_sets + dset_off[order] laid out [3][n_e][n_e];
   out_packed[m * total + off[e] + i] = sum_j D^{(p_e)}[m][i][j] u_packed[off[e]+j]. */
void orc_dg_batched(int nmat, int64_t nelem, const int8_t* order, const int64_t* off,
                    const double* D_sets, const int64_t* dset_off,
                    const double* u_packed, double* out_packed) {
    int64_t total = off[nelem];
    for (int64_t e = 0; e < nelem; ++e) {
        int p = order[e];
        int n = (p + 1) * (p + 1) * (p + 1);
        const double* D = D_sets + dset_off[p];
        const double* ue = u_packed + off[e];
        for (int m = 0; m < nmat; ++m)
            for (int i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j)
                    acc += D[((int64_t)m * n + i) * n + j] * ue[j];
                out_packed[(int64_t)m * total + off[e] + i] = acc;
            }
    }
}

/* ---------------------------------------------------------------- DG adjoint */

/* For L = sum_{m,e,i} g[m][e][i] * out[m][e][i] with out as in orc_dg_forward:
     grad_u[e][j]    = dL/du[e][j]    = sum_m sum_i D[m][i][j] g[m][e][i]
     grad_D[m][i][j] = dL/dD[m][i][j] = sum_e g[m][e][i] u[e][j]
   Either output pointer may be NULL. */
void orc_dg_adjoint(int nmat, int64_t nelem, int nunit,
                    const double* D, const double* u, const double* g,
                    double* grad_u, double* grad_D) {
    if (grad_u) {
        for (int64_t e = 0; e < nelem; ++e)
            for (int j = 0; j < nunit; ++j) {
                double acc = 0.0;
                for (int m = 0; m < nmat; ++m)
                    for (int i = 0; i < nunit; ++i)
                        acc += D[((int64_t)m * nunit + i) * nunit + j] *
                               g[((int64_t)m * nelem + e) * nunit + i];
                grad_u[e * nunit + j] = acc;
            }
    }
    if (grad_D) {
        for (int m = 0; m < nmat; ++m)
            for (int i = 0; i < nunit; ++i)
                for (int j = 0; j < nunit; ++j) {
                    double acc = 0.0;
                    for (int64_t e = 0; e < nelem; ++e)
                        acc += g[((int64_t)m * nelem + e) * nunit + i] * u[e * nunit + j];
                    grad_D[((int64_t)m * nunit + i) * nunit + j] = acc;
                }
    }
}

/* grad_D entries (m, i, j) listed in mm/ii/jj: sum_e g[m][e][i] u[e][j]. */
void orc_dg_adjoint_D_select(int nmat, int64_t nelem, int nunit, const double* u, const double* g,
                             int64_t cnt, const int64_t* mm, const int64_t* ii, const int64_t* jj,
                             double* out) {
    (void)nmat;
    for (int64_t s = 0; s < cnt; ++s) {
        double acc = 0.0;
        for (int64_t e = 0; e < nelem; ++e)
            acc += g[(mm[s] * nelem + e) * nunit + ii[s]] * u[e * nunit + jj[s]];
        out[s] = acc;
    }
}

/* ---------------------------------------------------------------- stencil */

/* res[i][j] = u[i][j+1] + u[i+1][j] - 4 u[i+1][j+1] + u[i+1][j+2] + u[i+2][j+1],
   0 <= i, j < n; u is (n+2) rows with leading dimension ld_u >= n+2. */
void orc_stencil5(int64_t n, const double* u, int64_t ld_u, double* res, int64_t ld_res) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            res[i * ld_res + j] = u[i * ld_u + (j + 1)] + u[(i + 1) * ld_u + j]
                                - 4.0 * u[(i + 1) * ld_u + (j + 1)]
                                + u[(i + 1) * ld_u + (j + 2)] + u[(i + 2) * ld_u + (j + 1)];
}

/* The same definition for a list of output points (i, j). */
void orc_stencil5_select(int64_t n, const double* u, int64_t ld_u,
                         int64_t cnt, const int64_t* ii, const int64_t* jj, double* out) {
    (void)n;
    for (int64_t s = 0; s < cnt; ++s) {
        int64_t i = ii[s], j = jj[s];
        out[s] = u[i * ld_u + (j + 1)] + u[(i + 1) * ld_u + j]
               - 4.0 * u[(i + 1) * ld_u + (j + 1)]
               + u[(i + 1) * ld_u + (j + 2)] + u[(i + 2) * ld_u + (j + 1)];
    }
}

/* ---------------------------------------------------------------- matmul */

/* c[i][j] = sum_k a[i][k] b[k][j], square n x n, row-major. */
void orc_matmul(int64_t n, const double* a, const double* b, double* c) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += a[i * n + k] * b[k * n + j];
            c[i * n + j] = acc;
        }
}

/* Selected entries c[ii[s]][jj[s]]. */
void orc_matmul_select(int64_t n, const double* a, const double* b,
                       int64_t cnt, const int64_t* ii, const int64_t* jj, double* out) {
    for (int64_t s = 0; s < cnt; ++s) {
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k)
            acc += a[ii[s] * n + k] * b[k * n + jj[s]];
        out[s] = acc;
    }
}

/* ---------------------------------------------------------------- encodings */

/* Round x to an integer multiple of the quantum q (a power of two), ties to
   even multiple.  x/q is exact because q is a power of two. */
static double rne_to_quantum(double x, double q) {
    int old = fegetround();
    fesetround(FE_TONEAREST);
    double r = nearbyint(x / q) * q;
    fesetround(old);
    return r;
}

/* BF16: 1 sign, 8 exponent (bias 127), 7 stored mantissa bits; the same
   exponent range as FP32, so its value set is every FP32 number whose low 16
   bits are zero.  Rounding: nearest, ties to even; overflow beyond the largest
   finite value (and its half-quantum) goes to infinity as in IEEE; NaN is kept
   and made quiet. */
uint16_t orc_bf16_encode(float xf) {
    uint32_t bits;
    memcpy(&bits, &xf, 4);
    uint16_t sign = (uint16_t)((bits >> 16) & 0x8000u);
    if (isnan(xf)) return (uint16_t)(sign | 0x7FC0u | ((bits >> 16) & 0x3Fu));
    double ax = fabs((double)xf);
    if (isinf(xf)) return (uint16_t)(sign | 0x7F80u);
    if (ax == 0.0) return sign;
    int e;
    frexp(ax, &e);                 /* ax = f * 2^e, f in [0.5, 1): unit in last place 2^(e-8) */
    double q = ldexp(1.0, e - 8);
    double qmin = ldexp(1.0, -133); /* subnormal spacing 2^-126 * 2^-7 */
    if (q < qmin) q = qmin;
    double r = rne_to_quantum(ax, q);
    if (r >= ldexp(1.0, 128)) return (uint16_t)(sign | 0x7F80u);
    float rf = (float)r;            /* exact: r has at most 8 significant bits */
    uint32_t rb;
    memcpy(&rb, &rf, 4);
    return (uint16_t)(sign | (rb >> 16));
}

float orc_bf16_decode(uint16_t h) {
    uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, 4);
    return f;
}

/* OCP OFP8 E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
   infinities, NaN = S.1111.111, largest finite 1.75 * 2^8 = 448, smallest
   normal 2^-6, subnormal spacing 2^-9.  Encoding: round to nearest, ties to
   even (subnormals included); magnitudes beyond 448 saturate to 448; NaN maps
   to NaN (sign kept); infinities saturate. */
double orc_e4m3_decode(uint8_t c) {
    int s = (c >> 7) & 1;
    int E = (c >> 3) & 0xF;
    int M = c & 7;
    double v;
    if (E == 0xF && M == 7) return s ? -NAN : NAN;
    if (E == 0) v = ldexp((double)M, -9);
    else v = ldexp(1.0 + M / 8.0, E - 7);
    return s ? -v : v;
}

uint8_t orc_e4m3_encode(double x) {
    uint8_t sign = signbit(x) ? 0x80 : 0x00;
    if (isnan(x)) return (uint8_t)(sign | 0x7F);
    double ax = fabs(x);
    if (ax >= 448.0) return (uint8_t)(sign | 0x7E);  /* saturate (covers +-inf) */
    if (ax == 0.0) return sign;
    double q;
    if (ax < ldexp(1.0, -6)) {
        q = ldexp(1.0, -9);                 /* subnormal range: fixed spacing */
    } else {
        int e;
        frexp(ax, &e);                      /* ax in [2^(e-1), 2^e) */
        q = ldexp(1.0, (e - 1) - 3);        /* 3 mantissa bits below the leading one */
    }
    double r = rne_to_quantum(ax, q);
    if (r > 448.0) r = 448.0;               /* rounding up past the top saturates */
    if (r == 0.0) return sign;
    /* find the code of r by its exponent and mantissa */
    if (r < ldexp(1.0, -6)) {
        int M = (int)(r / ldexp(1.0, -9));
        return (uint8_t)(sign | M);
    }
    int e;
    double f = frexp(r, &e);                /* r = f 2^e, f in [0.5,1) */
    int E = (e - 1) + 7;
    int M = (int)((2.0 * f - 1.0) * 8.0);
    return (uint8_t)(sign | (E << 3) | M);
}

/* Power-of-two scale that brings amax just inside the format maximum:
   s = 2^floor(log2(fmax / amax)), s = 1 when amax is 0 (or not finite); the
   exponent is capped at 127 so that s stays a finite FP32 number. */
double orc_pow2_scale(double amax, double fmax) {
    if (!(amax > 0.0) || isinf(amax)) return 1.0;
    double t = fmax / amax;
    int e;
    double f = frexp(t, &e);                /* t = f 2^e, f in [0.5,1): floor(log2 t) = e-1 */
    (void)f;
    if (e - 1 > 127) return ldexp(1.0, 127);
    return ldexp(1.0, e - 1);
}

/* Quantise a [rows][cols] FP32 matrix.
   to = 0: BF16, plain RNE cast, inverse scales all 1.
   to = 1: E4M3, q = RNE(x * s) with s a power of two chosen per row
           (per_row = 1) or for the whole matrix (per_row = 0); inv_scale[r] = 1/s.
   q is uint16 [rows][cols] for BF16 and uint8 [rows][cols] for E4M3. */
void orc_quantize(int to, int64_t rows, int64_t cols, int per_row,
                  const float* x, void* q, float* inv_scale) {
    if (to == 0) {
        uint16_t* qb = (uint16_t*)q;
        for (int64_t r = 0; r < rows; ++r) {
            for (int64_t c = 0; c < cols; ++c) qb[r * cols + c] = orc_bf16_encode(x[r * cols + c]);
            if (inv_scale && (per_row || r == 0)) inv_scale[per_row ? r : 0] = 1.0f;
        }
        return;
    }
    uint8_t* q8 = (uint8_t*)q;
    double whole = 0.0;
    if (!per_row)
        for (int64_t k = 0; k < rows * cols; ++k) {
            double a = fabs((double)x[k]);
            if (a > whole) whole = a;
        }
    for (int64_t r = 0; r < rows; ++r) {
        double amax = whole;
        if (per_row) {
            amax = 0.0;
            for (int64_t c = 0; c < cols; ++c) {
                double a = fabs((double)x[r * cols + c]);
                if (a > amax) amax = a;
            }
        }
        double s = orc_pow2_scale(amax, 448.0);
        for (int64_t c = 0; c < cols; ++c) q8[r * cols + c] = orc_e4m3_encode((double)x[r * cols + c] * s);
        if (per_row) inv_scale[r] = (float)(1.0 / s);
        else if (r == 0) inv_scale[0] = (float)(1.0 / s);
    }
}
