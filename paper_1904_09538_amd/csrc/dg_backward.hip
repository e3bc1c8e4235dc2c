// Adjoint of the DG differentiation operator, FP32 and FP64.  For a loss L with
// upstream gradient g[m][e][i] = dL/dout[m][e][i]:
//     grad_u[e][j]    = sum_m sum_i D[m][i][j] * g[m][e][i]
//     grad_D[m][i][j] = sum_e g[m][e][i] * u[e][j]
//
// grad_u runs on the forward's contraction kernel (dg_kernel.hpp) with the
// operator transposed and the g slabs as contraction segments.  When the
// nmat segments do not fit the register budget, each operator is applied in
// its own launch and the later launches accumulate (stream-ordered).
//
// grad_D is a GEMM C[(m,i)][j] = sum_e G_m^T[i][e] U[e][j] with a very long
// contraction (the element count).  It is split: work-group (tile, split)
// multiplies one 64x64 output tile over one contiguous element range on the
// matrix cores and writes an FP32/FP64 partial tile to the caller's
// workspace; a second kernel adds the partials of every entry in split order
// 0, 1, 2, ...  The result is therefore deterministic (no atomics, no
// order-dependent accumulation).
#include "dg_kernel.hpp"

namespace dg {
namespace {

using namespace kern;

// ------------------------------------------------------------------ grad_D

constexpr int GT = 64;      // output tile (rows i x cols j)
constexpr int GK = 16;      // elements per LDS chunk
constexpr int GLD = GT + 4; // LDS row stride

struct GdArgs {
    const void* g;
    const void* u;
    void* ws;             // [nsplit][nmat][nunit][nunit]
    int64_t nelem;
    int64_t split_len;    // elements per split (multiple of GK)
    int nmat;
    int nunit;
    int ntile;            // ceil(nunit / GT)
    int vec;              // 16-byte loads allowed
};

template <typename T>
__device__ inline void gd_load(const GdArgs& a, const T* __restrict__ gm, const T* __restrict__ u,
                               int64_t e0, int64_t e_hi, int i0, int j0, int t, T (&rg)[4],
                               T (&ru)[4]) {
    const int el = t >> 4;           // element within the chunk
    const int x = (t & 15) * 4;      // 4 consecutive nodes
    const int64_t e = e0 + el;
    const bool ev = e < e_hi;
    const int n = a.nunit;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        rg[q] = (ev && i0 + x + q < n) ? gm[e * n + i0 + x + q] : T(0);
        ru[q] = (ev && j0 + x + q < n) ? u[e * n + j0 + x + q] : T(0);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) grad_d_partial_kernel(GdArgs a) {
    typedef typename Mma<T>::acc_t acc_t;
    __shared__ __attribute__((aligned(16))) T lds[2][2][GK * GLD];  // [buf][g|u]
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int wr = wave >> 1, wc = wave & 1;
    const int tiles_per_m = a.ntile * a.ntile;
    const int m = blockIdx.x / tiles_per_m;
    const int ti = (blockIdx.x % tiles_per_m) / a.ntile;
    const int tj = blockIdx.x % a.ntile;
    const int i0 = ti * GT, j0 = tj * GT;
    const int64_t split = blockIdx.y;
    const int64_t e_lo = split * a.split_len;
    const int64_t e_hi = min<int64_t>(a.nelem, e_lo + a.split_len);
    const T* __restrict__ gm = static_cast<const T*>(a.g) + (int64_t)m * a.nelem * a.nunit;
    const T* __restrict__ u = static_cast<const T*>(a.u);

    acc_t acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = acc_t(T(0));

    const int64_t nchunk = e_hi > e_lo ? ceil_div(e_hi - e_lo, GK) : 0;
    T rg[4], ru[4];
    const int el_w = t >> 4, x_w = (t & 15) * 4;
    if (nchunk > 0) {
        gd_load<T>(a, gm, u, e_lo, e_hi, i0, j0, t, rg, ru);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lds[0][0][el_w * GLD + x_w + q] = rg[q];
            lds[0][1][el_w * GLD + x_w + q] = ru[q];
        }
    }
    __syncthreads();
    for (int64_t kc = 0; kc < nchunk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nchunk) gd_load<T>(a, gm, u, e_lo + (kc + 1) * GK, e_hi, i0, j0, t, rg, ru);
        const T* Gs = lds[buf][0];
        const T* Us = lds[buf][1];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int el = 4 * g + s;  // lane group g contracts elements 4g..4g+3 of the chunk
            T av[2], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) av[p] = Gs[el * GLD + wr * 32 + p * 16 + c];
#pragma unroll
            for (int q = 0; q < 2; ++q) bv[q] = Us[el * GLD + wc * 32 + q * 16 + c];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q) acc[p][q] = Mma<T>::step(av[p], bv[q], acc[p][q]);
        }
        if (kc + 1 < nchunk) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lds[buf ^ 1][0][el_w * GLD + x_w + q] = rg[q];
                lds[buf ^ 1][1][el_w * GLD + x_w + q] = ru[q];
            }
        }
        __syncthreads();
    }

    // accumulator register r of lane group g: row acc_row(g, r), column c
    T* ws = static_cast<T*>(a.ws) + (split * a.nmat + m) * (int64_t)a.nunit * a.nunit;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr * 32 + p * 16 + Mma<T>::acc_row(g, r);
                const int j = j0 + wc * 32 + q * 16 + c;
                if (i < a.nunit && j < a.nunit) ws[(int64_t)i * a.nunit + j] = acc[p][q][r];
            }
}

template <typename T>
__global__ void __launch_bounds__(256) grad_d_reduce_kernel(const T* __restrict__ ws,
                                                            T* __restrict__ out, int64_t count,
                                                            int64_t nsplit) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    T s = T(0);
    for (int64_t k = 0; k < nsplit; ++k) s += ws[k * count + idx];  // fixed order
    out[idx] = s;
}

struct SplitPlan {
    int64_t nsplit;
    int64_t split_len;
};

SplitPlan plan_splits(int nmat, int64_t nelem, int nunit) {
    const int64_t tiles = (int64_t)nmat * ceil_div(nunit, GT) * ceil_div(nunit, GT);
    const int64_t target = 2048;  // work-groups to fill 256 CUs several times over
    int64_t ns = std::max<int64_t>(1, ceil_div(target, tiles));
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, ceil_div(nelem, 256)));
    int64_t len = round_up(ceil_div(std::max<int64_t>(nelem, 1), ns), GK);
    ns = std::max<int64_t>(1, ceil_div(nelem, len));
    return {ns, len};
}

template <typename T>
dg_status launch_grad_d(int nmat, int64_t nelem, int nunit, const void* u, const void* g,
                        void* grad_D, void* ws, size_t ws_bytes, hipStream_t s) {
    const int64_t count = (int64_t)nmat * nunit * nunit;
    if (nelem == 0) {
        // empty sum: zeros, written by the reduce kernel with no partials
        hipLaunchKernelGGL(grad_d_reduce_kernel<T>, dim3((unsigned)ceil_div(count, 256)), dim3(256),
                           0, s, static_cast<const T*>(nullptr), static_cast<T*>(grad_D), count,
                           (int64_t)0);
        DG_HIP_CHECK(hipGetLastError());
        return DG_OK;
    }
    const SplitPlan sp = plan_splits(nmat, nelem, nunit);
    const size_t need = (size_t)sp.nsplit * count * sizeof(T);
    if (!ws || ws_bytes < need) return fail(DG_EINVAL, "dgdiff_backward: workspace too small");
    GdArgs a;
    a.g = g;
    a.u = u;
    a.ws = ws;
    a.nelem = nelem;
    a.split_len = sp.split_len;
    a.nmat = nmat;
    a.nunit = nunit;
    a.ntile = (int)ceil_div(nunit, GT);
    a.vec = 0;
    dim3 grid((unsigned)(nmat * a.ntile * a.ntile), (unsigned)sp.nsplit);
    hipLaunchKernelGGL(grad_d_partial_kernel<T>, grid, dim3(256), 0, s, a);
    DG_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(grad_d_reduce_kernel<T>, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s,
                       static_cast<const T*>(ws), static_cast<T*>(grad_D), count, sp.nsplit);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

// ------------------------------------------------------------------ grad_u

template <typename T>
dg_status launch_grad_u(int nmat, int64_t nelem, int nunit, const void* D, const void* g,
                        void* grad_u, const dg_tile* tile, hipStream_t s) {
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    const int waves = (tile && tile->waves) ? tile->waves : 4;
    if (waves < 1 || waves > 8) return fail(DG_EINVAL, "tile.waves must be in 1..8");
    KArgs a = {};
    a.nelem = nelem;
    a.nunit = nunit;
    a.transpose = 1;
    a.out = grad_u;
    a.seg_stride = nelem * (int64_t)nunit;
    a.D = D;
    a.src = g;
    // all operators in one pass when their segments fit the registers
    kern_fn one = nmat == 1 ? pick_kernel<T, 1, 1>(kq)
                : nmat == 2 ? pick_kernel<T, 1, 2>(kq)
                : nmat == 3 ? pick_kernel<T, 1, 3>(kq) : nullptr;
    if (one) {
        if (nmat == 1) return launch<T, 1>(a, 1, kq, 1, tile, waves, one, s);
        if (nmat == 2) return launch<T, 2>(a, 1, kq, 1, tile, waves, one, s);
        return launch<T, 3>(a, 1, kq, 1, tile, waves, one, s);
    }
    // one operator per launch; launches after the first accumulate
    for (int m = 0; m < nmat; ++m) {
        KArgs am = a;
        am.D = static_cast<const T*>(D) + (int64_t)m * nunit * nunit;
        am.src = static_cast<const T*>(g) + (int64_t)m * nelem * nunit;
        am.seg_stride = 0;
        kern_fn fn = nullptr;
#define X(k) \
        if (kq == k) fn = m == 0 ? (kern_fn)dg_kernel<T, k, 1, 1, false> : (kern_fn)dg_kernel<T, k, 1, 1, true>;
        DG_KQ_LIST(X)
#undef X
        if (!fn) return fail(DG_EUNSUPPORTED, "no grad_u kernel instance");
        dg_status st = launch<T, 1>(am, 1, kq, 1, tile, waves, fn, s);
        if (st != DG_OK) return st;
    }
    return DG_OK;
}

}  // namespace

size_t backward_workspace_bytes(dg_dtype t, int nmat, int64_t nelem, int nunit) {
    if (nelem <= 0) return 0;
    const SplitPlan sp = plan_splits(nmat, nelem, nunit);
    return (size_t)sp.nsplit * nmat * nunit * nunit * dtype_size(t);
}

dg_status launch_dg_backward(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                             const void* u, const void* g, void* grad_u, void* grad_D, void* ws,
                             size_t ws_bytes, hipStream_t s) {
    if (grad_D) {
        dg_status st = t == DG_F32
                           ? launch_grad_d<float>(nmat, nelem, nunit, u, g, grad_D, ws, ws_bytes, s)
                           : launch_grad_d<double>(nmat, nelem, nunit, u, g, grad_D, ws, ws_bytes, s);
        if (st != DG_OK) return st;
    }
    if (grad_u && nelem > 0) {
        dg_status st = t == DG_F32 ? launch_grad_u<float>(nmat, nelem, nunit, D, g, grad_u, nullptr, s)
                                   : launch_grad_u<double>(nmat, nelem, nunit, D, g, grad_u, nullptr, s);
        if (st != DG_OK) return st;
    }
    return DG_OK;
}

}  // namespace dg
