// Adjoint of the DG differentiation operator, FP32 and FP64.  For a loss L with
// upstream gradient g[m][e][i] = dL/dout[m][e][i]:
//     grad_u[e][j]    = sum_m sum_i D[m][i][j] * g[m][e][i]
//     grad_D[m][i][j] = sum_e g[m][e][i] * u[e][j]
//
// grad_u, FP32 rows of more than 96 nodes: a GEMM
//     grad_u^T[j][e] = sum_(m,i) D[m][i][j] g[m][e][i]
// on 128 x 128 tiles (output nodes x elements) whose contraction over (m, i)
// streams through LDS in chunks of 16 nodes of one operator, so the operator
// is not held resident (at p = 4 its panels for all three slabs leave room
// for a single work-group of 4 waves per CU).  Otherwise grad_u runs on the
// forward's contraction kernel (dg_kernel.hpp) with the operator transposed
// and the g slabs as contraction segments; when the nmat segments do not fit
// the register budget, each operator is applied in its own launch and the
// later launches accumulate (stream-ordered).
//
// grad_D is a GEMM C[(m,i)][j] = sum_e G_m^T[i][e] U[e][j] with a very long
// contraction (the element count).  It is split: work-group (tile, split)
// multiplies one 128x128 output tile over one contiguous element range on the
// matrix cores and writes an FP32/FP64 partial tile to the caller's
// workspace; a second kernel adds the partials of every entry in split order
// 0, 1, 2, ...  The result is therefore deterministic (no atomics, no
// order-dependent accumulation).
#include <mutex>

#include "dg_kernel.hpp"

namespace dg {
namespace {

using namespace kern;

// ------------------------------------------------------------------ grad_D

constexpr int GT = kBwdTile;    // output tile (rows i x cols j): all of i and j up to nunit 128
constexpr int GK = kBwdChunk;   // elements per LDS chunk

struct GdArgs {
    const void* g;
    const void* u;
    void* ws;             // [nsplit][nmat][nunit][nunit]
    int64_t nelem;
    int64_t split_len;    // elements per split (multiple of GK)
    int nmat;
    int nunit;
    int ntile;            // ceil(nunit / GT)
};

// Four consecutive values of a row from any element-size boundary (one or
// two 16-byte loads, the copy left to the compiler); `avail` of them belong
// to the row, the rest read as zero.
template <typename T>
__device__ inline void gd_load4(const T* p, bool ok, int avail, T (&v)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = T(0);
    if (!ok || avail <= 0) return;
    if (avail >= 4) {
        __builtin_memcpy(v, p, 4 * sizeof(T));
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (q < avail) v[q] = p[q];
    }
}

// Partial grad_D tile: C[i][j] = sum over the split's elements of g_m[e][i] u[e][j].
// A work-group owns a GT x GT tile (4 waves of 64 x 64, 4 x 4 MFMA tiles
// each) and walks its elements in chunks of GK.  Each chunk of g and u rows
// is loaded with 16-byte vectors and stored element-major in LDS with
// 16-byte stores (sixteen lanes per row: no bank conflicts); lane group g
// contracts elements 4g .. 4g+3 of the chunk, reading each operand value
// with one LDS load.  Chunks are double-buffered: the next one is fetched
// into registers while the current one is multiplied.
template <typename T>
__global__ void __launch_bounds__(256) grad_d_partial_kernel(GdArgs a) {
    typedef typename Mma<T>::acc_t acc_t;
    constexpr int NP = GT + 16 / (int)sizeof(T);  // LDS row stride (nodes + padding)
    __shared__ __attribute__((aligned(16))) T lds[2][2][GK * NP];  // [buf][g|u][element][node]
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
    const int n = a.nunit;
    const T* __restrict__ gm = static_cast<const T*>(a.g) + (int64_t)m * a.nelem * n;
    const T* __restrict__ u = static_cast<const T*>(a.u);

    // staging: thread t loads element el = t/16 of the chunk, nodes x .. x+7
    const int el_s = t >> 4, x_s = (t & 15) * 8;
    T rg[8], ru[8];
    auto load = [&](int64_t e0) {
        const int64_t e = e0 + el_s;
        const bool ok = e < e_hi;
        const int64_t eo = (ok ? e : 0) * n;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            T v[4];
            gd_load4<T>(gm + eo + i0 + x_s + 4 * h, ok, n - (i0 + x_s + 4 * h), v);
#pragma unroll
            for (int q = 0; q < 4; ++q) rg[4 * h + q] = v[q];
            gd_load4<T>(u + eo + j0 + x_s + 4 * h, ok, n - (j0 + x_s + 4 * h), v);
#pragma unroll
            for (int q = 0; q < 4; ++q) ru[4 * h + q] = v[q];
        }
    };
    auto store = [&](int buf) {
        // one element row per sixteen lanes, 8 nodes per lane: 16-byte stores
        __builtin_memcpy(&lds[buf][0][el_s * NP + x_s], rg, 8 * sizeof(T));
        __builtin_memcpy(&lds[buf][1][el_s * NP + x_s], ru, 8 * sizeof(T));
    };

    acc_t acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = acc_t(T(0));

    const int64_t nchunk = e_hi > e_lo ? ceil_div(e_hi - e_lo, GK) : 0;
    if (nchunk > 0) {
        load(e_lo);
        store(0);
    }
    __syncthreads();
    for (int64_t kc = 0; kc < nchunk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nchunk;
        if (more) load(e_lo + (kc + 1) * GK);
        T av[4][4], bv[4][4];  // [tile][element 4g + s]
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const T* Gr = &lds[buf][0][(4 * g + s4) * NP];
            const T* Ur = &lds[buf][1][(4 * g + s4) * NP];
#pragma unroll
            for (int p = 0; p < 4; ++p) av[p][s4] = Gr[wr * 64 + p * 16 + c];
#pragma unroll
            for (int q = 0; q < 4; ++q) bv[q][s4] = Ur[wc * 64 + q * 16 + c];
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = Mma<T>::step(av[p][s4], bv[q][s4], acc[p][q]);
        if (more) store(buf ^ 1);
        __syncthreads();
    }

    // accumulator register r of lane group g: row acc_row(g, r), column c
    T* ws = static_cast<T*>(a.ws) + (split * a.nmat + m) * (int64_t)n * n;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr * 64 + p * 16 + Mma<T>::acc_row(g, r);
                const int j = j0 + wc * 64 + q * 16 + c;
                if (i < n && j < n) ws[(int64_t)i * n + j] = acc[p][q][r];
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

// Partials are summed in two fixed-order stages (groups of kRedGroup splits,
// then the group sums), so the result does not depend on scheduling.
constexpr int64_t kRedGroup = kBwdRedGroup;

template <typename T>
__global__ void __launch_bounds__(256) grad_d_reduce_groups_kernel(const T* __restrict__ ws,
                                                                   T* __restrict__ ws2, int64_t count,
                                                                   int64_t nsplit) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    const int64_t k0 = (int64_t)blockIdx.y * kRedGroup;
    const int64_t k1 = min<int64_t>(nsplit, k0 + kRedGroup);
    T s = T(0);
    for (int64_t k = k0; k < k1; ++k) s += ws[k * count + idx];  // fixed order
    ws2[(int64_t)blockIdx.y * count + idx] = s;
}

// Resident work-groups per CU of the split-partial kernel on the current device.
template <typename T>
dg_status grad_d_per_cu(int* per_cu) {
    DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, reinterpret_cast<const void*>(grad_d_partial_kernel<T>), 256, 0));
    *per_cu = std::max(*per_cu, 1);
    return DG_OK;
}

template <typename T>
dg_status plan_splits(int nmat, int64_t nelem, int nunit, SplitPlan* sp, size_t cap_bytes = 0) {
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    int per_cu = 1;
    st = grad_d_per_cu<T>(&per_cu);
    if (st != DG_OK) return st;
    if (!bwd_split_plan(nmat, nelem, nunit, per_cu, dev.num_cu, sizeof(T), cap_bytes, sp))
        return fail(DG_EUNSUPPORTED, "grad_D partials exceed the fixed scratch");
    return DG_OK;
}

template <typename T>
dg_status launch_grad_d(int nmat, int64_t nelem, int nunit, const void* u, const void* g,
                        void* grad_D, void* ws, size_t ws_bytes, bool fit_ws, hipStream_t s) {
    const int64_t count = (int64_t)nmat * nunit * nunit;
    if (nelem == 0) {
        // empty sum: zeros, written by the reduce kernel with no partials
        hipLaunchKernelGGL(grad_d_reduce_kernel<T>, dim3((unsigned)ceil_div(count, 256)), dim3(256),
                           0, s, static_cast<const T*>(nullptr), static_cast<T*>(grad_D), count,
                           (int64_t)0);
        DG_HIP_CHECK(hipGetLastError());
        return DG_OK;
    }
    SplitPlan sp;
    dg_status st = plan_splits<T>(nmat, nelem, nunit, &sp, fit_ws ? ws_bytes : 0);
    if (st != DG_OK) return st;
    const size_t need = (size_t)(sp.nsplit + sp.ngroups) * count * sizeof(T);
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
    dim3 grid((unsigned)(nmat * a.ntile * a.ntile), (unsigned)sp.nsplit);
    hipLaunchKernelGGL(grad_d_partial_kernel<T>, grid, dim3(256), 0, s, a);
    DG_HIP_CHECK(hipGetLastError());
    T* ws2 = static_cast<T*>(ws) + sp.nsplit * count;
    hipLaunchKernelGGL(grad_d_reduce_groups_kernel<T>, dim3((unsigned)ceil_div(count, 256), (unsigned)sp.ngroups),
                       dim3(256), 0, s, static_cast<const T*>(ws), ws2, count, sp.nsplit);
    DG_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(grad_d_reduce_kernel<T>, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s,
                       static_cast<const T*>(ws2), static_cast<T*>(grad_D), count, sp.ngroups);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

// ------------------------------------------------------------------ grad_u

constexpr int UT = 128;      // tile: output nodes j x elements
constexpr int UK = 16;       // contraction nodes per chunk (one operator)
constexpr int UA = UT + 4;   // LDS row stride of the operator chunk
constexpr int UB = UK + 4;   // LDS row stride of the element chunk
constexpr int kGradUGemmMin = 97;  // FP32 nunit from which grad_u runs as a GEMM

struct GuArgs {
    const float* D;   // [nmat][n][n]
    const float* g;   // [nmat][nelem][n]
    float* gu;        // [nelem][n]
    int64_t nelem;
    int64_t ntile_e;  // ceil(nelem / UT)
    int nmat;
    int n;
    int ntile_j;      // ceil(n / UT)
};

// Work-group: 4 waves, 2 x 2 of 64 x 64 (4 x 4 MFMA tiles of 16 x 16).  The
// chunk's operator rows D[m][i0 .. i0+15][j0 ..] are kept as they lie in
// memory (row = contraction node, column = output node: lane group g reads
// its four nodes 4g .. 4g+3 with one LDS load each); the element rows
// g[m][e][i0 .. i0+15] are kept per element (one 16-byte LDS load per lane
// per tile).  Chunks are double-buffered: the next is fetched into registers
// while the current one is multiplied.  Blocks that share an element tile sit
// on one XCD (block b on XCD b % 8), so the other output-node tiles re-read
// it from that XCD's L2.
__global__ void __launch_bounds__(256) grad_u_gemm_kernel(GuArgs a) {
    __shared__ __attribute__((aligned(16))) float As[2][UK * UA];
    __shared__ __attribute__((aligned(16))) float Bs[2][UT * UB];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const int xcd = blockIdx.x & 7;
    const int kb = blockIdx.x >> 3;
    const int64_t te = (int64_t)(kb / a.ntile_j) * 8 + xcd;
    if (te >= a.ntile_e) return;  // whole block past the end: no barrier reached
    const int j0 = (kb % a.ntile_j) * UT;
    const int64_t e0 = te * UT;
    const int n = a.n;
    const int kpm = (n + UK - 1) / UK;  // chunks per operator
    const int nchunk = a.nmat * kpm;

    // staging: operator chunk row ka = t/32 (+8), output nodes ja .. ja+3;
    // element eb = t/4 (+64), contraction nodes kq .. kq+3
    const int ka = t >> 5, ja = (t & 31) * 4;
    const int eb = t >> 2, kq = (t & 3) * 4;
    const bool e_ok[2] = {e0 + eb < a.nelem, e0 + eb + 64 < a.nelem};
    float ra[2][4], rb[2][4];
    auto load = [&](int kc) {
        const int m = kc / kpm;
        const int i0 = (kc % kpm) * UK;
        const float* Dm = a.D + (int64_t)m * n * n;
        const float* gm = a.g + (int64_t)m * a.nelem * n;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = i0 + ka + 8 * h;
            const int j = j0 + ja;
            gd_load4<float>(Dm + (int64_t)(i < n ? i : 0) * n + j, i < n, n - j, ra[h]);
            const int64_t e = e0 + eb + 64 * h;
            gd_load4<float>(gm + (e_ok[h] ? e : 0) * n + i0 + kq, e_ok[h], n - (i0 + kq), rb[h]);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __builtin_memcpy(&As[buf][(ka + 8 * h) * UA + ja], ra[h], 16);
            __builtin_memcpy(&Bs[buf][(eb + 64 * h) * UB + kq], rb[h], 16);
        }
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};

    load(0);
    store(0);
    __syncthreads();
    for (int kc = 0; kc < nchunk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nchunk;
        if (more) load(kc + 1);
        float av[4][4];  // [tile][node 4g + s]
        f32x4 bv[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const float* Ar = &As[buf][(4 * g + s4) * UA + wm * 64 + c];
#pragma unroll
            for (int p = 0; p < 4; ++p) av[p][s4] = Ar[p * 16];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            bv[q] = *reinterpret_cast<const f32x4*>(&Bs[buf][(wn * 64 + q * 16 + c) * UB + 4 * g]);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p][s4], bv[q][s4], acc[p][q], 0, 0, 0);
        if (more) store(buf ^ 1);
        __syncthreads();
    }

    // lane holds output nodes j .. j+3 (j = j0 + wm*64 + p*16 + 4g) of
    // element e0 + wn*64 + q*16 + c
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t e = e0 + wn * 64 + q * 16 + c;
        if (e >= a.nelem) continue;
        float* row = a.gu + e * n;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int j = j0 + wm * 64 + p * 16 + 4 * g;
            if (j + 4 <= n) {
                __builtin_memcpy(row + j, &acc[p][q], 16);
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    if (j + r < n) row[j + r] = acc[p][q][r];
            }
        }
    }
}

dg_status launch_grad_u_gemm(int nmat, int64_t nelem, int nunit, const void* D, const void* g,
                             void* grad_u, hipStream_t s) {
    GuArgs a;
    a.D = static_cast<const float*>(D);
    a.g = static_cast<const float*>(g);
    a.gu = static_cast<float*>(grad_u);
    a.nelem = nelem;
    a.ntile_e = ceil_div(nelem, (int64_t)UT);
    a.nmat = nmat;
    a.n = nunit;
    a.ntile_j = (int)ceil_div(nunit, UT);
    const int64_t blocks = ceil_div(a.ntile_e, (int64_t)8) * 8 * a.ntile_j;
    if (blocks > INT32_MAX) return fail(DG_EUNSUPPORTED, "grad_u: too many elements for one launch");
    hipLaunchKernelGGL(grad_u_gemm_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

template <typename T>
dg_status launch_grad_u(int nmat, int64_t nelem, int nunit, const void* D, const void* g,
                        void* grad_u, const dg_tile* tile, hipStream_t s) {
    if (sizeof(T) == 4 && nunit >= kGradUGemmMin)
        return launch_grad_u_gemm(nmat, nelem, nunit, D, g, grad_u, s);
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
    // one operator per launch; launches after the first accumulate, with the
    // first launch's resident work-groups per CU (one schedule for all)
    dg_tile tm = tile ? *tile : dg_tile{};
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
        int per_cu = 0;
        dg_status st = launch<T, 1>(am, 1, kq, 1, &tm, waves, fn, s, nullptr, &per_cu);
        if (st != DG_OK) return st;
        tm.groups_per_cu = per_cu;
    }
    return DG_OK;
}

}  // namespace

namespace {

template <typename T>
dg_status resolve_bwd(int nmat, int64_t nelem, int nunit, dg_tile* tu, dg_tile* td) {
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    if (td) {
        *td = dg_tile{};
        int per_cu = 1;
        st = grad_d_per_cu<T>(&per_cu);
        if (st != DG_OK) return st;
        td->groups_per_cu = per_cu;
    }
    if (!tu) return DG_OK;
    *tu = dg_tile{};
    if (sizeof(T) == 4 && nunit >= kGradUGemmMin) {
        int per_cu = 1;
        DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(grad_u_gemm_kernel), 256, 0));
        *tu = dg_tile{UT, 4, std::max(per_cu, 1), 0, DG_TILE_BATCH_GEMM};
        return DG_OK;
    }
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    const int nseg = grad_u_segments(sizeof(T), nmat, kq);
    kern_fn fn = nseg == 1 ? pick_kernel<T, 1, 1>(kq)
               : nseg == 2 ? pick_kernel<T, 1, 2>(kq) : pick_kernel<T, 1, 3>(kq);
    if (!fn) return fail(DG_EUNSUPPORTED, "no grad_u kernel instance");
    const int V = (int)(16 / sizeof(T));
    const bool vec = nunit % V == 0 && (nseg == 1 || (nelem * nunit) % V == 0);
    Plan P;
    st = make_plan(sizeof(T), nseg, 1, nelem, nunit, kq, 1, 4, 0, 1, dev.num_cu, vec, &P);
    if (st != DG_OK) return st;
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
    int per_cu = 1;
    DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                              256, P.smem));
    *tu = dg_tile{16, 4, std::max(per_cu, 1), P.ppg, 0};
    return DG_OK;
}

}  // namespace

dg_status resolve_backward(dg_dtype t, int nmat, int64_t nelem, int nunit, dg_tile* tu, dg_tile* td) {
    return t == DG_F64 ? resolve_bwd<double>(nmat, nelem, nunit, tu, td)
                       : resolve_bwd<float>(nmat, nelem, nunit, tu, td);
}

size_t backward_workspace_bytes(dg_dtype t, int nmat, int64_t nelem, int nunit) {
    if (nelem <= 0) return 0;
    SplitPlan sp;
    const dg_status st = t == DG_F64 ? plan_splits<double>(nmat, nelem, nunit, &sp)
                                     : plan_splits<float>(nmat, nelem, nunit, &sp);
    if (st != DG_OK) return 0;
    return (size_t)(sp.nsplit + sp.ngroups) * nmat * nunit * nunit * dtype_size(t);
}

namespace {

dg_status backward(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D, const void* u,
                   const void* g, void* grad_u, void* grad_D, void* ws, size_t ws_bytes, bool fit_ws,
                   hipStream_t s) {
    if (grad_D) {
        dg_status st =
            t == DG_F32
                ? launch_grad_d<float>(nmat, nelem, nunit, u, g, grad_D, ws, ws_bytes, fit_ws, s)
                : launch_grad_d<double>(nmat, nelem, nunit, u, g, grad_D, ws, ws_bytes, fit_ws, s);
        if (st != DG_OK) return st;
    }
    if (grad_u && nelem > 0) {
        dg_status st = t == DG_F32 ? launch_grad_u<float>(nmat, nelem, nunit, D, g, grad_u, nullptr, s)
                                   : launch_grad_u<double>(nmat, nelem, nunit, D, g, grad_u, nullptr, s);
        if (st != DG_OK) return st;
    }
    return DG_OK;
}

// Fixed scratch of the no-allocation backward: grad_D's split partials and
// group sums.  Every work-group of the partial kernel writes its whole tile
// and the group stage writes every group sum, so nothing needs clearing
// between calls.  In host code `scratch` names a host-side stand-in; kernels
// get the device address taken by hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kBackwardScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

dg_status scratch_ptr(void** out) {
    int dev = -1;
    DG_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DG_OK;
}

}  // namespace

dg_status launch_dg_backward(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                             const void* u, const void* g, void* grad_u, void* grad_D, void* ws,
                             size_t ws_bytes, hipStream_t s) {
    return backward(t, nmat, nelem, nunit, D, u, g, grad_u, grad_D, ws, ws_bytes, false, s);
}

dg_status launch_dg_backward_noalloc(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                                     const void* u, const void* g, void* grad_u, void* grad_D,
                                     hipStream_t s) {
    void* ws = nullptr;
    if (grad_D && nelem > 0) {
        dg_status st = scratch_ptr(&ws);
        if (st != DG_OK) return st;
    }
    return backward(t, nmat, nelem, nunit, D, u, g, grad_u, grad_D, ws, ws ? kBackwardScratchBytes : 0,
                    true, s);
}

}  // namespace dg
