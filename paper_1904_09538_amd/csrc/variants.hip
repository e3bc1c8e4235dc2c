// Program variants of the paper's three evaluation computations (Sections
// "Matrix Multiplication", "DG Differentiation" and "Finite Differences"):
// equivalent formulations of one operation that differ in how work-items map
// onto the data, what is staged in LDS and how the element data is laid out.
// The model's task is to rank them (Section "Introduction": a model is useful
// when it orders equivalent variants correctly), so they are written the way
// the paper describes them, as FP32 vector-ALU code with 16 x 16 (or 18 x 18)
// work-groups, not as the library's tuned kernels.  Every variant also has
// work-removed twins (Algorithm "remove work"): the same loops and global
// accesses to a chosen subset of arrays, each load added to one per-work-item
// sum, no LDS, no barriers, no other arithmetic, the sum stored where the
// kernel stores its result or, when that store is removed, one float per
// work-item into a destination array.
//
// Work-item coordinates: threadIdx.x = l0 + L l1 with L = 16 (18 for the
// 18 x 18 stencil), l0 = lid(0), l1 = lid(1); blockIdx.x = gid(0),
// blockIdx.y = gid(1).  A 64-wide wave therefore holds four lid(1) rows of a
// 16-wide work-group.
//
// Loads are never predicated: a work-item whose element (or grid point) lies
// past the end loads the last one instead, so every work-item issues the same
// loads and only the result stores are guarded.
#include <algorithm>

#include "common.hpp"

namespace dg {

VariantShape variant_shape(const dg_variant_desc* d) {
    VariantShape s{0, 0, 256};
    switch (d->kind) {
        case DG_V_MM_PF:
        case DG_V_MM_NOPF:
            s.gx = s.gy = d->n / 16;
            break;
        case DG_V_DG_NOPF:
        case DG_V_DG_PFU:
        case DG_V_DG_PFDM:
        case DG_V_DG_PFDMT:
            s.gx = ceil_div(d->n, 16);
            s.gy = d->nunit / 16;
            break;
        case DG_V_FD16:
            s.gx = s.gy = ceil_div(d->n, 14);
            break;
        case DG_V_FD18:
            s.gx = s.gy = ceil_div(d->n, 16);
            s.threads = 324;
            break;
    }
    return s;
}

dg_status check_variant(const dg_variant_desc* d) {
    if (d->work_removed != 0 && d->work_removed != 1) return fail(DG_EINVAL, "variant: work_removed 0 or 1");
    if (d->keep < 0 || d->keep > 7 || (!d->work_removed && d->keep))
        return fail(DG_EINVAL, "variant: keep is a subset of DG_V_KEEP_* and only for work-removed twins");
    if (d->n < 0) return fail(DG_EINVAL, "variant: negative size");
    switch (d->kind) {
        case DG_V_MM_PF:
        case DG_V_MM_NOPF:
            if (d->n % 16 || d->n > 16 * (int64_t)65535)
                return fail(DG_EINVAL, "matmul variant: n a multiple of 16, at most 16 x 65535");
            return DG_OK;
        case DG_V_DG_NOPF:
        case DG_V_DG_PFU:
        case DG_V_DG_PFDM:
        case DG_V_DG_PFDMT:
            if (d->nunit < 16 || d->nunit > 512 || d->nunit % 16 || d->nmat < 1 || d->nmat > 8)
                return fail(DG_EINVAL, "DG variant: nunit a multiple of 16 in 16..512, nmat 1..8");
            if (ceil_div(d->n, 16) > INT32_MAX) return fail(DG_EINVAL, "DG variant: too many elements");
            return DG_OK;
        case DG_V_FD16:
        case DG_V_FD18:
            if (d->keep & DG_V_KEEP_IN1) return fail(DG_EINVAL, "stencil variant: one input array");
            if (ceil_div(d->n, d->kind == DG_V_FD16 ? 14 : 16) > 65535)
                return fail(DG_EINVAL, "stencil variant: n too large");
            if (d->ld_u < d->n + 2 || d->ld_res < d->n)
                return fail(DG_EINVAL, "stencil variant: ld_u >= n + 2 and ld_res >= n");
            return DG_OK;
    }
    return fail(DG_EINVAL, "unknown variant");
}

namespace {

constexpr int kIn0 = DG_V_KEEP_IN0, kIn1 = DG_V_KEEP_IN1, kOut = DG_V_KEEP_OUT;

struct VArgs {
    const float* in0;
    const float* in1;
    float* out;
    int64_t n;
    int nunit, nmat;
    int64_t ld_u, ld_res;
};

// A work-removed twin's destination: one float per work-item, work-group
// after work-group.
__device__ inline void store_dest(float* dest, float v, int threads) {
    const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    dest[wg * threads + threadIdx.x] = v;
}

// ---------------------------------------------------------------- matmul

// Tiled: per 16-wide k step the work-group stages a 16 x 16 tile of a (rows
// of the work-group's i range) and of b (columns of its j range) in LDS, one
// value per work-item, then each work-item takes 16 products from LDS.
template <bool TWIN, int KEEP>
__global__ void __launch_bounds__(256) v_mm_pf(VArgs p) {
    __shared__ float at[16][16], bt[16][16];
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int64_t n = p.n;
    const int64_t i = 16 * (int64_t)blockIdx.y + l1, j = 16 * (int64_t)blockIdx.x + l0;
    float acc = 0.f;
    for (int64_t ko = 0; ko < n / 16; ++ko) {
        if constexpr (!TWIN) {
            __syncthreads();
            at[l1][l0] = p.in0[i * n + 16 * ko + l0];
            bt[l1][l0] = p.in1[(16 * ko + l1) * n + j];
            __syncthreads();
#pragma unroll
            for (int ki = 0; ki < 16; ++ki) acc = fmaf(at[l1][ki], bt[ki][l0], acc);
        } else {
            if constexpr ((KEEP & kIn0) != 0) acc += p.in0[i * n + 16 * ko + l0];
            if constexpr ((KEEP & kIn1) != 0) acc += p.in1[(16 * ko + l1) * n + j];
        }
    }
    if (!TWIN || (KEEP & kOut)) p.out[i * n + j] = acc;
    else store_dest(p.out, acc, 256);
}

// Untiled: each work-item walks its row of a and column of b in global memory.
template <bool TWIN, int KEEP>
__global__ void __launch_bounds__(256) v_mm_nopf(VArgs p) {
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int64_t n = p.n;
    const int64_t i = 16 * (int64_t)blockIdx.y + l1, j = 16 * (int64_t)blockIdx.x + l0;
    float acc = 0.f;
    for (int64_t k = 0; k < n; ++k) {
        if constexpr (!TWIN) {
            acc = fmaf(p.in0[i * n + k], p.in1[k * n + j], acc);
        } else {
            if constexpr ((KEEP & kIn0) != 0) acc += p.in0[i * n + k];
            if constexpr ((KEEP & kIn1) != 0) acc += p.in1[k * n + j];
        }
    }
    if (!TWIN || (KEEP & kOut)) p.out[i * n + j] = acc;
    else store_dest(p.out, acc, 256);
}

// ---------------------------------------------------------------- DG

// Work-item (l0, l1) of work-group (g0, g1) owns element k = 16 g0 + l0 and
// node i = 16 g1 + l1.  Element-major layout: u[k][j], res[m][k][i]; the
// transposed layout: u[j][k], res[m][i][k].
template <bool T_LAYOUT>
__device__ inline int64_t u_at(int64_t k, int j, int64_t E, int nu) {
    return T_LAYOUT ? (int64_t)j * E + k : k * nu + j;
}
template <bool T_LAYOUT>
__device__ inline int64_t res_at(int m, int64_t k, int i, int64_t E, int nu) {
    return T_LAYOUT ? ((int64_t)m * nu + i) * E + k : ((int64_t)m * E + k) * nu + i;
}

// All operands from global memory; loop order m, j.
template <bool TWIN, int KEEP>
__global__ void __launch_bounds__(256) v_dg_nopf(VArgs p) {
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int64_t E = p.n;
    const int nu = p.nunit;
    const int64_t k = 16 * (int64_t)blockIdx.x + l0, kc = std::min<int64_t>(k, E - 1);
    const int i = 16 * blockIdx.y + l1;
    const float* urow = p.in0 + kc * nu;
    float tw = 0.f;
#pragma unroll 1
    for (int m = 0; m < p.nmat; ++m) {
        const float* drow = p.in1 + ((int64_t)m * nu + i) * nu;
        float acc = 0.f;
        for (int j = 0; j < nu; ++j) {
            if constexpr (!TWIN) {
                acc = fmaf(drow[j], urow[j], acc);
            } else {
                if constexpr ((KEEP & kIn1) != 0) tw += drow[j];
                if constexpr ((KEEP & kIn0) != 0) tw += urow[j];
            }
        }
        if constexpr (!TWIN) {
            if (k < E) p.out[res_at<false>(m, k, i, E, nu)] = acc;
        } else if constexpr ((KEEP & kOut) != 0) {
            if (k < E) p.out[res_at<false>(m, k, i, E, nu)] = tw;
        }
    }
    if constexpr (TWIN && (KEEP & kOut) == 0) store_dest(p.out, tw, 256);
}

// u staged in LDS: per 16-wide j step the work-group loads the 16 x 16 tile
// u[16 g0 .. +16][16 jo .. +16] (lid(0) along j, so consecutive lanes read
// consecutive values), then each work-item takes its element's 16 values
// from LDS and updates its NM sums (the m loop innermost, sums in registers).
template <int NM, bool TWIN, int KEEP>
__global__ void __launch_bounds__(256) v_dg_pfu(VArgs p) {
    __shared__ float ut[16][16];   // [element in tile][j in step]
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int64_t E = p.n;
    const int nu = p.nunit;
    const int64_t k = 16 * (int64_t)blockIdx.x + l0;
    const int64_t kf = std::min<int64_t>(16 * (int64_t)blockIdx.x + l1, E - 1);
    const int i = 16 * blockIdx.y + l1;
    float acc[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = 0.f;
    float tw = 0.f;
    for (int jo = 0; jo < nu / 16; ++jo) {
        if constexpr (!TWIN) {
            __syncthreads();
            ut[l1][l0] = p.in0[kf * nu + 16 * jo + l0];
            __syncthreads();
        } else if constexpr ((KEEP & kIn0) != 0) {
            tw += p.in0[kf * nu + 16 * jo + l0];
        }
        const float* dcol = p.in1 + (int64_t)i * nu + 16 * jo;
#pragma unroll 4
        for (int ji = 0; ji < 16; ++ji) {
            if constexpr (!TWIN) {
                const float uv = ut[l0][ji];
#pragma unroll
                for (int m = 0; m < NM; ++m) acc[m] = fmaf(dcol[(int64_t)m * nu * nu + ji], uv, acc[m]);
            } else if constexpr ((KEEP & kIn1) != 0) {
#pragma unroll
                for (int m = 0; m < NM; ++m) tw += dcol[(int64_t)m * nu * nu + ji];
            }
        }
    }
    if constexpr (!TWIN) {
        if (k < E) {
#pragma unroll
            for (int m = 0; m < NM; ++m) p.out[res_at<false>(m, k, i, E, nu)] = acc[m];
        }
    } else if constexpr ((KEEP & kOut) != 0) {
        if (k < E) {
#pragma unroll
            for (int m = 0; m < NM; ++m) p.out[res_at<false>(m, k, i, E, nu)] = tw;
        }
    } else {
        store_dest(p.out, tw, 256);
    }
}

// D staged in LDS: for each operator m and 16-wide j step the work-group
// loads the 16 x 16 tile D[m][16 g1 .. +16][16 jo .. +16] (lid(0) along j),
// then each work-item multiplies its row of the tile with its element's u
// values from global memory.  T_LAYOUT: the transposed element layout.
template <bool T_LAYOUT, bool TWIN, int KEEP>
__global__ void __launch_bounds__(256) v_dg_pfdm(VArgs p) {
    __shared__ float dt[16][16];   // [i in tile][j in step]
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int64_t E = p.n;
    const int nu = p.nunit;
    const int64_t k = 16 * (int64_t)blockIdx.x + l0, kc = std::min<int64_t>(k, E - 1);
    const int i = 16 * blockIdx.y + l1;
    float tw = 0.f;
#pragma unroll 1
    for (int m = 0; m < p.nmat; ++m) {
        const float* dtile = p.in1 + ((int64_t)m * nu + 16 * blockIdx.y + l1) * nu + l0;
        float acc = 0.f;
        for (int jo = 0; jo < nu / 16; ++jo) {
            if constexpr (!TWIN) {
                __syncthreads();
                dt[l1][l0] = dtile[16 * jo];
                __syncthreads();
#pragma unroll
                for (int ji = 0; ji < 16; ++ji)
                    acc = fmaf(dt[l1][ji], p.in0[u_at<T_LAYOUT>(kc, 16 * jo + ji, E, nu)], acc);
            } else {
                if constexpr ((KEEP & kIn1) != 0) tw += dtile[16 * jo];
                if constexpr ((KEEP & kIn0) != 0) {
#pragma unroll
                    for (int ji = 0; ji < 16; ++ji) tw += p.in0[u_at<T_LAYOUT>(kc, 16 * jo + ji, E, nu)];
                }
            }
        }
        if constexpr (!TWIN) {
            if (k < E) p.out[res_at<T_LAYOUT>(m, k, i, E, nu)] = acc;
        } else if constexpr ((KEEP & kOut) != 0) {
            if (k < E) p.out[res_at<T_LAYOUT>(m, k, i, E, nu)] = tw;
        }
    }
    if constexpr (TWIN && (KEEP & kOut) == 0) store_dest(p.out, tw, 256);
}

// ---------------------------------------------------------------- stencil

// L x L work-items stage the L x L grid tile whose corner is u[B g1][B g0]
// (B = L - 2; one value each, clamped at the far edges), then the B x B
// work-items with l0, l1 < B compute the outputs res[B g1 + l1][B g0 + l0].
template <int L, bool TWIN, int KEEP>
__global__ void __launch_bounds__(L * L) v_fd(VArgs p) {
    constexpr int B = L - 2;
    __shared__ float t[L][L];
    const int l0 = threadIdx.x % L, l1 = threadIdx.x / L;
    const int64_t n = p.n;
    const int64_t gi = std::min<int64_t>(B * (int64_t)blockIdx.y + l1, n + 1);
    const int64_t gj = std::min<int64_t>(B * (int64_t)blockIdx.x + l0, n + 1);
    const int64_t oi = B * (int64_t)blockIdx.y + l1, oj = B * (int64_t)blockIdx.x + l0;
    const bool inner = l0 < B && l1 < B;
    if constexpr (!TWIN) {
        t[l1][l0] = p.in0[gi * p.ld_u + gj];
        __syncthreads();
        if (inner) {
            float s = t[l1][l0 + 1] + t[l1 + 1][l0];
            s += t[l1 + 1][l0 + 2];
            s += t[l1 + 2][l0 + 1];
            const float r = fmaf(-4.f, t[l1 + 1][l0 + 1], s);
            if (oi < n && oj < n) p.out[oi * p.ld_res + oj] = r;
        }
    } else {
        float tw = 0.f;
        if constexpr ((KEEP & kIn0) != 0) tw += p.in0[gi * p.ld_u + gj];
        if constexpr ((KEEP & kOut) != 0) {
            if (inner && oi < n && oj < n) p.out[oi * p.ld_res + oj] = tw;
        } else {
            store_dest(p.out, tw, L * L);
        }
    }
}

// ---------------------------------------------------------------- dispatch

typedef void (*VKernel)(VArgs);

template <int KEEP>
VKernel pick_keep(dg_variant kind, int nmat) {
    switch (kind) {
        case DG_V_MM_PF: return v_mm_pf<true, KEEP>;
        case DG_V_MM_NOPF: return v_mm_nopf<true, KEEP>;
        case DG_V_DG_NOPF: return v_dg_nopf<true, KEEP>;
        case DG_V_DG_PFU:
            switch (nmat) {
                case 1: return v_dg_pfu<1, true, KEEP>;
                case 2: return v_dg_pfu<2, true, KEEP>;
                case 3: return v_dg_pfu<3, true, KEEP>;
                case 4: return v_dg_pfu<4, true, KEEP>;
                case 5: return v_dg_pfu<5, true, KEEP>;
                case 6: return v_dg_pfu<6, true, KEEP>;
                case 7: return v_dg_pfu<7, true, KEEP>;
                default: return v_dg_pfu<8, true, KEEP>;
            }
        case DG_V_DG_PFDM: return v_dg_pfdm<false, true, KEEP>;
        case DG_V_DG_PFDMT: return v_dg_pfdm<true, true, KEEP>;
        case DG_V_FD16: return v_fd<16, true, KEEP>;
        case DG_V_FD18: return v_fd<18, true, KEEP>;
    }
    return nullptr;
}

VKernel pick(const dg_variant_desc* d) {
    if (d->work_removed) {
        switch (d->keep) {
            case 0: return pick_keep<0>(d->kind, d->nmat);
            case 1: return pick_keep<1>(d->kind, d->nmat);
            case 2: return pick_keep<2>(d->kind, d->nmat);
            case 3: return pick_keep<3>(d->kind, d->nmat);
            case 4: return pick_keep<4>(d->kind, d->nmat);
            case 5: return pick_keep<5>(d->kind, d->nmat);
            case 6: return pick_keep<6>(d->kind, d->nmat);
            default: return pick_keep<7>(d->kind, d->nmat);
        }
    }
    switch (d->kind) {
        case DG_V_MM_PF: return v_mm_pf<false, 0>;
        case DG_V_MM_NOPF: return v_mm_nopf<false, 0>;
        case DG_V_DG_NOPF: return v_dg_nopf<false, 0>;
        case DG_V_DG_PFU:
            switch (d->nmat) {
                case 1: return v_dg_pfu<1, false, 0>;
                case 2: return v_dg_pfu<2, false, 0>;
                case 3: return v_dg_pfu<3, false, 0>;
                case 4: return v_dg_pfu<4, false, 0>;
                case 5: return v_dg_pfu<5, false, 0>;
                case 6: return v_dg_pfu<6, false, 0>;
                case 7: return v_dg_pfu<7, false, 0>;
                default: return v_dg_pfu<8, false, 0>;
            }
        case DG_V_DG_PFDM: return v_dg_pfdm<false, false, 0>;
        case DG_V_DG_PFDMT: return v_dg_pfdm<true, false, 0>;
        case DG_V_FD16: return v_fd<16, false, 0>;
        case DG_V_FD18: return v_fd<18, false, 0>;
    }
    return nullptr;
}

}  // namespace

// Bytes each array of a variant spans (in0, in1, out; out = the result array,
// or the twin's destination when its result store is removed).
void variant_extents(const dg_variant_desc* d, size_t* b0, size_t* b1, size_t* bout) {
    const int64_t n = d->n;
    const VariantShape s = variant_shape(d);
    *b0 = *b1 = *bout = 0;
    switch (d->kind) {
        case DG_V_MM_PF:
        case DG_V_MM_NOPF:
            *b0 = *b1 = *bout = (size_t)n * n * 4;
            break;
        case DG_V_DG_NOPF:
        case DG_V_DG_PFU:
        case DG_V_DG_PFDM:
        case DG_V_DG_PFDMT:
            *b0 = (size_t)n * d->nunit * 4;
            *b1 = (size_t)d->nmat * d->nunit * d->nunit * 4;
            *bout = (size_t)d->nmat * n * d->nunit * 4;
            break;
        case DG_V_FD16:
        case DG_V_FD18:
            *b0 = (size_t)((n + 1) * d->ld_u + n + 2) * 4;
            *bout = n ? (size_t)((n - 1) * d->ld_res + n) * 4 : 0;
            break;
    }
    if (d->work_removed && !(d->keep & DG_V_KEEP_OUT)) *bout = (size_t)(s.gx * s.gy * s.threads) * 4;
}

}  // namespace dg

using namespace dg;

extern "C" {

dg_status dg_variant_shape(const dg_variant_desc* d, int64_t* workgroups, int32_t* threads) {
    set_error("");
    if (!d) return fail(DG_EINVAL, "dg_variant_shape: NULL descriptor");
    const dg_status st = check_variant(d);
    if (st != DG_OK) return st;
    const VariantShape s = variant_shape(d);
    if (workgroups) *workgroups = s.gx * s.gy;
    if (threads) *threads = s.threads;
    return DG_OK;
}

dg_status dg_variant_run(const dg_variant_desc* d, const void* in0, const void* in1, void* out,
                         dg_stream_t stream) {
    set_error("");
    if (!d) return fail(DG_EINVAL, "dg_variant_run: NULL descriptor");
    dg_status st = check_variant(d);
    if (st != DG_OK) return st;
    const VariantShape s = variant_shape(d);
    if (s.gx * s.gy == 0) return DG_OK;
    const bool fd = d->kind == DG_V_FD16 || d->kind == DG_V_FD18;
    const bool need0 = !d->work_removed || (d->keep & DG_V_KEEP_IN0);
    const bool need1 = !fd && (!d->work_removed || (d->keep & DG_V_KEEP_IN1));
    if (!out || (need0 && !in0) || (need1 && !in1)) return fail(DG_EINVAL, "dg_variant_run: NULL array");
    size_t b0, b1, bout;
    variant_extents(d, &b0, &b1, &bout);
    if ((need0 && overlaps(out, bout, in0, b0)) || (need1 && overlaps(out, bout, in1, b1)))
        return fail(DG_EINVAL, "dg_variant_run: the output overlaps an input");
    VArgs a;
    a.in0 = static_cast<const float*>(in0);
    a.in1 = static_cast<const float*>(in1);
    a.out = static_cast<float*>(out);
    a.n = d->n;
    a.nunit = d->nunit;
    a.nmat = d->nmat;
    a.ld_u = d->ld_u;
    a.ld_res = d->ld_res;
    VKernel k = pick(d);
    hipLaunchKernelGGL(k, dim3((unsigned)s.gx, (unsigned)s.gy), dim3(s.threads), 0,
                       reinterpret_cast<hipStream_t>(stream), a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // extern "C"
