// DG differentiation with BF16 or FP8-E4M3FN operands and FP32 accumulation:
//     out[m][e][i] = inv_sD[m] * inv_su[e] * sum_j qD[m][i][j] * qu[e][j]
// where qD, qu are the quantised operators and element data and inv_s* the
// inverse power-of-two scales of the quantiser (exact de-scaling).
//
// Same scheme as the FP32/FP64 kernel (C^T = D_stack U^T on 16x16 MFMA tiles,
// resident operator panel groups, XCD-aware tile streams), on
// v_mfma_f32_16x16x32_bf16 (and, opt-in, v_mfma_f32_16x16x32_fp8_fp8): each
// lane feeds eight consecutive nodes per k-step.  Lane group g owns nodes
// [g*KQ, (g+1)*KQ) and k-step s covers g*KQ + 8s .. g*KQ + 8s + 7, so the
// element data arrive as 16-byte (BF16) or 8-byte (FP8) vector loads and the
// operator rows as LDS reads of the same width.  The 16x16 FP32 accumulator
// layout is that of the FP32 instruction: lane group g holds rows 4g..4g+3.
#include "common.hpp"

namespace dg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Operand formats.  G = element type in HBM, L = element type staged in LDS,
// F = the 8-value MFMA operand fragment of one lane.
//   0  BF16 in HBM, BF16 MFMA.
//   1  FP8 in HBM, native FP8 MFMA (v_mfma_f32_16x16x32_fp8_fp8).  Measured on
//      gfx950: the instruction's internal sum of its 32 products drops terms
//      about 2^13 below the largest, short of FP32 accumulation, so this is
//      opt-in (DG_TILE_FP8_NATIVE).
//   2  FP8 in HBM, widened exactly to BF16 in registers / at LDS staging and
//      multiplied on the BF16 matrix cores: FP8 bandwidth, exact products,
//      FP32 accumulation.  Default for FP8 input.
template <int FMT>
struct LP;

template <>
struct LP<0> {
    typedef uint16_t G;
    typedef uint16_t L;
    typedef u32x4 GF;  // 8 values as loaded from HBM
    typedef u32x4 F;
    __device__ static inline F widen(GF v) { return v; }
    __device__ static inline L widen1(G v) { return v; }
    __device__ static inline f32x4 mma(F a, F b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};

template <>
struct LP<1> {
    typedef uint8_t G;
    typedef uint8_t L;
    typedef u32x2 GF;
    typedef u32x2 F;
    __device__ static inline F widen(GF v) { return v; }
    __device__ static inline L widen1(G v) { return v; }
    __device__ static inline f32x4 mma(F a, F b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                          __builtin_bit_cast(long, b), c, 0, 0, 0);
    }
};

// Exact E4M3FN -> BF16: every E4M3 value (subnormals included) is a BF16 value.
__device__ inline uint32_t e4m3_to_bf16_bits(uint32_t b) {
    const uint32_t mag = b & 0x7Fu;
    // normal: exponent+mantissa field moves up 4 bits, exponent rebias 127-7
    const uint32_t norm = (mag << 4) + (120u << 7);
    // subnormal (exponent field 0): M * 2^-9, exact in FP32, upper half is BF16
    const uint32_t sub = __builtin_bit_cast(uint32_t, (float)mag * 0.001953125f) >> 16;
    uint32_t r = mag >= 8u ? norm : sub;
    if (mag == 0x7Fu) r = 0x7FC0u;  // NaN
    return r | ((b & 0x80u) << 8);
}

template <>
struct LP<2> {
    typedef uint8_t G;
    typedef uint16_t L;
    typedef u32x2 GF;
    typedef u32x4 F;
    __device__ static inline F widen(GF v) {
        F r;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t w = v[h];
            r[2 * h] = e4m3_to_bf16_bits(w & 0xFFu) | (e4m3_to_bf16_bits((w >> 8) & 0xFFu) << 16);
            r[2 * h + 1] =
                e4m3_to_bf16_bits((w >> 16) & 0xFFu) | (e4m3_to_bf16_bits(w >> 24) << 16);
        }
        return r;
    }
    __device__ static inline L widen1(G v) { return (L)e4m3_to_bf16_bits(v); }
    __device__ static inline f32x4 mma(F a, F b, f32x4 c) { return LP<0>::mma(a, b, c); }
};

struct LpArgs {
    const void* D;
    const void* u;
    float* out;
    const float* inv_sD;
    const float* inv_su;
    int64_t nelem;
    int64_t ntiles;
    int nunit;
    int mblk;
    int panels_total;
    int ppg;
    int ngroups;
    int nstreams;
    int vec_in;
    int vec_out;
};

template <int FMT, int KS>
__device__ inline void lp_stage_panels(const typename LP<FMT>::G* __restrict__ D,
                                       typename LP<FMT>::L* dl, int p0, int np, int nunit,
                                       int mblk) {
    typedef typename LP<FMT>::L E;
    constexpr int KP = 32 * KS;
    constexpr int LDE = KP + 16 / (int)sizeof(E);
    const int total = np * 16 * KP;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int j = idx % KP;
        const int rr = idx / KP;
        const int panel = p0 + rr / 16;
        const int m = panel / mblk;
        const int i = (panel % mblk) * 16 + (rr % 16);
        E v = 0;
        if (i < nunit && j < nunit) v = LP<FMT>::widen1(D[((int64_t)m * nunit + i) * nunit + j]);
        dl[rr * LDE + j] = v;
    }
}

template <int FMT, int KS>
__device__ inline void lp_load_b(const typename LP<FMT>::G* __restrict__ u, int64_t e, int g,
                                 const LpArgs& a, typename LP<FMT>::F (&b)[KS]) {
    typedef typename LP<FMT>::G E;
    typedef typename LP<FMT>::GF F;
    constexpr int KQ = 8 * KS;
    const bool ev = e < a.nelem;
    const E* row = u + (ev ? e : 0) * a.nunit + g * KQ;
    if (a.vec_in) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            F v = F(0u);
            if (ev && g * KQ + 8 * s < a.nunit) v = *reinterpret_cast<const F*>(row + 8 * s);
            b[s] = LP<FMT>::widen(v);
        }
    } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            E tmp[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                tmp[t] = (ev && g * KQ + 8 * s + t < a.nunit) ? row[8 * s + t] : E(0);
            b[s] = LP<FMT>::widen(__builtin_bit_cast(F, tmp));
        }
    }
}

// Operator panels p_lo .. p_lo+np-1 against the element fragments b of one
// tile; results scaled and stored.  PAIR: two consecutive panels of one
// output slab at a time (np pairs never straddle a slab: panels per slab and
// per group are even), lanes c and c^8 trading halves (a DPP rotation by 8
// within each 16-lane row) so that one store covers elements 0..7 and the
// other 8..15, each element's 32 nodes i0 .. i0+31 in one 128-byte run.
template <int FMT, int KS, int CB, bool PAIR>
__device__ inline void lp_panels(const typename LP<FMT>::F (&b)[CB][KS], const float (&esc)[CB],
                                 int64_t e0, int c, int g, int p_lo, int np,
                                 const typename LP<FMT>::L* dl, const float* s_inv_sD,
                                 const LpArgs& a) {
    typedef typename LP<FMT>::L E;
    typedef typename LP<FMT>::F F;
    constexpr int KQ = 8 * KS;
    constexpr int KP = 4 * KQ;
    constexpr int LDE = KP + 16 / (int)sizeof(E);
    const int nunit = a.nunit;
    int pp = 0;
    if constexpr (PAIR) {
        for (; pp + 1 < np; pp += 2) {
            const int panel = p_lo + pp;
            const int m = panel / a.mblk;
            const int i0 = (panel % a.mblk) * 16;
            f32x4 accA[CB], accB[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                accA[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
                accB[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            const E* arowA = dl + (pp * 16 + c) * LDE + g * KQ;
            const E* arowB = arowA + 16 * LDE;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const F avA = *reinterpret_cast<const F*>(arowA + 8 * s);
                const F avB = *reinterpret_cast<const F*>(arowB + 8 * s);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    accA[cb] = LP<FMT>::mma(avA, b[cb][s], accA[cb]);
                    accB[cb] = LP<FMT>::mma(avB, b[cb][s], accB[cb]);
                }
            }
            const float msc = s_inv_sD[m];
            const bool lo = c < 8;
            const int i = i0 + (lo ? 0 : 16) + 4 * g;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                // scale with the lane's own element before the exchange
                const float sc = msc * esc[cb];
                const f32x4 vA = accA[cb] * sc;
                const f32x4 vB = accB[cb] * sc;
                f32x4 x1, x2;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float send = lo ? vB[r] : vA[r];
                    const float got = __builtin_bit_cast(
                        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, send),
                                                           0x128 /* row_ror:8 */, 0xF, 0xF, false));
                    x1[r] = lo ? vA[r] : got;
                    x2[r] = lo ? got : vB[r];
                }
                const int64_t e1 = e0 + cb * 16 + (c & 7);
                const int64_t e2 = e1 + 8;
                if (i < nunit) {
                    if (e1 < a.nelem)
                        *reinterpret_cast<f32x4*>(a.out + ((int64_t)m * a.nelem + e1) * nunit + i) = x1;
                    if (e2 < a.nelem)
                        *reinterpret_cast<f32x4*>(a.out + ((int64_t)m * a.nelem + e2) * nunit + i) = x2;
                }
            }
        }
    }
    for (; pp < np; ++pp) {
        const int panel = p_lo + pp;
        const int m = panel / a.mblk;
        const int i0 = (panel % a.mblk) * 16;
        f32x4 acc[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const E* arow = dl + (pp * 16 + c) * LDE + g * KQ;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const F av = *reinterpret_cast<const F*>(arow + 8 * s);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[cb] = LP<FMT>::mma(av, b[cb][s], acc[cb]);
        }
        const float msc = s_inv_sD[m];
        const int i = i0 + 4 * g;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int64_t e = e0 + cb * 16 + c;
            if (e >= a.nelem) continue;
            const float sc = msc * esc[cb];  // product of powers of two: exact
            const f32x4 v = acc[cb] * sc;
            float* dst = a.out + ((int64_t)m * a.nelem + e) * nunit + i;
            if (a.vec_out) {
                if (i < nunit) *reinterpret_cast<f32x4*>(dst) = v;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (i + r < nunit) dst[r] = v[r];
            }
        }
    }
}

// up to 8 waves per work-group while the element operand (KS*CB 16-byte
// fragments) takes at most 56 registers
template <int KS, int CB>
constexpr int lp_max_threads() {
    return KS * CB <= 14 ? 512 : 256;
}

template <int FMT, int KS, int CB, bool PAIR>
__global__ void __launch_bounds__((lp_max_threads<KS, CB>())) dg_lowp_kernel(LpArgs a) {
    typedef typename LP<FMT>::L E;
    typedef typename LP<FMT>::G GE;
    typedef typename LP<FMT>::F F;
    constexpr int KQ = 8 * KS;
    constexpr int KP = 4 * KQ;
    constexpr int LDE = KP + 16 / (int)sizeof(E);

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    E* dl = reinterpret_cast<E*>(smem);
    const GE* __restrict__ D = static_cast<const GE*>(a.D);
    const GE* __restrict__ u = static_cast<const GE*>(a.u);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int nunit = a.nunit;

    const int xcd = blockIdx.x & 7;
    const int k = blockIdx.x >> 3;
    const int pg = k % a.ngroups;
    const int64_t stream = (int64_t)(k / a.ngroups) * 8 + xcd;
    const int p_lo = pg * a.ppg;
    const int np = min(a.ppg, a.panels_total - p_lo);
    lp_stage_panels<FMT, KS>(D, dl, p_lo, np, nunit, a.mblk);
    // operator scales in LDS: a global load inside the panel loop would make
    // every panel wait for all earlier stores (one counter covers loads and
    // stores), serialising the loop
    __shared__ float s_inv_sD[8];
    if (threadIdx.x < 8) s_inv_sD[threadIdx.x] = (a.inv_sD && (int)threadIdx.x * a.mblk < a.panels_total)
                                                     ? a.inv_sD[threadIdx.x] : 1.0f;
    __syncthreads();

    const int64_t tile_elems = (int64_t)nw * 16 * CB;
    for (int64_t tile = stream; tile < a.ntiles; tile += a.nstreams) {
        const int64_t e0 = tile * tile_elems + (int64_t)wave * 16 * CB;
        if (e0 >= a.nelem) continue;
        F b[CB][KS];
        float esc[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int64_t e = e0 + cb * 16 + c;
            lp_load_b<FMT, KS>(u, e, g, a, b[cb]);
            esc[cb] = (a.inv_su && e < a.nelem) ? a.inv_su[e] : 1.0f;
        }
        lp_panels<FMT, KS, CB, PAIR>(b, esc, e0, c, g, p_lo, np, dl, s_inv_sD, a);
    }
}

typedef void (*lp_fn)(LpArgs);

template <int FMT, int CB>
lp_fn pick_lp(int ks, bool pair) {
    switch (ks) {
#define X(K) \
    case K: return pair ? dg_lowp_kernel<FMT, K, CB, true> : dg_lowp_kernel<FMT, K, CB, false>;
        X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    }
    return nullptr;
}

constexpr size_t kLpBudget = 80 * 1024;
constexpr size_t kLpMax = 160 * 1024;

lp_fn lp_kernel(int fmt, int ks, int cb, bool pair) {
    if (fmt == 0) return cb == 4 ? pick_lp<0, 4>(ks, pair) : cb == 2 ? pick_lp<0, 2>(ks, pair) : pick_lp<0, 1>(ks, pair);
    if (fmt == 1) return cb == 4 ? pick_lp<1, 4>(ks, pair) : cb == 2 ? pick_lp<1, 2>(ks, pair) : pick_lp<1, 1>(ks, pair);
    return cb == 4 ? pick_lp<2, 4>(ks, pair) : cb == 2 ? pick_lp<2, 2>(ks, pair) : pick_lp<2, 1>(ks, pair);
}

}  // namespace

int lp_format(dg_dtype in_t, const dg_tile* tile) {
    const bool native = tile && (tile->flags & DG_TILE_FP8_NATIVE);
    return (in_t == DG_BF16) ? 0 : native ? 1 : 2;
}

dg_status make_lp_plan(int fmt, int nmat, int64_t nelem, int nunit, const dg_tile* tile, int per_cu,
                       int num_cu, LpPlan* P) {
    P->fmt = fmt;
    P->ks = (int)ceil_div(nunit, 32);
    if (P->ks > 16) return fail(DG_EUNSUPPORTED, "nunit too large");
    // defaults measured at p = 5 (2^20 elements): BF16 one column block, FP8
    // two, both with 8 waves per work-group where the variant allows it
    const int epw = (tile && tile->elems_per_wave) ? tile->elems_per_wave : (fmt == 0 ? 16 : 32);
    if (epw == 16) P->cb = 1;
    else if (epw == 32) P->cb = 2;
    else if (epw == 64 && P->ks <= 8) P->cb = 4;
    else return fail(DG_EINVAL, "tile.elems_per_wave must be 16, 32 (or 64 for nunit <= 256)");
    const int wdef = P->ks * P->cb <= 14 ? 8 : 4;  // lp_max_threads() allows 512 threads
    P->waves = (tile && tile->waves) ? tile->waves : wdef;
    if (P->waves < 1 || P->waves > 8) return fail(DG_EINVAL, "tile.waves must be in 1..8");
    P->lds_esz = fmt == 1 ? 1 : 2;
    P->mblk = (int)ceil_div(nunit, 16);
    P->panels_total = nmat * P->mblk;
    P->panel_bytes = (size_t)16 * (32 * P->ks * P->lds_esz + 16);
    int ppg;
    if (tile && tile->d_panels > 0) {
        ppg = std::min(tile->d_panels, P->panels_total);
    } else if ((size_t)P->panels_total * P->panel_bytes <= kLpBudget) {
        ppg = P->panels_total;
    } else {
        const int fit = std::max<int>(1, (int)(kLpMax / P->panel_bytes));
        const int groups = (int)ceil_div(P->panels_total, fit);
        ppg = (int)ceil_div(P->panels_total, groups);
    }
    P->ppg = ppg;
    P->ngroups = (int)ceil_div(P->panels_total, ppg);
    P->smem = (size_t)ppg * P->panel_bytes;
    if (P->smem > kLpMax) return fail(DG_EINVAL, "tile.d_panels exceeds the 160 KB LDS");
    P->ntiles = ceil_div(nelem, (int64_t)16 * P->cb * P->waves);
    const int64_t cap = std::max<int64_t>(1, (int64_t)per_cu * num_cu / (8 * P->ngroups));
    P->slots = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(P->ntiles, 8)));
    P->grid = 8 * P->ngroups * P->slots;
    return DG_OK;
}

// Paired stores (lp_panels) for rows of a multiple of 32 nodes written as
// 16-byte vectors, with an even number of panels per group.
bool lp_pair_ok(const LpPlan& P, int nunit, bool vec_out) {
    return vec_out && nunit % 32 == 0 && P.mblk % 2 == 0 && P.ppg % 2 == 0;
}

static dg_status lp_occupancy(const LpPlan& P, bool pair, int* per_cu) {
    lp_fn fn = lp_kernel(P.fmt, P.ks, P.cb, pair);
    if (!fn) return fail(DG_EUNSUPPORTED, "no low-precision DG kernel instance");
    hipFuncAttributes fa;
    DG_HIP_CHECK(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(fn)));
    if (64 * P.waves > fa.maxThreadsPerBlock)
        return fail(DG_EINVAL, "tile.waves above 4 needs a shape whose element data fit 64 registers");
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
    DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void*>(fn),
                                                              64 * P.waves, P.smem));
    if (*per_cu < 1) *per_cu = 1;
    return DG_OK;
}

dg_status resolve_forward_lowp(dg_dtype in_t, int nmat, int64_t nelem, int nunit, dg_tile* tile) {
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    LpPlan P;
    st = make_lp_plan(lp_format(in_t, tile), nmat, nelem, nunit, tile, 1, dev.num_cu, &P);
    if (st != DG_OK) return st;
    tile->waves = P.waves;
    tile->elems_per_wave = 16 * P.cb;
    tile->d_panels = P.ppg;
    if (tile->groups_per_cu == 0) {
        int per_cu = 0;
        // the kernel a launch into 16-byte aligned output would take
        st = lp_occupancy(P, lp_pair_ok(P, nunit, nunit % 4 == 0), &per_cu);
        if (st != DG_OK) return st;
        tile->groups_per_cu = per_cu;
    }
    return DG_OK;
}

dg_status launch_dg_forward_lowp(dg_dtype in_t, int nmat, int64_t nelem, int nunit, const void* D,
                                 const void* u, void* out, const float* inv_sD,
                                 const float* inv_su, const dg_tile* tile, hipStream_t s) {
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    LpPlan P;
    st = make_lp_plan(lp_format(in_t, tile), nmat, nelem, nunit, tile, 1, dev.num_cu, &P);
    if (st != DG_OK) return st;
    const bool vec_out = (nunit % 4 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    const bool pair = lp_pair_ok(P, nunit, vec_out);
    int per_cu = (tile && tile->groups_per_cu > 0) ? tile->groups_per_cu : 0;
    if (per_cu == 0) {
        st = lp_occupancy(P, pair, &per_cu);
        if (st != DG_OK) return st;
    }
    st = make_lp_plan(P.fmt, nmat, nelem, nunit, tile, per_cu, dev.num_cu, &P);
    if (st != DG_OK) return st;
    lp_fn fn = lp_kernel(P.fmt, P.ks, P.cb, pair);
    if (!fn) return fail(DG_EUNSUPPORTED, "no low-precision DG kernel instance");
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
    LpArgs a;
    a.D = D;
    a.u = u;
    a.out = static_cast<float*>(out);
    a.inv_sD = inv_sD;
    a.inv_su = inv_su;
    a.nelem = nelem;
    a.ntiles = P.ntiles;
    a.nunit = nunit;
    a.mblk = P.mblk;
    a.panels_total = P.panels_total;
    a.ppg = P.ppg;
    a.ngroups = P.ngroups;
    a.nstreams = (int)(8 * P.slots);
    a.vec_in = (nunit % 8 == 0) && (reinterpret_cast<uintptr_t>(u) % 16 == 0);  // 8 values / load
    a.vec_out = vec_out;
    hipLaunchKernelGGL(fn, dim3((unsigned)P.grid), dim3(64 * P.waves), P.smem, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
