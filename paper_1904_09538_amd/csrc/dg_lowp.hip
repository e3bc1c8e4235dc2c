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
#include <type_traits>

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

// Eight E4M3FN values (two words) to eight BF16 values on gfx950's packed
// conversion (two values per instruction, scale 1): the same bits as
// e4m3_to_bf16_bits for every finite code, NaN for NaN.
__device__ inline u32x4 e4m3x8_to_bf16x8(u32x2 v) {
    u32x4 r;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        r[2 * h] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[h], 1.0f, false));
        r[2 * h + 1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[h], 1.0f, true));
    }
    return r;
}

template <>
struct LP<2> {
    typedef uint8_t G;
    typedef uint16_t L;
    typedef u32x2 GF;
    typedef u32x4 F;
    __device__ static inline F widen(GF v) { return e4m3x8_to_bf16x8(v); }
    __device__ static inline L widen1(G v) { return (L)e4m3_to_bf16_bits(v); }
    __device__ static inline f32x4 mma(F a, F b, f32x4 c) { return LP<0>::mma(a, b, c); }
};

// 3  BF16 operator; element data FP32 in HBM, rounded to BF16 as the staged
//    body copies them into LDS (DG_TILE_QUANT_U): the operator loads follow
//    format 0.  The eight values of a chunk are kept as their FP32 bit
//    patterns and rounded on the bits.  (A __builtin_bit_cast applied to a
//    vector component, bit_cast(float, v[i]), read component 0 whatever i
//    with this compiler, in the assembly; values leave a vector by value,
//    through a function parameter or an element copy, before any bit cast.)
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

template <>
struct LP<3> {
    typedef float G;
    typedef uint16_t L;
    typedef u32x8 GF;
    typedef u32x4 F;
    __device__ static inline F widen(GF v) {
        u32x4 r;
#pragma unroll
        for (int h = 0; h < 4; ++h)
            r[h] = (uint32_t)round_bf16_bits(v[2 * h]) | ((uint32_t)round_bf16_bits(v[2 * h + 1]) << 16);
        return r;
    }
    __device__ static inline L widen1(G v) { return round_bf16(v); }
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

// ---------------------------------------------------------------- staged body
// Operator rows in registers; element tiles and result rows staged in LDS.
//
// A work-group owns rb = waves x PW consecutive 16-row blocks of one operator
// slab m (a row group, rows r0 .. r0 + rows_g); each wave keeps the MFMA A
// fragments of its PW blocks in registers for the whole launch (PW x KS x 4
// registers).  Per tile of 16 CB consecutive elements:
//   - the tile's element rows, contiguous in HBM, are copied into LDS in
//     fragment order (chunk row j = 8-node chunk, one 16-byte BF16 vector
//     per element; FP8 widened to BF16 on the way), their scales beside;
//   - every wave multiplies its blocks (C^T = D_rows U^T on 16x16x32 BF16
//     MFMA tiles, the k-steps in the same order as the LDS-panel body) and
//     writes the scaled results into an LDS copy of the tile's output rows;
//   - after one barrier the work-group writes those rows with 16-byte
//     stores: rows_g x 4 contiguous bytes per element, and one contiguous
//     block of 16 CB x nunit x 4 bytes when the row group is the whole row.
// Element rows are loaded into registers two tiles ahead (two register
// sets), so each load has a whole loop iteration to arrive, and are copied to
// the LDS buffer the tile after next will read; one barrier per tile orders
// everything (two element and two result buffers).

// word 3 of a raw buffer resource on gfx9-family parts (32-bit data format,
// no swizzle): range-checked loads and stores on plain byte offsets
constexpr int kBufferWord3 = 0x00020000;
// cache policy of the staged body's output stores: non-temporal at system
// scope (nt sc0 sc1), streamed past the L2.  The kernel never reads its
// output, and keeping it out of the L2 keeps resident the element tiles the
// other operator groups re-read (measured at p = 5, 2^20 elements: FP8
// 0.76 -> 0.54 ms)
constexpr int kStreamStore = 2 | 1 | 16;

struct LsArgs {
    const void* D;
    const void* u;
    float* out;
    const float* inv_sD;
    const float* inv_su;
    int64_t nelem;
    int64_t ntiles;
    int nunit;
    int mblk;
    int rb;        // row blocks per work-group
    int nrg;       // row groups per slab
    int ngroups;   // nmat x nrg
    int nstreams;
    int upitch;    // bytes per chunk row of an element buffer (16 CB elements + pad)
};

// up to 16 waves per work-group (128 registers per lane); shapes with two
// column blocks and two row blocks per wave take at most 8 (256 registers)
template <int CB, int PW>
constexpr int ls_max_threads() {
    return CB == 2 && PW == 2 ? 512 : 1024;
}

template <int FMT, int KS, int CB, int PW>
__global__ void __launch_bounds__((ls_max_threads<CB, PW>())) dg_lowp_staged_kernel(LsArgs a) {
    typedef typename LP<FMT>::G GE;     // element data in HBM
    typedef typename LP<FMT>::GF GF;
    constexpr int DFMT = FMT == 3 ? 0 : FMT;   // the operator's format
    typedef typename LP<DFMT>::G DE;
    typedef typename LP<DFMT>::GF DGF;
    typedef u32x4 F;   // BF16 fragment (FP8 widened)
    constexpr int KQ = 8 * KS;
    constexpr int TE = 16 * CB;   // elements per tile

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int c = lane & 15;
    const int g = lane >> 4;
    const int nunit = a.nunit;

    const int xcd = blockIdx.x & 7;
    const int k = blockIdx.x >> 3;
    const int gi = k % a.ngroups;
    const int m = gi / a.nrg;
    const int rg = gi % a.nrg;
    const int64_t stream = (int64_t)(k / a.ngroups) * 8 + xcd;
    if (stream >= a.ntiles) return;   // a work-group without tiles does nothing
    const int r0 = rg * a.rb * 16;
    const int rows_g = min(a.rb * 16, nunit - r0);
    const int nch_u = nunit / 8;    // 8-node chunks per element row
    const int nch_o = rows_g / 4;   // 4-row result chunks per element and row group

    const int usz = 4 * KS * a.upitch;          // bytes per element buffer
    const int osz = TE * a.rb * 16;             // floats per result buffer
    unsigned char* us = smem;
    float* os = reinterpret_cast<float*>(smem + 2 * usz);
    float* ssu = os + 2 * osz;

    // chunk rows past the element row stay zero (both buffers)
    {
        const int zrows = 4 * KS - nch_u;
        for (int idx = tid; idx < 2 * zrows * TE; idx += T) {
            const int b = idx / (zrows * TE);
            const int r = idx % (zrows * TE);
            *reinterpret_cast<u32x4*>(us + b * usz + (nch_u + r / TE) * a.upitch + (r % TE) * 16) = u32x4(0u);
        }
    }
    // this wave's operator rows: blocks lb = wave * PW + b of the row group
    int nbw = 0;
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        const int lb = wave * PW + b;
        if (lb < a.rb && r0 + lb * 16 < nunit) nbw = b + 1;
    }
    F A[PW][KS];
    {
        const DE* __restrict__ D = static_cast<const DE*>(a.D);
#pragma unroll
        for (int b = 0; b < PW; ++b) {
            const int i = r0 + (wave * PW + b) * 16 + c;
            const bool rowok = b < nbw && i < nunit;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int col = g * KQ + 8 * s;
                DGF v = DGF(0u);
                if (rowok && col < nunit)
                    v = *reinterpret_cast<const DGF*>(D + ((int64_t)m * nunit + i) * nunit + col);
                A[b][s] = LP<DFMT>::widen(v);
            }
        }
    }
    const float msc = a.inv_sD ? a.inv_sD[m] : 1.0f;
    constexpr int NI = ls_chunks_in(CB);
    constexpr int NO = ls_chunks_out(CB);
    // per-thread element chunk offsets, fixed for the launch (q = tid + kk T):
    // element chunk q -> LDS (chunk row q % nch_u, element q / nch_u)
    int uoff[NI];
#pragma unroll
    for (int kk = 0; kk < NI; ++kk) {
        const int q = tid + kk * T;
        uoff[kk] = (q % nch_u) * a.upitch + (q / nch_u) * 16;
    }
    // result chunk q: element q / nch_o, rows 4 (q % nch_o) of the group, at
    // this byte offset from the tile's first output row of the group (4 q
    // floats, one contiguous run, when the group is the whole row); chunks
    // past the tile's elements fall outside the store's buffer range
    int goff[NO];
#pragma unroll
    for (int kk = 0; kk < NO; ++kk) {
        const int q = tid + kk * T;
        goff[kk] = ((q / nch_o) * nunit + 4 * (q % nch_o)) * 4;
    }

    // Element loads and output stores are buffer operations whose range check
    // (out-of-range loads read 0, out-of-range stores are dropped) replaces
    // per-lane branches: every thread issues the same fixed number of them
    // per tile, so the compiler's wait for a tile's loads leaves the stores
    // and loads issued after them in flight.
    constexpr int CHB = (int)sizeof(GF);   // bytes of an 8-node chunk in HBM
    const GE* __restrict__ u = static_cast<const GE*>(a.u);
    unsigned char* dump = reinterpret_cast<unsigned char*>(ssu + 2 * TE) + tid * 16;
    struct Pf {
        GF v[NI];
        float s;
    };
    auto issue = [&](Pf& pf, int64_t tt) {
        const int64_t e0 = tt * TE;
        const int nel = (int)min<int64_t>(TE, a.nelem - e0);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<GE*>(u + e0 * nunit), 0, nel * nch_u * CHB, kBufferWord3);
#pragma unroll
        for (int kk = 0; kk < NI; ++kk) {
            if constexpr (CHB == 32) {
                const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(rs, (tid + kk * T) * CHB, 0, 0);
                const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(rs, (tid + kk * T) * CHB + 16, 0, 0);
                pf.v[kk] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            } else if constexpr (CHB == 16) {
                pf.v[kk] = __builtin_amdgcn_raw_buffer_load_b128(rs, (tid + kk * T) * CHB, 0, 0);
            } else {
                pf.v[kk] = __builtin_amdgcn_raw_buffer_load_b64(rs, (tid + kk * T) * CHB, 0, 0);
            }
        }
        // the element scales as a buffer of nel floats (none without scales:
        // every read out of range, 0, replaced by 1 at the commit)
        const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
            a.inv_su ? const_cast<float*>(a.inv_su + e0) : a.out, 0, a.inv_su ? nel * 4 : 0, kBufferWord3);
        pf.s = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rq, 4 * (tid % TE), 0, 0));
    };
    auto commit = [&](const Pf& pf, int b, int64_t tt) {
        const int nq = (int)min<int64_t>(TE, a.nelem - tt * TE) * nch_u;
        unsigned char* ub = us + b * usz;
#pragma unroll
        for (int kk = 0; kk < NI; ++kk) {
            const int q = tid + kk * T;
            *reinterpret_cast<u32x4*>(q < nq ? ub + uoff[kk] : dump) = LP<FMT>::widen(pf.v[kk]);
        }
        ssu[b * TE + tid % TE] = a.inv_su ? pf.s : 1.0f;   // every thread of a slot writes the same value
    };
    // NB valid row blocks: the k-steps' B fragments read ahead of the
    // products (all of them while registers allow, else one k-step at a time)
    auto multiply = [&](int b, auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        constexpr int AHEAD = KS * CB * PW <= 16 ? KS : 1;
        const unsigned char* ub = us + b * usz;
        f32x4 acc[NB][CB];
#pragma unroll
        for (int p = 0; p < NB; ++p)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[p][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s0 = 0; s0 < KS; s0 += AHEAD) {
            F bf[AHEAD][CB];
#pragma unroll
            for (int s = 0; s < AHEAD; ++s)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    bf[s][cb] = *reinterpret_cast<const F*>(ub + (g * KS + s0 + s) * a.upitch + (cb * 16 + c) * 16);
#pragma unroll
            for (int s = 0; s < AHEAD; ++s)
#pragma unroll
                for (int p = 0; p < NB; ++p)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[p][cb] = LP<0>::mma(A[p][s0 + s], bf[s][cb], acc[p][cb]);
        }
        float* ob = os + b * osz;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const float sc = msc * ssu[b * TE + cb * 16 + c];  // product of powers of two: exact
#pragma unroll
            for (int p = 0; p < NB; ++p) {
                const int row = (wave * PW + p) * 16 + 4 * g;
                if (row < rows_g)
                    *reinterpret_cast<f32x4*>(ob + (cb * 16 + c) * rows_g + row) = acc[p][cb] * sc;
            }
        }
    };
    auto multiply_tile = [&](int b) {
        if (nbw == PW) multiply(b, std::integral_constant<int, PW>{});
        else if (PW == 2 && nbw == 1) multiply(b, std::integral_constant<int, 1>{});
    };
    auto write = [&](int b, int64_t tt) {
        const int64_t e0 = tt * TE;
        const int nel = (int)min<int64_t>(TE, a.nelem - e0);
        const float* ob = os + b * osz;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            a.out + ((int64_t)m * a.nelem + e0) * nunit + r0, 0, (nel * nunit - r0) * 4, kBufferWord3);
        const int qmax = TE * nch_o - 1;
        f32x4 v[NO];
#pragma unroll
        for (int kk = 0; kk < NO; ++kk)
            v[kk] = *reinterpret_cast<const f32x4*>(ob + 4 * min(tid + kk * T, qmax));
#pragma unroll
        for (int kk = 0; kk < NO; ++kk)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v[kk]), rs, goff[kk], 0,
                                                   kStreamStore);
    };

    // the stream's tiles t_k = stream + k ns, k < K; indices past the end
    // repeat the last tile (their loads are re-reads into idle buffers)
    const int64_t ns = a.nstreams;
    const int64_t K = (a.ntiles - stream + ns - 1) / ns;
    auto tile_at = [&](int64_t k) { return stream + (k < K ? k : K - 1) * ns; };
    Pf pa, pb;
    // prologue: tile 0 staged; tiles 1 and 2 loading; tile 0 multiplied;
    // tile 1 staged
    issue(pa, tile_at(0));
    commit(pa, 0, tile_at(0));
    __syncthreads();
    issue(pb, tile_at(1));
    issue(pa, tile_at(2));
    multiply_tile(0);
    commit(pb, 1, tile_at(1));
    __syncthreads();
    // iteration k: results of tile k in result buffer k & 1, tile k + 1 in
    // element buffer (k + 1) & 1, tile k + 2 loading into `ahead`; load tile
    // k + 3 into `next`, store tile k, multiply tile k + 1, stage tile k + 2
    auto step = [&](int64_t k, Pf& ahead, Pf& next) {
        const int b = (int)(k & 1);
        issue(next, tile_at(k + 3));
        write(b, tile_at(k));
        multiply_tile(b ^ 1);
        commit(ahead, b, tile_at(k + 2));
        __syncthreads();
    };
    for (int64_t k = 0;; k += 2) {
        if (k + 1 >= K) {
            write((int)(k & 1), tile_at(k));
            break;
        }
        step(k, pa, pb);
        if (k + 2 >= K) {
            write((int)((k + 1) & 1), tile_at(k + 1));
            break;
        }
        step(k + 1, pb, pa);
    }
}

typedef void (*ls_fn)(LsArgs);

// two row blocks per wave only while their operator rows fit 64 registers
template <int FMT, int CB, int PW>
ls_fn pick_ls(int ks) {
    switch (ks) {
#define X(K) \
    case K: return dg_lowp_staged_kernel<FMT, K, CB, PW>;
        X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
    }
    if constexpr (PW == 1) {
        switch (ks) {
#define X(K) \
    case K: return dg_lowp_staged_kernel<FMT, K, CB, PW>;
            X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
        }
    }
    return nullptr;
}

ls_fn ls_kernel(int fmt, int ks, int cb, int pw) {
    if (fmt == 0) {
        if (cb == 1) return pw == 1 ? pick_ls<0, 1, 1>(ks) : pick_ls<0, 1, 2>(ks);
        return pw == 1 ? pick_ls<0, 2, 1>(ks) : pick_ls<0, 2, 2>(ks);
    }
    if (fmt == 2) {
        if (cb == 1) return pw == 1 ? pick_ls<2, 1, 1>(ks) : pick_ls<2, 1, 2>(ks);
        return pw == 1 ? pick_ls<2, 2, 1>(ks) : pick_ls<2, 2, 2>(ks);
    }
    if (fmt == 3 && cb == 1) return pw == 1 ? pick_ls<3, 1, 1>(ks) : pick_ls<3, 1, 2>(ks);
    return nullptr;
}

}  // namespace

int lp_format(dg_dtype in_t, const dg_tile* tile) {
    const bool native = tile && (tile->flags & DG_TILE_FP8_NATIVE);
    const bool fused = tile && (tile->flags & DG_TILE_QUANT_U);
    return (in_t == DG_BF16) ? (fused ? 3 : 0) : native ? 1 : 2;
}

// The staged body's plan (see dg_lowp_staged_kernel).  Defaults: one column
// block per tile, two row blocks per wave while the operator rows take at
// most 64 registers (KS <= 8), else one, and as many waves (up to 16) as
// cover one slab's row blocks.
static dg_status make_staged_plan(int nmat, int64_t nelem, int nunit, const dg_tile* tile, int per_cu,
                                  int num_cu, LpPlan* P) {
    const int epw = (tile && tile->elems_per_wave) ? tile->elems_per_wave : 16;
    if (epw == 16) P->cb = 1;
    else if (epw == 32) P->cb = 2;
    else return fail(DG_EINVAL, "tile.elems_per_wave must be 16 or 32 (elements per tile)");
    P->mblk = (int)ceil_div(nunit, 16);
    P->panels_total = nmat * P->mblk;
    const int pw_def = P->ks <= 8 ? 2 : 1;
    const int tw = tile ? tile->waves : 0, tp = tile ? tile->d_panels : 0;
    int W, pw;
    if (tw > 0 && tp > 0) {
        if (tp % tw) return fail(DG_EINVAL, "tile.d_panels must be 1 or 2 row blocks per wave");
        W = tw;
        pw = tp / tw;
    } else if (tp > 0) {
        pw = (tp % 2 == 0 && pw_def == 2) ? 2 : 1;
        W = tp / pw;
    } else if (tw > 0) {
        W = tw;
        pw = pw_def;
    } else {
        pw = pw_def;
        W = std::min<int>(16, (int)ceil_div(P->mblk, pw));
    }
    if (pw != 1 && pw != 2) return fail(DG_EINVAL, "tile.d_panels must be 1 or 2 row blocks per wave");
    if (pw == 2 && P->ks > 8) return fail(DG_EINVAL, "two row blocks per wave need nunit <= 256");
    if (W < 1 || W > 16) return fail(DG_EINVAL, "tile.waves must be in 1..16 for the staged body");
    if (pw == 2 && P->cb == 2 && W > 8)
        return fail(DG_EINVAL, "two row blocks and two column blocks per wave allow at most 8 waves");
    P->waves = W;
    P->pw = pw;
    P->rb = W * pw;
    P->nrg = (int)ceil_div(P->mblk, P->rb);
    const int tile_elems = 16 * P->cb;
    const int rows_max = std::min(P->rb * 16, nunit);
    if (tile_elems * (nunit / 8) > 64 * W * ls_chunks_in(P->cb) ||
        tile_elems * rows_max / 4 > 64 * W * ls_chunks_out(P->cb))
        return fail(DG_EINVAL, "too few waves to stage a tile of the staged body (nunit / 32 at least)");
    P->upitch = tile_elems * 16 + 16;
    P->lds_esz = 2;
    P->panel_bytes = 0;
    P->smem = (size_t)2 * 4 * P->ks * P->upitch + (size_t)2 * tile_elems * P->rb * 16 * 4 +
              (size_t)2 * tile_elems * 4 + (size_t)64 * W * 16;
    if (P->smem > 160 * 1024) return fail(DG_EINVAL, "staged body: tile exceeds the 160 KB LDS");
    P->ppg = P->rb;
    P->ngroups = nmat * P->nrg;
    P->ntiles = ceil_div(nelem, (int64_t)tile_elems);
    const int64_t cap = std::max<int64_t>(1, (int64_t)per_cu * num_cu / (8 * P->ngroups));
    P->slots = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(P->ntiles, 8)));
    P->grid = 8 * P->ngroups * P->slots;
    return DG_OK;
}

dg_status make_lp_plan(int fmt, int nmat, int64_t nelem, int nunit, const dg_tile* tile, int per_cu,
                       int num_cu, LpPlan* P, bool aligned) {
    P->fmt = fmt;
    P->ks = (int)ceil_div(nunit, 32);
    if (P->ks > 16) return fail(DG_EUNSUPPORTED, "nunit too large");
    P->staged = fmt != 1 && nunit % 8 == 0 && aligned && !(tile && (tile->flags & DG_TILE_LP_LDS_PANELS));
    P->pw = P->rb = P->nrg = P->upitch = 0;
    if (fmt == 3) {
        // the fused rounding lives in the staged body only
        if (!P->staged)
            return fail(DG_EUNSUPPORTED, "DG_TILE_QUANT_U needs the staged body (nunit % 8 == 0, 16-byte "
                                         "aligned arrays, no DG_TILE_LP_LDS_PANELS)");
        if (tile && tile->elems_per_wave && tile->elems_per_wave != 16)
            return fail(DG_EUNSUPPORTED, "DG_TILE_QUANT_U: one column block per tile (elems_per_wave 16)");
    }
    if (P->staged) return make_staged_plan(nmat, nelem, nunit, tile, per_cu, num_cu, P);
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
    if (P.staged) {
        ls_fn fn = ls_kernel(P.fmt, P.ks, P.cb, P.pw);
        if (!fn) return fail(DG_EUNSUPPORTED, "no staged low-precision DG kernel instance");
        DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
        DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            per_cu, reinterpret_cast<const void*>(fn), 64 * P.waves, P.smem));
        if (*per_cu < 1) *per_cu = 1;
        return DG_OK;
    }
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
    const bool aligned = reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(u) % 16 == 0 && reinterpret_cast<uintptr_t>(D) % 16 == 0;
    if (!aligned) {
        st = make_lp_plan(P.fmt, nmat, nelem, nunit, tile, 1, dev.num_cu, &P, false);
        if (st != DG_OK) return st;
    }
    const bool pair = lp_pair_ok(P, nunit, vec_out);
    int per_cu = (tile && tile->groups_per_cu > 0) ? tile->groups_per_cu : 0;
    if (per_cu == 0) {
        st = lp_occupancy(P, pair, &per_cu);
        if (st != DG_OK) return st;
    }
    st = make_lp_plan(P.fmt, nmat, nelem, nunit, tile, per_cu, dev.num_cu, &P, aligned);
    if (st != DG_OK) return st;
    if (P.staged) {
        ls_fn fn = ls_kernel(P.fmt, P.ks, P.cb, P.pw);
        if (!fn) return fail(DG_EUNSUPPORTED, "no staged low-precision DG kernel instance");
        DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
        LsArgs a;
        a.D = D;
        a.u = u;
        a.out = static_cast<float*>(out);
        a.inv_sD = inv_sD;
        a.inv_su = inv_su;
        a.nelem = nelem;
        a.ntiles = P.ntiles;
        a.nunit = nunit;
        a.mblk = P.mblk;
        a.rb = P.rb;
        a.nrg = P.nrg;
        a.ngroups = P.ngroups;
        a.nstreams = (int)(8 * P.slots);
        a.upitch = P.upitch;
        hipLaunchKernelGGL(fn, dim3((unsigned)P.grid), dim3(64 * P.waves), P.smem, s, a);
        DG_HIP_CHECK(hipGetLastError());
        return DG_OK;
    }
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
