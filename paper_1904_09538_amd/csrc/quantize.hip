// Quantisation of FP32 operands for the low-precision DG path.
//
//   BF16:      q = RNE(x) to bfloat16 (upper half of the FP32 encoding), NaN kept
//              quiet, overflow to infinity; inverse scales (if requested) are 1.
//   FP8 E4M3:  q = RNE(x * s) to OCP E4M3FN (bias 7, max 448, no infinities),
//              magnitudes past 448 saturate, NaN stays NaN; s is the largest
//              power of two with amax * s <= 448 (s = 1 when amax is 0 or not
//              finite; at most 2^127; NaN entries are ignored), chosen per row
//              (per_row = 1) or for the whole array; inv_scale = 1/s.  Scaling by a power of two is exact, so the
//              de-scaling in the DG epilogue is exact too.
//
// Rows up to 1024 values: one wave per row held in registers (below).  Longer
// rows: one wave per row, a max-reduction over the row (order-independent,
// exact), then the encode pass reading the row again.  One scale for the
// whole array (FP8): the maximum over the whole grid (an integer atomic
// maximum of |x|'s bit pattern, which orders non-negative floats, taken in
// inv_scale[0] itself), then an encode pass over the grid, then inv_scale[0]
// is replaced by 1/s.  Every path's launch shape is a pure function of the
// sizes (quant_plan), shared with the feature counter.
#include "common.hpp"

namespace dg {
namespace {

__device__ inline uint32_t f32_bits(float f) { return __builtin_bit_cast(uint32_t, f); }

__device__ inline uint16_t bf16_rne(float f) { return round_bf16(f); }

// E4M3FN encode of an FP32 value by its bit fields.
__device__ inline uint8_t e4m3_rne(float f) {
    const uint32_t b = f32_bits(f);
    const uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
    const uint32_t a = b & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return sign | 0x7F;          // NaN
    if (a >= 0x43E00000u) return sign | 0x7E;         // |f| >= 448 (incl. inf): saturate
    const int e = (int)(a >> 23) - 127;               // unbiased exponent (normal FP32)
    if (e < -6) {
        // E4M3 subnormal range: integer multiple of 2^-9, RNE by the hardware
        // round-to-nearest-even of an exactly scaled value
        const float m = __builtin_rintf(__builtin_bit_cast(float, a) * 512.0f);
        return sign | (uint8_t)m;                     // m in 0..8; 8 is the smallest normal
    }
    // keep 3 of the 23 mantissa bits, ties to even; a carry bumps the exponent
    uint32_t t = a + 0x7FFFFu + ((a >> 20) & 1u);
    const uint32_t E = (t >> 23) - 127 + 7;
    const uint32_t M = (t >> 20) & 7u;
    uint32_t code = (E << 3) | M;
    if (code > 0x7E) code = 0x7E;
    return sign | (uint8_t)code;
}

// Exponent k of the largest power of two s = 2^k with amax * s <= 448, from
// the exponent and mantissa of amax (exact; no division).  k <= 127.
__device__ inline int pow2_scale_exp_448(float amax) {
    const uint32_t a = f32_bits(amax) & 0x7FFFFFFFu;
    if (a == 0 || a >= 0x7F800000u) return 0;
    int E;
    uint32_t mant;
    if ((a >> 23) == 0) {  // FP32 subnormal amax: normalise
        const int lz = __builtin_clz(a) - 8;
        E = -126 - lz;
        mant = (a << lz) & 0x7FFFFFu;
    } else {
        E = (int)(a >> 23) - 127;
        mant = a & 0x7FFFFFu;
    }
    // amax = 1.mant * 2^E and 448 = 1.75 * 2^8 (0x600000 is the mantissa of 1.75)
    const int k = (mant <= 0x600000u) ? 8 - E : 7 - E;
    return k > 127 ? 127 : k;
}

// 2^k as an FP32 bit pattern, k in [-149, 127] (subnormal results built
// directly, so no flush-to-zero can touch them).
__device__ inline float exp2_bits(int k) {
    if (k >= -126) return __builtin_bit_cast(float, (uint32_t)(k + 127) << 23);
    return __builtin_bit_cast(float, 1u << (k + 149));
}

__device__ inline float wave_max(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void __launch_bounds__(256) quantize_rows_kernel(int to_fp8, int64_t rows, int64_t cols,
                                                           const float* __restrict__ x,
                                                           void* __restrict__ q,
                                                           float* __restrict__ inv_scale) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < rows; r += nwaves) {
        const float* xr = x + r * cols;
        if (!to_fp8) {
            uint16_t* qr = static_cast<uint16_t*>(q) + r * cols;
            for (int64_t c = lane; c < cols; c += 64) qr[c] = bf16_rne(xr[c]);
            if (inv_scale && lane == 0) inv_scale[r] = 1.0f;
            continue;
        }
        float amax = 0.0f;
        for (int64_t c = lane; c < cols; c += 64) {
            const float v = fabsf(xr[c]);
            amax = v > amax ? v : amax;   // NaN entries do not take part in the scale
        }
        amax = wave_max(amax);
        const int ks = pow2_scale_exp_448(amax);
        const float s = exp2_bits(ks);
        uint8_t* qr = static_cast<uint8_t*>(q) + r * cols;
        for (int64_t c = lane; c < cols; c += 64) qr[c] = e4m3_rne(xr[c] * s);
        if (lane == 0) inv_scale[r] = exp2_bits(-ks);
    }
}

// Rows of at most 256*NV values (every element row of the DG operands), held
// in registers between the max pass and the encode pass: a row takes SW
// lanes (SW = 64 for rows over 256 values), lane t of the row owning values
// 4(t + 64k) .. +3, k < NV, so a wave holds 64 / SW consecutive rows (a
// "slot"); loads are 16-byte vectors from any 4-byte boundary and each lane
// writes its four codes with one store.  A wave takes four slots per step so
// that the later slots' loads are in flight while the first is reduced and
// encoded.
typedef float f4v __attribute__((ext_vector_type(4)));

// Four E4M3FN codes: the hardware FP32-to-FP8 conversion (round to nearest
// even, subnormals included) for |y| < 448; the format's saturation (|y| >=
// 448, infinities included) and the NaN code are set here rather than taken
// from the instruction.  Bit-equal to the encoder by bit fields above (tests:
// random FP32 bit patterns, special values).
__device__ inline void e4m3_rne4(f4v y, uint8_t (&b)[4]) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], w, true);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint8_t code = (uint8_t)((uint32_t)w >> (8 * t));
        if (!(fabsf(y[t]) < 448.0f)) {
            const uint8_t sign = (uint8_t)((f32_bits(y[t]) >> 24) & 0x80u);
            code = sign | (y[t] != y[t] ? 0x7F : 0x7E);
        }
        b[t] = code;
    }
}


__device__ inline f4v load4_any(const float* p, int avail) {
    f4v v = {0.f, 0.f, 0.f, 0.f};
    if (avail >= 4) {
        __builtin_memcpy(&v, p, 16);
    } else {
        for (int t = 0; t < 3; ++t)
            if (t < avail) v[t] = p[t];
    }
    return v;
}

// Maximum over the SW lanes of each row (SW a power of two; lanes of one row
// are SW consecutive lanes, so every exchange stays inside the row).
template <int SW>
__device__ inline float row_max(float v) {
#pragma unroll
    for (int off = SW / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// lane: the lane's index within its row (0 .. SW - 1)
template <int NV, int SW>
__device__ inline void quantize_short_row(int to_fp8, int64_t r, int64_t cols, const f4v (&v)[NV],
                                          void* __restrict__ q, float* __restrict__ inv_scale, int lane) {
    if (!to_fp8) {
        uint16_t* qr = static_cast<uint16_t*>(q) + r * cols;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t c = 4 * (lane + 64 * k);
            const int64_t avail = cols - c;
            if (avail <= 0) continue;
            uint16_t h[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) h[t] = bf16_rne(v[k][t]);
            if (avail >= 4) {
                __builtin_memcpy(qr + c, h, 8);
            } else {
                for (int t = 0; t < 3; ++t)
                    if (t < avail) qr[c + t] = h[t];
            }
        }
        if (inv_scale && lane == 0) inv_scale[r] = 1.0f;
        return;
    }
    float amax = 0.0f;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float a = fabsf(v[k][t]);
            amax = a > amax ? a : amax;  // NaN entries do not take part in the scale
        }
    amax = row_max<SW>(amax);
    const int ks = pow2_scale_exp_448(amax);
    const float sc = exp2_bits(ks);
    uint8_t* qr = static_cast<uint8_t*>(q) + r * cols;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int64_t c = 4 * (lane + 64 * k);
        const int64_t avail = cols - c;
        if (avail <= 0) continue;
        uint8_t b[4];
        e4m3_rne4(v[k] * sc, b);
        if (avail >= 4) {
            __builtin_memcpy(qr + c, b, 4);
        } else {
            for (int t = 0; t < 3; ++t)
                if (t < avail) qr[c + t] = b[t];
        }
    }
    if (lane == 0) inv_scale[r] = exp2_bits(-ks);
}

// Slot b of the array holds rows b * (64 / SW) + (lane / SW); wave w takes
// slots w, w + W, w + 2W, w + 3W in one step, then w + 4W ... (W waves).
template <int NV, int SW>
__global__ void __launch_bounds__(256) quantize_short_rows_kernel(int to_fp8, int64_t rows, int64_t cols,
                                                                 const float* __restrict__ x,
                                                                 void* __restrict__ q,
                                                                 float* __restrict__ inv_scale) {
    static_assert(NV == 1 || SW == 64, "rows over 256 values take a whole wave");
    constexpr int RS = 4;            // slots in flight per wave
    constexpr int RPW = 64 / SW;     // rows per slot
    const int lane = threadIdx.x & 63;
    const int t = lane & (SW - 1), seg = lane / SW;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nslots = (rows + RPW - 1) / RPW;
    for (int64_t b0 = wave; b0 < nslots; b0 += RS * nwaves) {
        f4v v[RS][NV];
#pragma unroll
        for (int j = 0; j < RS; ++j) {
            const int64_t r = (b0 + j * nwaves) * RPW + seg;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int64_t c = 4 * (t + 64 * k);
                v[j][k] = r < rows ? load4_any(x + r * cols + c, (int)min<int64_t>(cols - c, 4))
                                   : f4v{0.f, 0.f, 0.f, 0.f};
            }
        }
#pragma unroll
        for (int j = 0; j < RS; ++j) {
            const int64_t r = (b0 + j * nwaves) * RPW + seg;
            // whole rows drop out past the end: the reduction's exchanges stay
            // inside a row, so the remaining rows' lanes never read them
            if (r < rows) quantize_short_row<NV, SW>(to_fp8, r, cols, v[j], q, inv_scale, t);
        }
    }
}

// ---- one scale for the whole array (FP8): four launches on the stream.
// inv_scale[0] holds the bit pattern of amax between the first and the last.

__global__ void __launch_bounds__(64) quantize_global_init(uint32_t* amax_bits) {
    if (threadIdx.x == 0) *amax_bits = 0u;
}

// Values i of the flat array taken by a thread: 4-value vectors 4*(gid + k*stride)
// while a whole vector fits (the array is 16-byte aligned), then the tail
// value by value (threads 0 .. N%4-1 of the grid).
template <bool VEC>
__global__ void __launch_bounds__(256) quantize_global_amax(const float* __restrict__ x, int64_t N,
                                                            uint32_t* amax_bits) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float amax = 0.0f;
    int64_t tail = 0;
    if (VEC) {
        const int64_t nv = N / 4;
        for (int64_t v = gid; v < nv; v += stride) {
            f4v t;
            __builtin_memcpy(&t, x + 4 * v, 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float a = fabsf(t[q]);
                amax = a > amax ? a : amax;   // NaN entries do not take part
            }
        }
        tail = 4 * nv;
    }
    for (int64_t i = tail + gid; i < N; i += stride) {
        const float a = fabsf(x[i]);
        amax = a > amax ? a : amax;
    }
    // the work-group's maximum (four wave maxima through LDS), then one
    // atomic per work-group: thousands of waves contending for one word
    // cost more than the pass itself on small arrays
    __shared__ float wmax[4];
    amax = wave_max(amax);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = wmax[0];
        for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        atomicMax(amax_bits, f32_bits(m));
    }
}

template <bool VEC>
__global__ void __launch_bounds__(256) quantize_global_encode(const float* __restrict__ x, int64_t N,
                                                              uint8_t* __restrict__ q,
                                                              const uint32_t* __restrict__ amax_bits) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int ks = pow2_scale_exp_448(__builtin_bit_cast(float, *amax_bits));
    const float sc = exp2_bits(ks);
    int64_t tail = 0;
    if (VEC) {
        const int64_t nv = N / 4;
        for (int64_t v = gid; v < nv; v += stride) {
            f4v t;
            __builtin_memcpy(&t, x + 4 * v, 16);
            uint8_t b[4];
            e4m3_rne4(t * sc, b);
            __builtin_memcpy(q + 4 * v, b, 4);
        }
        tail = 4 * nv;
    }
    for (int64_t i = tail + gid; i < N; i += stride) q[i] = e4m3_rne(x[i] * sc);
}

__global__ void __launch_bounds__(64) quantize_global_final(uint32_t* amax_bits_then_inv) {
    if (threadIdx.x == 0) {
        const int ks = pow2_scale_exp_448(__builtin_bit_cast(float, *amax_bits_then_inv));
        *reinterpret_cast<float*>(amax_bits_then_inv) = exp2_bits(-ks);
    }
}

__global__ void __launch_bounds__(64) quantize_set_one(float* inv_scale) {
    if (threadIdx.x == 0) *inv_scale = 1.0f;
}

}  // namespace

QuantPlan quant_plan(int fp8, int64_t rows, int64_t cols, int per_row) {
    QuantPlan P = {};
    P.rows = rows;
    P.cols = cols;
    if (!per_row && fp8) {
        P.kind = QuantPlan::kGlobal;
        P.blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows * cols, 1024), 1024));
        return P;
    }
    if (cols <= 1024) {
        // four row slots per wave and step; a slot is one row (sw = 64 lanes)
        // or, for rows of at most 256 values, 64 / sw consecutive rows of sw
        // lanes each (sw the smallest power of two with 4 sw >= cols);
        // measured at 2^20 rows of 216: BF16 is fastest with one step per
        // wave, FP8 with four (65536 waves)
        P.kind = QuantPlan::kShortRows;
        P.nv = cols <= 256 ? 1 : cols <= 512 ? 2 : 4;
        P.sw = 64;
        if (P.nv == 1)
            while (P.sw > 1 && 4 * (P.sw / 2) >= cols) P.sw /= 2;
        const int64_t slots = ceil_div(rows, 64 / P.sw);
        const int64_t waves = std::min<int64_t>(ceil_div(slots, 4), fp8 ? 65536 : 262144);
        P.blocks = ceil_div(waves, 4);
    } else {
        P.kind = QuantPlan::kRows;
        P.blocks = ceil_div(std::min<int64_t>(rows, 65536), 4);
    }
    return P;
}

dg_status launch_quantize(dg_dtype to, int64_t rows, int64_t cols, int per_row, const float* x,
                          void* q, float* inv_scale, hipStream_t s) {
    const int fp8 = to == DG_FP8E4M3 ? 1 : 0;
    const QuantPlan P = quant_plan(fp8, rows, cols, per_row);
    if (P.kind == QuantPlan::kGlobal) {
        const int64_t N = rows * cols;
        uint32_t* bits = reinterpret_cast<uint32_t*>(inv_scale);
        const bool vec = reinterpret_cast<uintptr_t>(x) % 16 == 0 && reinterpret_cast<uintptr_t>(q) % 4 == 0;
        hipLaunchKernelGGL(quantize_global_init, dim3(1), dim3(64), 0, s, bits);
        if (vec) {
            hipLaunchKernelGGL(quantize_global_amax<true>, dim3((unsigned)P.blocks), dim3(256), 0, s, x, N, bits);
            hipLaunchKernelGGL(quantize_global_encode<true>, dim3((unsigned)P.blocks), dim3(256), 0, s, x, N,
                               static_cast<uint8_t*>(q), bits);
        } else {
            hipLaunchKernelGGL(quantize_global_amax<false>, dim3((unsigned)P.blocks), dim3(256), 0, s, x, N, bits);
            hipLaunchKernelGGL(quantize_global_encode<false>, dim3((unsigned)P.blocks), dim3(256), 0, s, x, N,
                               static_cast<uint8_t*>(q), bits);
        }
        hipLaunchKernelGGL(quantize_global_final, dim3(1), dim3(64), 0, s, bits);
        DG_HIP_CHECK(hipGetLastError());
        return DG_OK;
    }
    // per-row scales, or BF16 (whose codes need no scale): one inverse scale
    // per row is written by the row kernels only when per_row is set
    float* inv_rows = per_row ? inv_scale : nullptr;
    if (P.kind == QuantPlan::kShortRows) {
        void (*k)(int, int64_t, int64_t, const float*, void*, float*) = nullptr;
        if (P.nv == 2) k = quantize_short_rows_kernel<2, 64>;
        else if (P.nv == 4) k = quantize_short_rows_kernel<4, 64>;
        else if (P.sw == 64) k = quantize_short_rows_kernel<1, 64>;
        else if (P.sw == 32) k = quantize_short_rows_kernel<1, 32>;
        else if (P.sw == 16) k = quantize_short_rows_kernel<1, 16>;
        else if (P.sw == 8) k = quantize_short_rows_kernel<1, 8>;
        else if (P.sw == 4) k = quantize_short_rows_kernel<1, 4>;
        else if (P.sw == 2) k = quantize_short_rows_kernel<1, 2>;
        else k = quantize_short_rows_kernel<1, 1>;
        hipLaunchKernelGGL(k, dim3((unsigned)P.blocks), dim3(256), 0, s, fp8, rows, cols, x, q, inv_rows);
    } else {
        hipLaunchKernelGGL(quantize_rows_kernel, dim3((unsigned)P.blocks), dim3(256), 0, s, fp8, rows, cols, x,
                           q, inv_rows);
    }
    if (!per_row && inv_scale) hipLaunchKernelGGL(quantize_set_one, dim3(1), dim3(64), 0, s, inv_scale);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
