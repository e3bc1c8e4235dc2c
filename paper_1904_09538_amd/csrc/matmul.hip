// Square matrix multiplication c = a b, FP32, on v_mfma_f32_16x16x4 (the
// paper's first example kernel, Section "Kernel Creation and Transformation").
//
// The matrix cores are fed the transposed product C^T = B^T A^T: the MFMA "A"
// operand comes from the b tile and its "B" operand from the a tile, so that
// the accumulator rows land on consecutive *columns* of c and every lane
// writes four consecutive floats of one c row (a 16-byte store).
//
// Tiling.  A work-group of 4 waves owns a 128x128 block of c (2x2 waves of
// 64x64 = 4x4 MFMA blocks each).  K advances in chunks of 16: the a chunk is
// staged in LDS as [row][k] (read with one 16-byte load per tile) and the b
// chunk as it lies in memory, [k][col] (read with one 4-byte load per tile and
// k-step; consecutive lanes take consecutive columns and the row stride puts
// lane groups g and g+1 sixteen banks apart).  Lane group g takes k = 4g..4g+3
// of the chunk, k-step s = 0..3 (any order of the contraction is exact up to
// rounding).  Both chunks are written with 16-byte LDS stores; transposing b
// on the way in (16 columns of one k landing on one bank) cost a 16-way bank
// conflict on every store.  The next chunk is loaded from global memory into
// registers while the current one is multiplied; LDS is double-buffered with
// one barrier per chunk.
#include "common.hpp"

namespace dg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;    // block rows / cols
constexpr int BK = 16;     // k chunk
constexpr int LDK = BK + 4;  // a chunk row stride (floats): 16-byte pad against bank conflicts
constexpr int LDB = BM + 4;  // b chunk row stride (floats)

template <bool VEC>
__device__ inline void load_chunk(const float* __restrict__ a, const float* __restrict__ b,
                                  int64_t n, int64_t row0, int64_t col0, int64_t k0, int t,
                                  f32x4 (&ra)[2], f32x4 (&rb)[2]) {
    // a: thread t loads row row0 + t/2, k = k0 + 8*(t%2) .. +7
    const int64_t ar = row0 + (t >> 1);
    const int64_t ak = k0 + 8 * (t & 1);
    // b: thread t loads k = k0 + t/16, cols col0 + 8*(t%16) .. +7
    const int64_t bk = k0 + (t >> 4);
    const int64_t bc = col0 + 8 * (t & 15);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if constexpr (VEC) {
            ra[h] = (ar < n) ? *reinterpret_cast<const f32x4*>(a + ar * n + ak + 4 * h)
                             : f32x4{0.f, 0.f, 0.f, 0.f};
            rb[h] = (bc + 4 * h < n) ? *reinterpret_cast<const f32x4*>(b + bk * n + bc + 4 * h)
                                     : f32x4{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t kk = ak + 4 * h + q;
                ra[h][q] = (ar < n && kk < n) ? a[ar * n + kk] : 0.f;
                const int64_t cc = bc + 4 * h + q;
                rb[h][q] = (bk < n && cc < n) ? b[bk * n + cc] : 0.f;
            }
        }
    }
}

__device__ inline void store_chunk(float* As, float* Bs, int t, const f32x4 (&ra)[2],
                                   const f32x4 (&rb)[2]) {
    float* arow = As + (t >> 1) * LDK + 8 * (t & 1);
    reinterpret_cast<f32x4*>(arow)[0] = ra[0];
    reinterpret_cast<f32x4*>(arow)[1] = ra[1];
    float* brow = Bs + (t >> 4) * LDB + 8 * (t & 15);
    reinterpret_cast<f32x4*>(brow)[0] = rb[0];
    reinterpret_cast<f32x4*>(brow)[1] = rb[1];
}

// WORK = false: the kernel with its on-chip work removed (the paper's
// work-removal transformation, Section "Measurement Workload Synthesis by
// Work Removal Transformation"): the same grid and the same global loads and
// stores, every loaded value added into one register, that register stored
// wherever the kernel stores a result; no LDS, no matrix-core work, no
// barriers.  It measures this kernel's global-memory access pattern alone.
template <bool VEC, bool WORK = true>
__global__ void __launch_bounds__(256) matmul_kernel(const float* __restrict__ a,
                                                     const float* __restrict__ b,
                                                     float* __restrict__ c, int64_t n) {
    if constexpr (!WORK) {
        const int t = threadIdx.x;
        const int lane = t & 63, wave = t >> 6, cl = lane & 15, g = lane >> 4;
        const int64_t row0 = (int64_t)blockIdx.y * BM, col0 = (int64_t)blockIdx.x * BM;
        float tgt = 0.f;
        for (int64_t kc = 0; kc < ceil_div(n, BK); ++kc) {
            f32x4 ra[2], rb[2];
            load_chunk<VEC>(a, b, n, row0, col0, kc * BK, t, ra, rb);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) tgt += ra[h][q] + rb[h][q];
        }
        const f32x4 v = {tgt, tgt, tgt, tgt};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = row0 + (wave >> 1) * 64 + i * 16 + cl;
            if (r >= n) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t col = col0 + (wave & 1) * 64 + j * 16 + 4 * g;
                if constexpr (VEC) {
                    if (col < n) *reinterpret_cast<f32x4*>(c + r * n + col) = v;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (col + q < n) c[r * n + col + q] = tgt;
                }
            }
        }
        return;
    }
    __shared__ __attribute__((aligned(16))) float As_[2][BM * LDK];  // [buf][row][k]
    __shared__ __attribute__((aligned(16))) float Bs_[2][BK * LDB];  // [buf][k][col]
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int cl = lane & 15;
    const int g = lane >> 4;
    const int wr = wave >> 1;  // wave row (64 rows of c)
    const int wc = wave & 1;   // wave col (64 cols of c)
    const int64_t row0 = (int64_t)blockIdx.y * BM;
    const int64_t col0 = (int64_t)blockIdx.x * BM;
    const int64_t nk = ceil_div(n, BK);

    f32x4 acc[4][4];  // [row block][col block]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    f32x4 ra[2], rb[2];
    load_chunk<VEC>(a, b, n, row0, col0, 0, t, ra, rb);
    store_chunk(As_[0], Bs_[0], t, ra, rb);
    __syncthreads();

    for (int64_t kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) load_chunk<VEC>(a, b, n, row0, col0, (kc + 1) * BK, t, ra, rb);
        const float* As = As_[buf];
        const float* Bs = Bs_[buf];
        f32x4 av[4];
        float bv[4][4];  // [col block][k-step]
#pragma unroll
        for (int i = 0; i < 4; ++i)
            av[i] = *reinterpret_cast<const f32x4*>(As + (wr * 64 + i * 16 + cl) * LDK + 4 * g);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j][s] = Bs[(4 * g + s) * LDB + wc * 64 + j * 16 + cl];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j][s], av[i][s], acc[i][j],
                                                                     0, 0, 0);
        if (kc + 1 < nk) store_chunk(As_[buf ^ 1], Bs_[buf ^ 1], t, ra, rb);
        __syncthreads();
    }

    // lane holds c[row][col .. col+3] with row = .. + cl, col = .. + 4g
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t r = row0 + wr * 64 + i * 16 + cl;
        if (r >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = col0 + wc * 64 + j * 16 + 4 * g;
            if constexpr (VEC) {
                if (col < n) *reinterpret_cast<f32x4*>(c + r * n + col) = acc[i][j];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (col + q < n) c[r * n + col + q] = acc[i][j][q];
            }
        }
    }
}

}  // namespace

bool matmul_vector_ok(int64_t n, const void* a, const void* b, const void* c) {
    return n % BK == 0 && reinterpret_cast<uintptr_t>(a) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(b) % 16 == 0 && reinterpret_cast<uintptr_t>(c) % 16 == 0;
}

dg_status launch_matmul(int64_t n, const void* a, const void* b, void* c, hipStream_t s, bool work) {
    dim3 grid((unsigned)ceil_div(n, BM), (unsigned)ceil_div(n, BM));
    const bool vec = matmul_vector_ok(n, a, b, c);
    auto fn = vec ? (work ? matmul_kernel<true, true> : matmul_kernel<true, false>)
                  : (work ? matmul_kernel<false, true> : matmul_kernel<false, false>);
    hipLaunchKernelGGL(fn, grid, dim3(256), 0, s, static_cast<const float*>(a), static_cast<const float*>(b),
                       static_cast<float*>(c), n);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
