// Measurement kernels: the calibration set of microbenchmarks (Sections
// "Measurement Kernel Design" and "Measurement Kernel Sets for Evaluation")
// and the work-removed twin of the DG kernel (Section "Measurement Workload
// Synthesis by Work Removal Transformation").  Each microbenchmark exercises
// one feature of the model while the others stay fixed; the twins keep a
// kernel's global-memory accesses and drop its on-chip work, so that the
// cost of exactly that access pattern can be measured.
//
//   stream    out = in_0 + ... + in_{nin-1}: 16-byte vectors, consecutive lanes
//             on consecutive vectors, grid-stride (global loads and stores of
//             the pattern the DG, stencil and quantiser kernels use)
//   strided   out[t] = in[t * S]: one 4-byte load per lane, lanes S floats
//             apart (S = 1 coalesced, S >= 32 one cache line per lane)
//   fma       32 FP32 registers updated by fused multiply-adds, 64 updates per
//             loop trip, none reading a register written in the last four
//             updates; the registers' sum stored
//   mfma      chains of v_mfma_f32_16x16x4f32 (or the BF16 16x16x32 form) on
//             register operands, eight independent accumulators per wave
//   lds       values moved around the wave's LDS slots (each trip reads the
//             neighbouring lane's slot and writes the lane's own; no bank
//             conflicts), 4- or 16-byte accesses
//   barrier   work-group barriers in a loop
//   overlap   one 16-byte global load, m LDS store/load pairs, one 16-byte
//             global store per thread (the paper's local/global overlap
//             kernel: m sets whether global or on-chip time dominates)
//   twin_dg   the DG forward's grid and global accesses without its on-chip
//             work (see dg_twin_kernel)
#include "dg_kernel.hpp"

namespace dg {
namespace {

using namespace kern;

__global__ void __launch_bounds__(256) ub_stream_kernel(const float* __restrict__ i0,
                                                        const float* __restrict__ i1,
                                                        const float* __restrict__ i2,
                                                        const float* __restrict__ i3, int nin,
                                                        int64_t n4, float* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n4; v += stride) {
        f32x4 s = reinterpret_cast<const f32x4*>(i0)[v];
        if (nin > 1) s += reinterpret_cast<const f32x4*>(i1)[v];
        if (nin > 2) s += reinterpret_cast<const f32x4*>(i2)[v];
        if (nin > 3) s += reinterpret_cast<const f32x4*>(i3)[v];
        reinterpret_cast<f32x4*>(out)[v] = s;
    }
}

__global__ void __launch_bounds__(256) ub_strided_kernel(const float* __restrict__ in, int64_t n,
                                                         int64_t S, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = in[t * S];
}

// Register r[v] takes r[v] * (-1/2) + r[(v + 16) % 32]: update k of a trip
// writes register k % 32 and reads registers written 16 and 32 updates
// earlier, so no update waits on the last four.
__global__ void __launch_bounds__(256) ub_fma_kernel(int iters, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float r[32];
#pragma unroll
    for (int v = 0; v < 32; ++v) r[v] = (float)(threadIdx.x & 255) * 0x1p-8f + (float)v * 0x1p-5f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const int v = k & 31;
            r[v] = __builtin_fmaf(r[v], -0.5f, r[(v + 16) & 31]);
        }
    }
    float s = r[0];
#pragma unroll
    for (int v = 1; v < 32; ++v) s += r[v];
    out[t] = s;
}

typedef short bf16x8 __attribute__((ext_vector_type(8)));

// Operands from the lane index (small integers, exact in FP32 and BF16):
// lane l supplies a(l) = (3l mod 7) - 3 and b(l) = (5l mod 9) - 4 to every
// position it holds.  Eight accumulators each take iters products; the lane
// stores their sum (four floats).
template <bool BF16>
__global__ void __launch_bounds__(256) ub_mfma_kernel(int iters, float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const float a = (float)((3 * lane) % 7 - 3);
    const float b = (float)((5 * lane) % 9 - 4);
    f32x4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
        // BF16 of a small integer: the upper half of its FP32 encoding
        const short ab = (short)(__builtin_bit_cast(uint32_t, a) >> 16);
        const short bb = (short)(__builtin_bit_cast(uint32_t, b) >> 16);
        bf16x8 av, bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            av[q] = ab;
            bv[q] = bb;
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[k], 0, 0, 0);
    } else {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
    }
    f32x4 s = acc[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) s += acc[k];
    reinterpret_cast<f32x4*>(out)[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// W floats per lane (1 or 4).  Slot of lane l of wave w: w*64 + l.  Trip k
// reads buffer k%2 at the next lane's slot and writes buffer (k+1)%2 at its
// own: after `iters` trips lane l holds the input of lane (l + iters) % 64.
template <int W>
__global__ void __launch_bounds__(256) ub_lds_kernel(const float* __restrict__ in, int iters,
                                                     float* __restrict__ out) {
    typedef float vec_t __attribute__((ext_vector_type(W)));
    __shared__ __attribute__((aligned(16))) vec_t buf[2][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    vec_t x;
    __builtin_memcpy(&x, in + g * W, sizeof(vec_t));
    buf[0][threadIdx.x] = x;
    wave_lds_sync();
    for (int k = 0; k < iters; ++k) {
        const vec_t y = buf[k & 1][wave * 64 + ((lane + 1) & 63)];
        buf[(k + 1) & 1][threadIdx.x] = y;
        wave_lds_sync();
    }
    x = buf[iters & 1][threadIdx.x];
    __builtin_memcpy(out + g * W, &x, sizeof(vec_t));
}

__global__ void __launch_bounds__(256) ub_barrier_kernel(int iters, float* __restrict__ out) {
    for (int k = 0; k < iters; ++k) __syncthreads();
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)iters;
}

// Thread g loads vector g (if it exists; otherwise zeros), moves it m times
// to the next lane of its wave through LDS (one 16-byte store and load each),
// and stores what it holds: vector g receives the input of lane (l + m) % 64
// of the same wave, or zeros where that vector does not exist.
// The square matmul's two operand-fetch patterns (the paper's pattern a and
// b): a 16 x 16 work-group reads, at each of n/16 trips, sixteen 64-byte row
// pieces -- moving along its rows (a) or down the rows (b) -- and each thread
// stores the sum of the n/16 values it read.
template <bool B>
__global__ void __launch_bounds__(256) ub_tile_read_kernel(const float* __restrict__ x, int n,
                                                           float* __restrict__ out) {
    const int l0 = threadIdx.x & 15, l1 = threadIdx.x >> 4;
    const int g0 = blockIdx.x, g1 = blockIdx.y;
    float s = 0.0f;
    for (int k = 0; k < n / 16; ++k) {
        const int64_t idx = B ? (int64_t)n * (16 * k + l1) + 16 * g0 + l0 : (int64_t)n * (16 * g1 + l1) + 16 * k + l0;
        s += x[idx];
    }
    out[(int64_t)n * (16 * g1 + l1) + 16 * g0 + l0] = s;
}

__global__ void __launch_bounds__(256) ub_overlap_kernel(const float* __restrict__ in, int64_t n4, int m,
                                                         float* __restrict__ out) {
    __shared__ f32x4 buf[2][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    f32x4 x = {0.f, 0.f, 0.f, 0.f};
    if (g < n4) x = reinterpret_cast<const f32x4*>(in)[g];
    for (int k = 0; k < m; ++k) {
        buf[k & 1][threadIdx.x] = x;
        wave_lds_sync();
        x = buf[k & 1][wave * 64 + ((lane + 1) & 63)];
        wave_lds_sync();
    }
    if (g < n4) reinterpret_cast<f32x4*>(out)[g] = x;
}

// ---------------------------------------------------------------- DG twin
//
// The DG forward (FP32) with its on-chip work removed: the same persistent,
// XCD-aware grid and launch plan (make_plan), and per work-group the same
// global accesses in the same order -- the operator entries its group
// stages, then per element tile the element rows (16-byte vectors from the
// row start, or the wave's contiguous slab for rows off 16-byte boundaries;
// the pipelined loads' whole wave-tiles, rows past the end clamped to the
// last element, where the forward pipelines them), then the output stores
// (paired panels, single panels, or the staged contiguous rows).  Every
// loaded value is added into one register and that register is what every
// store writes.  No LDS, no matrix-core work, no barriers.
struct TwinArgs {
    const float* D;
    const float* u;
    float* out;
    int64_t nelem, ntiles;
    int nunit, kq, cb, mblk, panels_total, ppg, ngroups, nstreams;
    int vec_in, use_slab, vec_out, stage_out, pair, piped;
};

__global__ void __launch_bounds__(512) dg_twin_kernel(TwinArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int n = a.nunit, KQ = a.kq, KP = 4 * a.kq, CB = a.cb;
    const int xcd = blockIdx.x & 7, kb = blockIdx.x >> 3;
    const int pg = kb % a.ngroups;
    const int64_t stream = (int64_t)(kb / a.ngroups) * 8 + xcd;
    const int p_lo = pg * a.ppg;
    const int np = min(a.ppg, a.panels_total - p_lo);
    float tgt = 0.f;
    // the operator entries this group stages (as stage_panels visits them)
    for (int idx = threadIdx.x; idx < np * 16 * KP; idx += blockDim.x) {
        const int k = idx % KP, rr = idx / KP;
        const int panel = p_lo + rr / 16;
        const int slab = panel / a.mblk, o = (panel % a.mblk) * 16 + rr % 16;
        if (o < n && k < n) tgt += a.D[((int64_t)slab * n + o) * n + k];
    }
    const int64_t tile_elems = (int64_t)nw * 16 * CB;
    for (int64_t tile = stream; tile < a.ntiles; tile += a.nstreams) {
        const int64_t e0 = tile * tile_elems + (int64_t)wave * 16 * CB;
        if (e0 >= a.nelem) continue;
        const int nel = (int)min<int64_t>(16 * CB, a.nelem - e0);
        // element data
        if (a.piped) {
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                const float* row = a.u + (e < a.nelem ? e : a.nelem - 1) * n;
                for (int s4 = 0; s4 < KQ / 4; ++s4) {
                    const int col = g * KQ + 4 * s4;
                    const f32x4 v = *reinterpret_cast<const f32x4*>(row + (col < n ? col : 0));
                    tgt += v[0] + v[1] + v[2] + v[3];
                }
            }
        } else if (a.vec_in) {
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                if (e >= a.nelem) continue;
                const float* row = a.u + e * n + g * KQ;
                for (int s = 0; s < KQ; s += 4)
                    if (g * KQ + s < n) {
                        const f32x4 v = *reinterpret_cast<const f32x4*>(row + s);
                        tgt += v[0] + v[1] + v[2] + v[3];
                    }
            }
        } else if (a.use_slab) {
            const int len = nel * n;
            const float* base = a.u + e0 * n;
            const int nvec = reinterpret_cast<uintptr_t>(a.u) % 16 == 0 ? len / 4 : 0;
            for (int q = lane; q < nvec; q += 64) {
                const f32x4 v = reinterpret_cast<const f32x4*>(base)[q];
                tgt += v[0] + v[1] + v[2] + v[3];
            }
            for (int f = nvec * 4 + lane; f < len; f += 64) tgt += base[f];
        } else {
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                const bool ok = e < a.nelem;
                const float* row = a.u + (ok ? e : 0) * n + g * KQ;
                for (int t = 0; t < KQ; t += 4) {
                    const f32x4 v = load_vec_any<float>(row + t, ok, n - g * KQ - t);
                    tgt += v[0] + v[1] + v[2] + v[3];
                }
            }
        }
        // output stores
        const f32x4 w = {tgt, tgt, tgt, tgt};
        int pp = 0;
        if (a.pair) {
            for (; pp + 1 < np; pp += 2) {
                const int panel = p_lo + pp;
                const int slab_o = panel / a.mblk;
                const int i = (panel % a.mblk) * 16 + (c < 8 ? 0 : 16) + 4 * g;
                for (int cb = 0; cb < CB; ++cb) {
                    const int64_t e1 = e0 + cb * 16 + (c & 7), e2 = e1 + 8;
                    if (i < n) {
                        if (e1 < a.nelem) *reinterpret_cast<f32x4*>(a.out + ((int64_t)slab_o * a.nelem + e1) * n + i) = w;
                        if (e2 < a.nelem) *reinterpret_cast<f32x4*>(a.out + ((int64_t)slab_o * a.nelem + e2) * n + i) = w;
                    }
                }
            }
        }
        for (; pp < np; ++pp) {
            const int panel = p_lo + pp;
            const int slab_o = panel / a.mblk;
            const int i0 = (panel % a.mblk) * 16;
            const int i = i0 + 4 * g;
            if (a.stage_out) {
                const int pf = max(p_lo, slab_o * a.mblk);
                const int pl = min(p_lo + np, (slab_o + 1) * a.mblk);
                if (panel + 1 != pl) continue;
                // the staged rows [r_lo, r_lo + rows) of the wave's elements, contiguous
                const int r_lo = (pf - slab_o * a.mblk) * 16;
                const int rows = min((pl - slab_o * a.mblk) * 16, n) - r_lo;
                float* dst = a.out + ((int64_t)slab_o * a.nelem + e0) * n;
                if (rows == n) {
                    const int len = nel * n;
                    int done = 0;
                    if (reinterpret_cast<uintptr_t>(dst) % 16 == 0) {
                        const int nv = len / 4;
                        for (int q = lane; q < nv; q += 64) reinterpret_cast<f32x4*>(dst)[q] = w;
                        done = nv * 4;
                    }
                    for (int f = done + lane; f < len; f += 64) dst[f] = tgt;
                } else {
                    for (int f = lane; f < nel * rows; f += 64) {
                        const int el = f / rows;
                        dst[(int64_t)el * n + r_lo + (f - el * rows)] = tgt;
                    }
                }
                continue;
            }
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                if (e >= a.nelem || i >= n) continue;
                float* dst = a.out + ((int64_t)slab_o * a.nelem + e) * n + i;
                if (a.vec_out) {
                    *reinterpret_cast<f32x4*>(dst) = w;
                } else {
                    const int av = n - i;
                    if (av >= 4) __builtin_memcpy(dst, &w, 16);
                    else
                        for (int t = 0; t < av; ++t) dst[t] = tgt;
                }
            }
        }
    }
}

}  // namespace

// The twin's launch: the plan dgdiff_apply would make with this (resolved)
// tile on this device, the forward's paths (pipelined loads, paired stores,
// slab, staged rows) decided as the forward decides them.
dg_status launch_dg_twin(int nmat, int64_t nelem, int nunit, const dg_tile* tile, const float* D,
                         const float* u, float* out, hipStream_t s) {
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    const bool rows_aligned = nunit % 4 == 0 && reinterpret_cast<uintptr_t>(u) % 16 == 0;
    int cb;
    dg_status st = forward_cb(4, kq, rows_aligned, tile->elems_per_wave, &cb);
    if (st != DG_OK) return st;
    if (tile->waves < 1 || tile->waves > 8 || tile->groups_per_cu < 1)
        return fail(DG_EINVAL, "DG twin: needs a resolved tile");
    DeviceInfo dev;
    st = current_device(&dev);
    if (st != DG_OK) return st;
    Plan P;
    st = make_plan(4, 1, nmat, nelem, nunit, kq, cb, tile->waves, tile->d_panels, tile->groups_per_cu,
                   dev.num_cu, rows_aligned, &P);
    if (st != DG_OK) return st;
    const bool vec_out = nunit % 4 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
    TwinArgs a = {};
    a.D = D;
    a.u = u;
    a.out = out;
    a.nelem = nelem;
    a.ntiles = P.ntiles;
    a.nunit = nunit;
    a.kq = kq;
    a.cb = cb;
    a.mblk = P.mblk;
    a.panels_total = P.panels_total;
    a.ppg = P.ppg;
    a.ngroups = P.ngroups;
    a.nstreams = (int)(8 * P.slots);
    a.vec_in = P.vec_in;
    a.use_slab = P.use_slab;
    a.vec_out = vec_out;
    a.stage_out = P.use_slab && !vec_out;
    a.pair = pair_eligible(4, nunit, vec_out, P) ? 1 : 0;
    a.piped = pipelined_loads(4, nunit, kq, cb, vec_out, P) ? 1 : 0;
    hipLaunchKernelGGL(dg_twin_kernel, dim3((unsigned)P.grid), dim3(64 * tile->waves), 0, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

dg_status launch_ubench(const dg_ubench_desc* d, const void* const* in, void* out, hipStream_t s) {
    float* o = static_cast<float*>(out);
    const int64_t n = d->n;
    switch (d->kind) {
        case DG_UB_STREAM: {
            const int nin = d->a;
            const float* p[4] = {nullptr, nullptr, nullptr, nullptr};
            for (int k = 0; k < nin; ++k) p[k] = static_cast<const float*>(in[k]);
            const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), kUbStreamBlocks));
            hipLaunchKernelGGL(ub_stream_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p[0], p[1], p[2], p[3],
                               nin, n, o);
            break;
        }
        case DG_UB_STRIDED:
            hipLaunchKernelGGL(ub_strided_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                               static_cast<const float*>(in[0]), n, (int64_t)d->a, o);
            break;
        case DG_UB_FMA:
            hipLaunchKernelGGL(ub_fma_kernel, dim3((unsigned)n), dim3(256), 0, s, d->a, o);
            break;
        case DG_UB_MFMA:
            if (d->dtype == DG_BF16)
                hipLaunchKernelGGL(ub_mfma_kernel<true>, dim3((unsigned)n), dim3(256), 0, s, d->a, o);
            else
                hipLaunchKernelGGL(ub_mfma_kernel<false>, dim3((unsigned)n), dim3(256), 0, s, d->a, o);
            break;
        case DG_UB_LDS:
            if (d->b == 4)
                hipLaunchKernelGGL(ub_lds_kernel<4>, dim3((unsigned)n), dim3(256), 0, s,
                                   static_cast<const float*>(in[0]), d->a, o);
            else
                hipLaunchKernelGGL(ub_lds_kernel<1>, dim3((unsigned)n), dim3(256), 0, s,
                                   static_cast<const float*>(in[0]), d->a, o);
            break;
        case DG_UB_BARRIER:
            hipLaunchKernelGGL(ub_barrier_kernel, dim3((unsigned)n), dim3(256), 0, s, d->a, o);
            break;
        case DG_UB_OVERLAP:
            hipLaunchKernelGGL(ub_overlap_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                               static_cast<const float*>(in[0]), n, d->a, o);
            break;
        case DG_UB_TILE_READ: {
            const dim3 grid((unsigned)(n / 16), (unsigned)(n / 16));
            if (d->a == 1)
                hipLaunchKernelGGL(ub_tile_read_kernel<true>, grid, dim3(256), 0, s,
                                   static_cast<const float*>(in[0]), (int)n, o);
            else
                hipLaunchKernelGGL(ub_tile_read_kernel<false>, grid, dim3(256), 0, s,
                                   static_cast<const float*>(in[0]), (int)n, o);
            break;
        }
        case DG_UB_TWIN_DG:
            return launch_dg_twin(d->b, n, d->a, &d->tile, static_cast<const float*>(in[0]),
                                  static_cast<const float*>(in[1]), o, s);
        case DG_UB_TWIN_STENCIL:
            return launch_stencil5(DG_F32, n, in[0], d->a, out, d->b, s, false);
        case DG_UB_TWIN_MATMUL:
            return launch_matmul(n, in[0], in[1], out, s, false);
        default:
            return fail(DG_EINVAL, "dg_ubench_run: unknown kind");
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
