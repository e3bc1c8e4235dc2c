// The DG contraction kernel shared by the forward operator and the adjoint's
// grad_u (FP32 and FP64, gfx950 matrix cores).
//
// Forward (paper, Section "DG Differentiation"):
//     out[m][e][i] = sum_j D[m][i][j] * u[e][j].
// Stacking the operators' rows, this is one tall-skinny GEMM
//     C^T[(m,i)][e] = sum_j D[(m,i)][j] * U^T[j][e]
// whose long dimension is the element count.  Adjoint, element part:
//     grad_u[e][j] = sum_m sum_i D[m][i][j] * g[m][e][i],
// the same shape with the operator transposed and a contraction index
// (m, i) that runs over nmat "segments" of the B operand (the slabs g[m]).
// One kernel serves both: a panel row is an output node, the contraction runs
// over NSEG segments of KP nodes each, and the B operand of segment s is read
// from src + s * seg_stride.
//
// MFMA mapping.  v_mfma_{f32,f64}_16x16x4: A = a 16-row panel of the
// (possibly transposed) operator stack, B = the data of 16 elements, so each
// lane's accumulator holds four output nodes of one element.  Lane group
// g = lane/16 supplies the k index: group g owns nodes [g*KQ, (g+1)*KQ) of a
// segment and k-step s contracts node g*KQ + s, so a lane reads KQ contiguous
// values of its element (16-byte vector loads straight from HBM) and KQ
// contiguous operator entries (16-byte LDS reads).  KP = 4*KQ >= nunit; the
// zero padding lives in registers and LDS only.
//
// Row order.  The f32 instruction returns rows 4g..4g+3 to lane group g; the
// f64 one returns rows g, g+4, g+8, g+12.  Panels are staged in the matching
// row order, so a lane's four results are always the consecutive nodes
// i0+4g .. i0+4g+3 (one 16-byte FP32 store).
//
// Operator residency.  The panels are split into `ngroups` groups of at most
// `ppg` panels; a work-group stages ONE group in LDS once and keeps it for its
// whole life, computing only those output rows for every element tile it
// visits.  Nothing is re-staged inside the tile loop.
//
// Grid (persistent, XCD-aware).  Work-groups are dispatched round-robin over
// the 8 XCDs (block b lands on XCD b % 8).  Block b takes panel group
// pg = (b/8) % ngroups and tile stream (b/8)/ngroups * 8 + b % 8, so the
// ngroups blocks that need the same element tile sit on the same XCD and walk
// the same tile sequence: the tile is fetched from HBM once and re-read from
// that XCD's L2 by the other groups.
//
// Paired stores.  A lane's four results of one panel are 16 bytes of one
// element row, so a panel's store writes 64-byte pieces of 16 rows.  FP32
// rows of a multiple of 32 nodes are written through a variant that computes
// two consecutive panels of one output slab together and trades halves
// between lanes c and c^8 (a DPP rotation by 8 within each 16-lane row): each
// of its two stores then covers 8 elements with 32 consecutive nodes, one
// 128-byte run each, which for such rows is a whole cache line.  Results and
// their rounding are unchanged.
//
// Unaligned rows.  When nunit is not a multiple of the 16-byte vector (or the
// source is not 16-byte aligned) a wave copies its contiguous slab of element
// data into a wave-private LDS area with aligned 16-byte loads and reads its
// fragments from there (or, if the slab would not fit, uses masked scalar
// loads).
#pragma once

#include "common.hpp"

namespace dg {
namespace kern {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// word 3 of a raw buffer resource (32-bit data format, no swizzle): plain
// byte offsets, range-checked
constexpr int kBufferWord3 = 0x00020000;
// cache policy of streaming output stores (DG_TILE_NT_STORE): non-temporal at
// system scope (nt sc0 sc1)
constexpr int kStreamStore = 2 | 1 | 16;

// A buffer view of [base, base + bytes) for streaming stores.  base and bytes
// are the same in every lane of the wave (callers pass wave-tile values);
// taking them from the first lane tells the compiler so, which keeps the
// resource in scalar registers (a per-lane resource would be stored through
// a loop over its distinct values).
__device__ inline __amdgpu_buffer_rsrc_t wave_buffer(void* base, int bytes) {
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    void* ub = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, 0, __builtin_amdgcn_readfirstlane(bytes), kBufferWord3);
}
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mma;

template <>
struct Mma<float> {
    typedef f32x4 acc_t;
    typedef f32x4 vec_t;  // one 16-byte vector
    static constexpr int V = 4;
    // accumulator register r of lane group g holds C row 4g + r
    __device__ static inline int acc_row(int g, int r) { return 4 * g + r; }
    __device__ static inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <>
struct Mma<double> {
    typedef f64x4 acc_t;
    typedef f64x2 vec_t;
    static constexpr int V = 2;
    // accumulator register r of lane group g holds C row g + 4r (interleaved)
    __device__ static inline int acc_row(int g, int r) { return g + 4 * r; }
    __device__ static inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

struct KArgs {
    const void* D;      // operator stack [nmat][nunit][nunit]
    const void* src;    // B operand: segment s, element e at src + s*seg_stride + e*nunit
    void* out;          // [out_slabs][nelem][nunit]
    int64_t nelem;
    int64_t ntiles;
    int64_t seg_stride; // elements between B segments (0 when NSEG == 1)
    int nunit;
    int transpose;      // 0: panel rows (m, i), k = j;  1: panel rows j, k = (m, i)
    int mblk;           // 16-row panels per output slab: ceil(nunit/16)
    int panels_total;   // out_slabs * mblk
    int ppg;            // panels per resident group
    int ngroups;        // ceil(panels_total / ppg)
    int nstreams;       // tile streams: 8 * (blocks per XCD per group)
    int vec_in;         // B rows may be read as 16-byte vectors
    int src_aligned;    // src itself is 16-byte aligned
    int use_slab;       // unaligned rows go through the wave-private LDS slab
    int vec_out;        // out rows may be written as 16-byte vectors
    int nt_store;       // streaming (non-temporal) output stores
    int stage_out;      // unaligned out rows: results staged in the wave's slab, written contiguously
};

__device__ inline int round_up_dev(int x, int v) { return (x + v - 1) / v * v; }

// Stage np panels starting at panel p0.  LDS row = output node, row stride
// NSEG*KP + V; entry (row, s*KP + k) is the operator value multiplying
// segment s, node k of the B operand.
template <typename T, int KQ, int NSEG>
__device__ inline void stage_panels(const T* __restrict__ D, T* dl, int p0, int np,
                                    const KArgs& a) {
    constexpr int KP = 4 * KQ;
    constexpr int LD = NSEG * KP + Mma<T>::V;
    const int nunit = a.nunit;
    const int total = np * 16 * NSEG * KP;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int kk = idx % (NSEG * KP);
        const int rr = idx / (NSEG * KP);  // output row within the staged group
        const int s = kk / KP;
        const int k = kk % KP;
        const int rn = rr % 16;            // node offset 4g + r within its panel
        const int panel = p0 + rr / 16;
        const int slab = panel / a.mblk;
        const int o = (panel % a.mblk) * 16 + rn;  // output node
        T v = T(0);
        if (o < nunit && k < nunit) {
            // forward: D[slab][o][k];  transposed: D[s][k][o]
            const int64_t idx_d = a.transpose ? ((int64_t)s * nunit + k) * nunit + o
                                              : ((int64_t)slab * nunit + o) * nunit + k;
            v = D[idx_d];
        }
        // Place node 4g + r at the panel row whose accumulator lands in
        // register r of lane group g.
        const int rho = Mma<T>::acc_row(rn >> 2, rn & 3);
        dl[(rr - rn + rho) * LD + kk] = v;
    }
}

// V consecutive values of a row that starts at any element-size boundary;
// `avail` of them (from p on) belong to the row, the rest read as zero.  A
// full vector is one 16-byte load (the 16-byte copy is left to the compiler,
// which issues a single vector access on this target); row tails go value
// by value.
template <typename T>
__device__ inline typename Mma<T>::vec_t load_vec_any(const T* p, bool ok, int avail) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    vec_t v = vec_t(T(0));
    if (!ok || avail <= 0) return v;
    if (avail >= V) {
        __builtin_memcpy(&v, p, 16);
    } else {
#pragma unroll
        for (int t = 0; t < V - 1; ++t)
            if (t < avail) v[t] = p[t];
    }
    return v;
}

// B fragments of one 16-element column block straight from global memory:
// KQ contiguous nodes of the lane's element from node g*KQ; zero beyond nunit
// or nelem.  Requires 16-byte aligned rows (vec_in).
template <typename T, int KQ>
__device__ inline void load_b_global(const T* __restrict__ src, int64_t e, int g, const KArgs& a,
                                     T (&b)[KQ]) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    const bool ev = e < a.nelem;
    const T* row = src + (ev ? e : 0) * a.nunit + g * KQ;
#pragma unroll
    for (int s = 0; s < KQ; s += V) {
        vec_t v = vec_t(T(0));
        if (ev && g * KQ + s < a.nunit) v = *reinterpret_cast<const vec_t*>(row + s);
#pragma unroll
        for (int t = 0; t < V; ++t) b[s + t] = v[t];
    }
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copy the wave's contiguous slab of nel elements (nel*nunit values starting
// at element ew0) into wave-private LDS.
template <typename T>
__device__ inline void stage_slab(const T* __restrict__ src, int64_t ew0, int nel, int nunit,
                                  bool aligned, T* slab, int lane) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    const int len = nel * nunit;
    const T* base = src + ew0 * nunit;
    // ew0 is a multiple of 16, so the slab starts 16-byte aligned iff src does
    const int nvec = aligned ? len / V : 0;
    for (int q = lane; q < nvec; q += 64)
        reinterpret_cast<vec_t*>(slab)[q] = reinterpret_cast<const vec_t*>(base)[q];
    for (int f = nvec * V + lane; f < len; f += 64) slab[f] = base[f];
}

// Write a wave's staged results: nel element rows of `rows` values (output
// nodes r_lo .. r_lo+rows-1) from st[el*rows + ii] to dst[el*nunit + r_lo + ii]
// (dst = the wave's first element row of one output slab).  Whole rows form
// one contiguous range, written with 16-byte vectors where aligned; partial
// rows go out as runs of consecutive scalars.  ACC adds to dst.
template <typename T, bool ACC>
__device__ inline void write_staged(const T* st, T* __restrict__ dst, int nel, int rows, int r_lo,
                                    int nunit, int lane, bool nt) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    if (rows == nunit) {
        const int len = nel * nunit;
        int done = 0;
        if (reinterpret_cast<uintptr_t>(dst) % 16 == 0) {
            const int nv = len / V;
            if (nt) {
                // streaming stores through a buffer view of the run
                const __amdgpu_buffer_rsrc_t rs = wave_buffer(dst, nv * 16);
                for (int q = lane; q < nv; q += 64) {
                    vec_t v = reinterpret_cast<const vec_t*>(st)[q];
                    if constexpr (ACC) v += reinterpret_cast<const vec_t*>(dst)[q];
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, q * 16, 0,
                                                           kStreamStore);
                }
            } else {
                for (int q = lane; q < nv; q += 64) {
                    vec_t v = reinterpret_cast<const vec_t*>(st)[q];
                    if constexpr (ACC) v += reinterpret_cast<const vec_t*>(dst)[q];
                    reinterpret_cast<vec_t*>(dst)[q] = v;
                }
            }
            done = nv * V;
        }
        for (int f = done + lane; f < len; f += 64) {
            T v = st[f];
            if constexpr (ACC) v += dst[f];
            dst[f] = v;
        }
    } else {
        for (int f = lane; f < nel * rows; f += 64) {
            const int el = f / rows;
            const int64_t o = (int64_t)el * nunit + r_lo + (f - el * rows);
            T v = st[f];
            if constexpr (ACC) v += dst[o];
            dst[o] = v;
        }
    }
}

// Panel pairs of one tile (see "Paired stores"): returns the number of panels
// done (np rounded down to even).  b: the lane's element fragments.
template <int KQ, int CB>
__device__ inline int paired_panels(const float (&b)[CB][KQ], int64_t e0, int p_lo, int np,
                                    const float* dl, float* __restrict__ out, const KArgs& a, int c,
                                    int g) {
    constexpr int V = 4;
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + V;
    const int nunit = a.nunit;
    int pp = 0;
    // panel pairs (pp, pp+1) start at even panels of a group whose first
    // panel is even, and slabs hold an even number of panels, so a pair
    // never straddles two output slabs
    for (; pp + 1 < np; pp += 2) {
        const int panel = p_lo + pp;
        const int slab_o = panel / a.mblk;
        const int i0 = (panel % a.mblk) * 16;
        f32x4 accA[CB], accB[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            accA[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
            accB[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        const float* arowA = dl + (pp * 16 + c) * LD + g * KQ;
        const float* arowB = arowA + 16 * LD;
#pragma unroll
        for (int t = 0; t < KQ; t += V) {
            const f32x4 avA = *reinterpret_cast<const f32x4*>(arowA + t);
            const f32x4 avB = *reinterpret_cast<const f32x4*>(arowB + t);
#pragma unroll
            for (int q = 0; q < V; ++q)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    accA[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avA[q], b[cb][t + q], accA[cb], 0, 0, 0);
                    accB[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avB[q], b[cb][t + q], accB[cb], 0, 0, 0);
                }
        }
        // lanes c < 8 keep panel A and take lane c+8's; lanes c >= 8 keep
        // panel B and take lane c-8's: store 1 holds elements c&7 (nodes
        // i0 .. i0+31), store 2 elements 8 + (c&7)
        const bool lo = c < 8;
        const int i = i0 + (lo ? 0 : 16) + 4 * g;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            f32x4 x1, x2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float send = lo ? accB[cb][r] : accA[cb][r];
                const float got = __builtin_bit_cast(
                    float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, send),
                                                       0x128 /* row_ror:8 */, 0xF, 0xF, false));
                x1[r] = lo ? accA[cb][r] : got;
                x2[r] = lo ? got : accB[cb][r];
            }
            const int64_t e1 = e0 + cb * 16 + (c & 7);
            const int64_t e2 = e1 + 8;
            if (a.nt_store) {
                // streaming stores through a range-checked buffer view of
                // this wave-tile's output rows of the slab (rows past the
                // last element fall outside it and are dropped)
                const int nel = (int)min<int64_t>(16 * CB, a.nelem - e0);
                const __amdgpu_buffer_rsrc_t rs =
                    wave_buffer(out + ((int64_t)slab_o * a.nelem + e0) * nunit, nel * nunit * 4);
                const int o1 = ((cb * 16 + (c & 7)) * nunit + i) * 4;
                if (i < nunit) {
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x1), rs, o1, 0,
                                                           kStreamStore);
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x2), rs, o1 + 8 * nunit * 4,
                                                           0, kStreamStore);
                }
                continue;
            }
            if (i < nunit) {
                if (e1 < a.nelem)
                    *reinterpret_cast<f32x4*>(out + ((int64_t)slab_o * a.nelem + e1) * nunit + i) = x1;
                if (e2 < a.nelem)
                    *reinterpret_cast<f32x4*>(out + ((int64_t)slab_o * a.nelem + e2) * nunit + i) = x2;
            }
        }
    }
    return pp;
}

// One panel of a paired-store tile (the odd last panel of a group).
template <int KQ, int CB>
__device__ inline void single_panel_vec(const float (&b)[CB][KQ], int64_t e0, int p_lo, int pp,
                                        const float* dl, float* __restrict__ out, const KArgs& a,
                                        int c, int g) {
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + 4;
    const int nunit = a.nunit;
    const int panel = p_lo + pp;
    const int slab_o = panel / a.mblk;
    const int i = (panel % a.mblk) * 16 + 4 * g;
    f32x4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float* arow = dl + (pp * 16 + c) * LD + g * KQ;
#pragma unroll
    for (int t = 0; t < KQ; t += 4) {
        const f32x4 av = *reinterpret_cast<const f32x4*>(arow + t);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], b[cb][t + q], acc[cb], 0, 0, 0);
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int64_t e = e0 + cb * 16 + c;
        if (e < a.nelem && i < nunit)
            *reinterpret_cast<f32x4*>(out + ((int64_t)slab_o * a.nelem + e) * nunit + i) = acc[cb];
    }
}

// ------------------------------------------------- pipelined element loads
// (paired-store kernels with 16-byte element rows)
// One counter tracks a wave's outstanding vector loads and stores, and the
// compiler's own wait before the first use of a loaded register counts every
// store issued since as pending: a persistent loop that loads the next tile
// and then stores the current one waits for all of its stores, and the load,
// at each tile boundary.  Here the next tile's element data are issued as
// loads the compiler does not track, before the current tile's stores, and the
// wave waits for them with an explicit count that leaves the current tile's
// stores in flight: waiting until at most m operations are outstanding, with
// m no more than the stores issued after the loads, completes the loads.
// Every lane loads from a valid address (rows past the end clamp to the last
// element, columns past the end to column 0); values are masked after the
// wait.
__device__ inline void async_load4(f32x4& r, const float* p) {
    asm volatile("global_load_dwordx4 %0, %1, off" : "=v"(r) : "v"(p) : "memory");
}
template <int N>
__device__ inline void vm_wait() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// wait until at most m vector memory operations are outstanding, for the
// largest bucket m <= n (n wave-uniform)
__device__ inline void vm_wait_below(int n) {
    if (n >= 32) vm_wait<32>();
    else if (n >= 16) vm_wait<16>();
    else if (n >= 8) vm_wait<8>();
    else if (n >= 4) vm_wait<4>();
    else vm_wait<0>();
}
// the loaded registers pass through an empty statement ordered after the
// wait, so that nothing reads them earlier
__device__ inline void settle(f32x4& r) { asm volatile("" : "+v"(r)); }

template <int KQ, int CB>
struct TileBuf {
    f32x4 v[CB][KQ / 4];
};

template <int KQ, int CB>
__device__ inline void tile_issue(const float* __restrict__ src, int64_t e0, int c, int g,
                                  const KArgs& a, TileBuf<KQ, CB>& t) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int64_t e = e0 + cb * 16 + c;
        const int64_t ec = e < a.nelem ? e : a.nelem - 1;
        const float* row = src + ec * a.nunit;
#pragma unroll
        for (int s4 = 0; s4 < KQ / 4; ++s4) {
            const int col = g * KQ + 4 * s4;
            async_load4(t.v[cb][s4], row + (col < a.nunit ? col : 0));
        }
    }
}

template <int KQ, int CB>
__device__ inline void tile_settle(TileBuf<KQ, CB>& t) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int s4 = 0; s4 < KQ / 4; ++s4) settle(t.v[cb][s4]);
}

// Fewest store instructions one tile issues: all of them (two per pair, one
// per single panel, per column block) when the tile's elements all exist, at
// least one per pair or single otherwise (its first element's).
template <int CB>
__device__ inline int tile_stores_min(int np, bool full) {
    const int pairs = np / 2, singles = np - 2 * pairs;
    return full ? (2 * pairs + singles) * CB : pairs + singles;
}

template <int KQ, int CB>
__device__ inline void tile_compute(const TileBuf<KQ, CB>& t, int64_t e0, int p_lo, int np,
                                    const float* dl, float* __restrict__ out, const KArgs& a, int c,
                                    int g) {
    float b[CB][KQ];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const bool ev = e0 + cb * 16 + c < a.nelem;
#pragma unroll
        for (int s4 = 0; s4 < KQ / 4; ++s4) {
            const bool ok = ev && g * KQ + 4 * s4 < a.nunit;
#pragma unroll
            for (int q = 0; q < 4; ++q) b[cb][4 * s4 + q] = ok ? t.v[cb][s4][q] : 0.f;
        }
    }
    const int pp = paired_panels<KQ, CB>(b, e0, p_lo, np, dl, out, a, c, g);
    if (pp < np) single_panel_vec<KQ, CB>(b, e0, p_lo, pp, dl, out, a, c, g);
}

// ACC: out += result instead of out = result (a compile-time switch: as a
// runtime branch it costs the FP32 kernels ~150 registers).
// Work-groups of up to 8 waves for variants whose element operand takes at
// most 64 registers (more waves then share one copy of the resident
// operator panels); the register-heavy variants keep 4 waves so that they
// may use the whole register file.
template <typename T, int KQ, int CB, int NSEG>
constexpr int dg_max_threads() {
    return CB * NSEG * KQ * (int)sizeof(T) <= 256 ? 512 : 256;
}

template <typename T, int KQ, int CB, int NSEG, bool ACC = false, bool PAIR = false>
__global__ void __launch_bounds__((dg_max_threads<T, KQ, CB, NSEG>())) dg_kernel(KArgs a) {
    typedef typename Mma<T>::acc_t acc_t;
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    constexpr int KP = 4 * KQ;
    constexpr int LD = NSEG * KP + V;  // one vector of row padding against bank conflicts

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T* dl = reinterpret_cast<T*>(smem);
    const T* __restrict__ D = static_cast<const T*>(a.D);
    const T* __restrict__ src = static_cast<const T*>(a.src);
    T* __restrict__ out = static_cast<T*>(a.out);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int c = lane & 15;  // MFMA column: the element within a 16-block
    const int g = lane >> 4;  // MFMA k index: which quarter of the nodes
    const int nunit = a.nunit;

    // XCD-aware placement: see the file comment.
    const int xcd = blockIdx.x & 7;
    const int kb = blockIdx.x >> 3;
    const int pg = kb % a.ngroups;
    const int64_t stream = (int64_t)(kb / a.ngroups) * 8 + xcd;
    const int p_lo = pg * a.ppg;
    const int np = min(a.ppg, a.panels_total - p_lo);

    stage_panels<T, KQ, NSEG>(D, dl, p_lo, np, a);
    // wave-private slab (all segments) for unaligned element rows
    const int slab_seg = round_up_dev(16 * CB * nunit, V);
    T* slab = dl + (size_t)a.ppg * 16 * LD + (size_t)wave * NSEG * slab_seg;
    __syncthreads();

    const int64_t tile_elems = (int64_t)nw * 16 * CB;
    if constexpr (PAIR && KQ * CB <= 32) {
        if (a.vec_in) {
            // pipelined element loads (see above); no block-level sync below
            const int64_t woff = (int64_t)__builtin_amdgcn_readfirstlane(wave) * 16 * CB;
            TileBuf<KQ, CB> A, B;
            int64_t t0 = stream;
            if (t0 >= a.ntiles) return;
            // a wave-tile whose first element is past the end loads nothing
            // (and computes nothing)
            if (t0 * tile_elems + woff < a.nelem) tile_issue<KQ, CB>(src, t0 * tile_elems + woff, c, g, a, A);
            vm_wait<0>();
            tile_settle(A);
            for (;;) {
                const int64_t t1 = t0 + a.nstreams;
                const bool more1 = t1 < a.ntiles;
                if (more1 && t1 * tile_elems + woff < a.nelem)
                    tile_issue<KQ, CB>(src, t1 * tile_elems + woff, c, g, a, B);
                const int64_t ea = t0 * tile_elems + woff;
                if (ea < a.nelem) tile_compute<KQ, CB>(A, ea, p_lo, np, dl, out, a, c, g);
                if (!more1) break;
                vm_wait_below(ea < a.nelem ? tile_stores_min<CB>(np, ea + 16 * CB <= a.nelem) : 0);
                tile_settle(B);
                const int64_t t2 = t1 + a.nstreams;
                const bool more2 = t2 < a.ntiles;
                if (more2 && t2 * tile_elems + woff < a.nelem)
                    tile_issue<KQ, CB>(src, t2 * tile_elems + woff, c, g, a, A);
                const int64_t eb = t1 * tile_elems + woff;
                if (eb < a.nelem) tile_compute<KQ, CB>(B, eb, p_lo, np, dl, out, a, c, g);
                if (!more2) break;
                vm_wait_below(eb < a.nelem ? tile_stores_min<CB>(np, eb + 16 * CB <= a.nelem) : 0);
                tile_settle(A);
                t0 = t2;
            }
            return;
        }
    }
    for (int64_t tile = stream; tile < a.ntiles; tile += a.nstreams) {
        const int64_t e0 = tile * tile_elems + (int64_t)wave * 16 * CB;
        if (e0 >= a.nelem) continue;  // whole wave past the end (no block-level sync below)

        T b[NSEG][CB][KQ];
        if (a.vec_in) {
#pragma unroll
            for (int s = 0; s < NSEG; ++s)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    load_b_global<T, KQ>(src + s * a.seg_stride, e0 + cb * 16 + c, g, a, b[s][cb]);
        } else if (!a.use_slab) {
            // unaligned rows too long for a wave slab: 16-byte vectors from
            // element-size boundaries, row tails value by value
#pragma unroll
            for (int s = 0; s < NSEG; ++s)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int64_t e = e0 + cb * 16 + c;
                    const bool ok = e < a.nelem;
                    const T* row = src + s * a.seg_stride + (ok ? e : 0) * nunit + g * KQ;
#pragma unroll
                    for (int t = 0; t < KQ; t += V) {
                        const vec_t v = load_vec_any<T>(row + t, ok, nunit - g * KQ - t);
#pragma unroll
                        for (int q = 0; q < V; ++q) b[s][cb][t + q] = v[q];
                    }
                }
        } else {
            const int nel = (int)min<int64_t>(16 * CB, a.nelem - e0);
#pragma unroll
            for (int s = 0; s < NSEG; ++s)
                stage_slab<T>(src + s * a.seg_stride, e0, nel, nunit, a.src_aligned,
                              slab + s * slab_seg, lane);
            wave_lds_sync();
#pragma unroll
            for (int s = 0; s < NSEG; ++s)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int el = cb * 16 + c;
                    const T* row = slab + s * slab_seg + el * nunit + g * KQ;
#pragma unroll
                    for (int t = 0; t < KQ; ++t)
                        b[s][cb][t] = (el < nel && g * KQ + t < nunit) ? row[t] : T(0);
                }
            wave_lds_sync();  // slab reads done before the next tile overwrites it
        }

        const int nel_w = (int)min<int64_t>(16 * CB, a.nelem - e0);  // valid elements of the wave
        int pp_first = 0;
        if constexpr (PAIR) {
            static_assert(V == 4 && NSEG == 1 && !ACC, "paired stores: FP32 forward only");
            pp_first = paired_panels<KQ, CB>(b[0], e0, p_lo, np, dl, out, a, c, g);
        }
        for (int pp = pp_first; pp < np; ++pp) {
            const int panel = p_lo + pp;
            const int slab_o = panel / a.mblk;
            const int i0 = (panel % a.mblk) * 16;
            acc_t acc[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[cb] = acc_t(T(0));
#pragma unroll
            for (int s = 0; s < NSEG; ++s) {
                const T* arow = dl + (pp * 16 + c) * LD + s * KP + g * KQ;
#pragma unroll
                for (int t = 0; t < KQ; t += V) {
                    const vec_t av = *reinterpret_cast<const vec_t*>(arow + t);
#pragma unroll
                    for (int q = 0; q < V; ++q)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            acc[cb] = Mma<T>::step(av[q], b[s][cb][t + q], acc[cb]);
                }
            }
            // Lane holds the results for nodes i0+4g .. i0+4g+3 of element column c.
            const int i = i0 + 4 * g;
            if (a.stage_out) {
                // rows [r_lo, r_hi) of output slab slab_o belong to this group;
                // they are collected in the wave's slab (free once the element
                // data sit in registers) and written when the slab's last
                // panel of the group is done
                const int pf = max(p_lo, slab_o * a.mblk);
                const int pl = min(p_lo + np, (slab_o + 1) * a.mblk);
                const int r_lo = (pf - slab_o * a.mblk) * 16;
                const int rows = min((pl - slab_o * a.mblk) * 16, nunit) - r_lo;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int el = cb * 16 + c;
                    if (el >= nel_w) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i + r < nunit) slab[el * rows + (i + r - r_lo)] = acc[cb][r];
                }
                if (panel + 1 == pl) {
                    wave_lds_sync();
                    write_staged<T, ACC>(slab, out + ((int64_t)slab_o * a.nelem + e0) * nunit, nel_w,
                                         rows, r_lo, nunit, lane, a.nt_store != 0);
                    wave_lds_sync();  // staged values read before the slab is reused
                }
                continue;
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                if (e >= a.nelem) continue;
                T* dst = out + ((int64_t)slab_o * a.nelem + e) * nunit + i;
                if constexpr (ACC) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i + r < nunit) acc[cb][r] += dst[r];
                }
                if (a.vec_out) {
                    if (i < nunit) {
                        if constexpr (V == 4) {
                            if (a.nt_store) {
                                // streaming store through a buffer view of the
                                // wave-tile's rows of this slab
                                const int nel = (int)min<int64_t>(16 * CB, a.nelem - e0);
                                const __amdgpu_buffer_rsrc_t rs = wave_buffer(
                                    out + ((int64_t)slab_o * a.nelem + e0) * nunit, nel * nunit * 4);
                                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, acc[cb]), rs,
                                                                       ((cb * 16 + c) * nunit + i) * 4, 0,
                                                                       kStreamStore);
                            } else {
                                *reinterpret_cast<f32x4*>(dst) = acc[cb];
                            }
                        } else {
                            f64x2 lo = {acc[cb][0], acc[cb][1]};
                            f64x2 hi = {acc[cb][2], acc[cb][3]};
                            reinterpret_cast<f64x2*>(dst)[0] = lo;
                            reinterpret_cast<f64x2*>(dst)[1] = hi;
                        }
                    }
                } else if (i < nunit) {
                    // unaligned row: 16-byte vectors from element-size
                    // boundaries, the row tail value by value
#pragma unroll
                    for (int h = 0; h < 4 / V; ++h) {
                        const int av = nunit - i - h * V;
                        vec_t w;
#pragma unroll
                        for (int t = 0; t < V; ++t) w[t] = acc[cb][h * V + t];
                        if (av >= V) {
                            __builtin_memcpy(dst + h * V, &w, 16);
                        } else {
#pragma unroll
                            for (int t = 0; t < V - 1; ++t)
                                if (t < av) dst[h * V + t] = w[t];
                        }
                    }
                }
            }
        }
    }
}

typedef void (*kern_fn)(KArgs);

// KQ values instantiated: every node count up to 512 is covered by the next
// listed value (KQ >= ceil(nunit/4) rounded up to 4).
#define DG_KQ_LIST(X) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) \
    X(72) X(80) X(88) X(96) X(112) X(128)

inline int kq_for(int nunit) {
    static const int kKQ[] = {
#define X(k) k,
        DG_KQ_LIST(X)
#undef X
    };
    const int need = (int)round_up(ceil_div(nunit, 4), 4);
    for (int k : kKQ)
        if (k >= need) return k;
    return -1;
}

// Register budget of the B fragments: CB*NSEG*KQ values of T per lane.
template <typename T, int CB, int NSEG, int KQ>
constexpr bool fits_registers() {
    return CB * NSEG * KQ * sizeof(T) <= (NSEG == 1 ? 1024u : 768u);
}

// pair: the paired-store variant (FP32 single-segment forward only; null
// otherwise)
template <typename T, int CB, int NSEG>
kern_fn pick_kernel(int kq, bool pair = false) {
#define X(k)                                                                    \
    if constexpr (fits_registers<T, CB, NSEG, k>()) {                           \
        if (kq == k) {                                                          \
            if (!pair) return dg_kernel<T, k, CB, NSEG>;                        \
            if constexpr (sizeof(T) == 4 && NSEG == 1)                          \
                return dg_kernel<T, k, CB, NSEG, false, true>;                  \
            return nullptr;                                                     \
        }                                                                       \
    }
    DG_KQ_LIST(X)
#undef X
    return nullptr;
}

constexpr size_t kLdsBudget = 64 * 1024;  // default: whole stack if it fits here
constexpr size_t kLdsMax = 160 * 1024;    // gfx950 LDS per CU

// The launch plan of one contraction: a pure function of the problem, the
// explicit launch shape and the device's CU count (shared with the feature
// counter, so counts follow the launched schedule exactly).
struct Plan {
    int kq, cb, waves, nseg;
    int mblk, panels_total, ppg, ngroups;
    int64_t ntiles, slots, grid;
    int vec_in, use_slab;
    size_t smem, panel_bytes, slab_bytes;
};

// per_cu: resident work-groups per CU (explicit, > 0).
inline dg_status make_plan(size_t tsize, int nseg, int out_slabs, int64_t nelem, int nunit, int kq,
                           int cb, int waves, int d_panels, int per_cu, int num_cu, bool src_vec_ok,
                           Plan* P) {
    const int V = (int)(16 / tsize);
    P->kq = kq;
    P->cb = cb;
    P->waves = waves;
    P->nseg = nseg;
    P->mblk = (int)ceil_div(nunit, 16);
    P->panels_total = out_slabs * P->mblk;
    P->panel_bytes = (size_t)16 * (nseg * 4 * kq + V) * tsize;
    P->vec_in = src_vec_ok ? 1 : 0;
    size_t slab = P->vec_in ? 0 : (size_t)waves * nseg * round_up(16 * cb * nunit, V) * tsize;
    P->use_slab = slab > 0 && slab + P->panel_bytes <= kLdsMax / 2;
    if (!P->use_slab) slab = 0;
    P->slab_bytes = slab;
    int ppg;
    if (d_panels > 0) {
        ppg = std::min(d_panels, P->panels_total);
    } else {
        const size_t budget = kLdsBudget > slab ? kLdsBudget - slab : 0;
        if ((size_t)P->panels_total * P->panel_bytes <= budget) {
            ppg = P->panels_total;
        } else {
            const size_t room = kLdsMax - slab;
            const int fit = std::max<int>(1, (int)(room / P->panel_bytes));
            const int groups = (int)ceil_div(P->panels_total, fit);
            ppg = (int)ceil_div(P->panels_total, groups);
        }
    }
    P->ppg = ppg;
    P->ngroups = (int)ceil_div(P->panels_total, ppg);
    P->smem = (size_t)ppg * P->panel_bytes + slab;
    if (P->smem > kLdsMax) return fail(DG_EINVAL, "tile.d_panels exceeds the 160 KB LDS");
    P->ntiles = ceil_div(nelem, (int64_t)16 * cb * waves);
    // blocks per XCD per group: fill the resident capacity, no more streams than tiles
    const int64_t cap = std::max<int64_t>(1, (int64_t)per_cu * num_cu / (8 * P->ngroups));
    P->slots = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(P->ntiles, 8)));
    P->grid = 8 * P->ngroups * P->slots;
    return DG_OK;
}

// The paired-store variant applies to FP32 rows of a multiple of 32 nodes
// written as 16-byte vectors, with an even number of panels per group.
inline bool pair_eligible(size_t tsize, int nunit, bool vec_out, const Plan& P) {
    return tsize == 4 && vec_out && nunit % 32 == 0 && P.mblk % 2 == 0 && P.ppg % 2 == 0;
}

// Paired-store launches whose element fragments are small (KQ * CB <= 32)
// and come as 16-byte vectors take the pipelined element loads; these load
// every row of a wave-tile that starts before the end (rows past it clamp to
// the last element).
inline bool pipelined_loads(size_t tsize, int nunit, int kq, int cb, bool vec_out, const Plan& P) {
    return pair_eligible(tsize, nunit, vec_out, P) && kq * cb <= 32 && P.vec_in;
}

// Launch one contraction with the kernel fn (or fn_pair where the paired
// stores apply); tile->groups_per_cu == 0 means "occupancy maximum" (queried
// for the kernel launched).
// stream_out: the launch writes an output nothing reads back before the
// launch ends (the forward), so it may stream it (see below)
template <typename T, int NSEG>
dg_status launch(KArgs a, int out_slabs, int kq, int cb, const dg_tile* tile, int waves, kern_fn fn,
                 hipStream_t s, kern_fn fn_pair = nullptr, int* per_cu_used = nullptr,
                 bool stream_out = false) {
    if (!fn) return fail(DG_EUNSUPPORTED, "no DG kernel instance for this shape");
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    {
        hipFuncAttributes fa;
        DG_HIP_CHECK(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(fn)));
        if (64 * waves > fa.maxThreadsPerBlock)
            return fail(DG_EINVAL, "tile.waves above 4 needs a shape whose element data fit 64 registers");
    }
    const bool src_vec_ok = (a.nunit % Mma<T>::V == 0) &&
                            (reinterpret_cast<uintptr_t>(a.src) % 16 == 0) &&
                            (a.seg_stride % Mma<T>::V == 0);
    Plan P;
    // first pass with a provisional occupancy to size the LDS request
    st = make_plan(sizeof(T), NSEG, out_slabs, a.nelem, a.nunit, kq, cb, waves,
                   tile ? tile->d_panels : 0, 1, dev.num_cu, src_vec_ok, &P);
    if (st != DG_OK) return st;
    const bool vec_out = (a.nunit % 4 == 0) && (reinterpret_cast<uintptr_t>(a.out) % 16 == 0);
    if (fn_pair && pair_eligible(sizeof(T), a.nunit, vec_out, P)) fn = fn_pair;
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
    int per_cu = (tile && tile->groups_per_cu > 0) ? tile->groups_per_cu : 0;
    if (per_cu == 0) {
        DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(fn), 64 * waves, P.smem));
        if (per_cu < 1) per_cu = 1;
    }
    st = make_plan(sizeof(T), NSEG, out_slabs, a.nelem, a.nunit, kq, cb, waves,
                   tile ? tile->d_panels : 0, per_cu, dev.num_cu, src_vec_ok, &P);
    if (st != DG_OK) return st;
    if (per_cu_used) *per_cu_used = per_cu;
    a.ntiles = P.ntiles;
    a.mblk = P.mblk;
    a.panels_total = P.panels_total;
    a.ppg = P.ppg;
    a.ngroups = P.ngroups;
    a.nstreams = (int)(8 * P.slots);
    a.vec_in = P.vec_in;
    a.src_aligned = reinterpret_cast<uintptr_t>(a.src) % 16 == 0;
    a.use_slab = P.use_slab;
    a.vec_out = vec_out;
    a.stage_out = a.use_slab && !a.vec_out;
    // streaming output stores on request, and by default for a forward
    // whose one operator group holds every panel: then no other work-group
    // re-reads an element tile, the output is never read back, and keeping
    // it out of the L2 measured faster (FP32 at 2^21 elements: p = 2 0.194 ->
    // 0.178 ms, p = 3 0.464 -> 0.444 ms; p = 1 at 2^22 0.157 -> 0.125 ms);
    // with several groups re-reading tiles from the L2 (p = 5, 7) it
    // measured slower
    a.nt_store = ((tile && (tile->flags & DG_TILE_NT_STORE)) || (stream_out && P.ngroups == 1)) ? 1 : 0;
    hipLaunchKernelGGL(fn, dim3((unsigned)P.grid), dim3(64 * waves), P.smem, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

// Column blocks per wave of the forward kernel: the measured default when the
// tile leaves it open (FP32, 2^21 elements: aligned short rows favour one
// column block per wave, i.e. more waves in flight; otherwise more column
// blocks, as registers allow), else the requested one.
inline dg_status forward_cb(size_t tsize, int kq, bool rows_aligned, int epw, int* cb) {
    if (epw == 0) {
        const int w = kq * (int)tsize / 4;  // KQ in 32-bit registers
        if (tsize == 4) {
            // FP32, measured on the hexahedral orders at 2^21 elements (with
            // the wave counts of forward_waves): p = 3 one column block, p = 2
            // and p = 4 (rows off 16-byte boundaries) two, p = 5 one
            if (w <= 16) *cb = rows_aligned ? 1 : 2;
            else if (w <= 32) *cb = 2;
            else *cb = 1;
        } else {
            if (w <= 16) *cb = 1;
            else if (w <= 32) *cb = 4;
            else if (w <= 64) *cb = 2;
            else *cb = 1;
        }
    } else if (epw == 16) {
        *cb = 1;
    } else if (epw == 32) {
        *cb = 2;
    } else if (epw == 64 && kq * (int)tsize <= 32 * 4) {
        *cb = 4;
    } else {
        return fail(DG_EINVAL,
                    "tile.elems_per_wave must be 16 or 32 (or 64 for nunit <= 128 in FP32)");
    }
    return DG_OK;
}

// Default waves per work-group: 8 (two copies' worth of waves sharing one
// set of resident operator panels) where the variant allows 512 threads and
// it measured faster -- FP32 rows off 16-byte boundaries, FP32 rows of 128 or
// more nodes per lane group, and the pipelined paired-store shapes (rows of
// a multiple of 32 nodes, KQ * CB <= 32) -- else 4.
inline int forward_waves(size_t tsize, int nunit, int kq, int cb, bool rows_aligned) {
    const bool fits = cb * kq * (int)tsize <= 256;  // dg_max_threads() == 512
    const bool piped = rows_aligned && nunit % 32 == 0 && kq * cb <= 32;
    if (tsize == 4 && fits && (!rows_aligned || kq >= 32 || piped)) return 8;
    return 4;
}

// Split plan of grad_D (the backward's split-K GEMM over elements): a pure
// function of the problem, the partial kernel's resident work-groups per CU
// and the CU count (shared with the feature counter).  As many splits as make
// one full round of resident work-groups -- a second, partial round would
// leave most of the GPU idle at the end -- and at most one per 256 elements;
// a non-zero cap_bytes bounds the workspace (partials plus group sums)
// instead: fewer, longer splits.
constexpr int kBwdTile = 128;     // output tile (rows i x cols j)
constexpr int kBwdChunk = 16;     // elements per LDS chunk
constexpr int64_t kBwdRedGroup = 16;  // splits summed per first-stage group

struct SplitPlan {
    int64_t nsplit;
    int64_t split_len;  // elements per split (multiple of kBwdChunk)
    int64_t ngroups;    // ceil(nsplit / kBwdRedGroup)
};

inline bool bwd_split_plan(int nmat, int64_t nelem, int nunit, int per_cu, int num_cu, size_t tsize,
                           size_t cap_bytes, SplitPlan* sp) {
    const int64_t tiles = (int64_t)nmat * ceil_div(nunit, kBwdTile) * ceil_div(nunit, kBwdTile);
    const int64_t target = (int64_t)std::max(per_cu, 1) * num_cu;
    int64_t ns = std::max<int64_t>(1, target / tiles);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, ceil_div(nelem, 256)));
    if (cap_bytes) {
        // nsplit + ceil(nsplit / kBwdRedGroup) partial tiles must fit
        const int64_t count_bytes = (int64_t)nmat * nunit * nunit * (int64_t)tsize;
        const int64_t fit = (int64_t)(cap_bytes / (size_t)count_bytes);
        int64_t cap = fit;
        while (cap > 0 && cap + ceil_div(cap, kBwdRedGroup) > fit) --cap;
        if (cap < 1) return false;
        ns = std::min(ns, cap);
    }
    const int64_t len = round_up(ceil_div(std::max<int64_t>(nelem, 1), ns), (int64_t)kBwdChunk);
    sp->nsplit = std::max<int64_t>(1, ceil_div(nelem, len));
    sp->split_len = len;
    sp->ngroups = ceil_div(sp->nsplit, kBwdRedGroup);
    return true;
}

// grad_u on the contraction kernel: the operator transposed, the nmat slabs
// of g as contraction segments of one launch when an instance with that many
// segments exists and its fragments fit the registers, else one launch per
// operator (later launches accumulate).  Returns the segments per launch.
inline int grad_u_segments(size_t tsize, int nmat, int kq) {
    return (nmat <= 3 && (nmat == 1 || (size_t)nmat * kq * tsize <= 768)) ? nmat : 1;
}

}  // namespace kern
}  // namespace dg
