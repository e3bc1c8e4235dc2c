// DG differentiation, FP32 and FP64, on the gfx950 matrix cores.
//
// The operation (paper, Section "DG Differentiation") is
//     out[m][e][i] = sum_j D[m][i][j] * u[e][j],
// i.e. for every operator m a product of the small square D_m with the
// element data.  Stacking the operators' rows, it is one tall-skinny GEMM
//     C^T[(m,i)][e] = sum_j D[(m,i)][j] * U^T[j][e]
// whose long dimension is the element count.  This kernel computes C^T with
// v_mfma_{f32,f64}_16x16x4: A = a 16-row panel of the operator stack, B = the
// data of 16 elements, so that the accumulator of each lane holds four
// consecutive output nodes i of one element — a 16-byte (FP32) store into the
// element-major output slab out[m].
//
// Contraction order.  Lane group g = lane/16 supplies the MFMA's k index; we
// give group g the node range j in [g*KQ, (g+1)*KQ) and walk it with step s,
// so k-step s contracts j = g*KQ + s for g = 0..3.  Each lane therefore reads
// KQ *contiguous* nodes of its element (vector loads straight from HBM, no LDS
// staging for u) and KQ contiguous entries of one operator row (16-byte LDS
// reads).  The padded node count is KP = 4*KQ >= nunit; padding is zero in
// registers and LDS only and never reaches HBM.
//
// Row order.  The f32 instruction returns rows 4g..4g+3 to lane group g; the
// f64 one returns rows g, g+4, g+8, g+12.  Panels are staged into LDS in the
// matching row order, so either way a lane's four results are the consecutive
// nodes i0+4g .. i0+4g+3.
//
// Operator residency.  The stack has nmat*ceil(nunit/16) panels of 16 rows.
// They are split into `ngroups` groups of at most `ppg` panels, each small
// enough for LDS; a work-group stages ONE group once and keeps it for its whole
// life, computing only those output rows for every element tile it visits.
// Operators are never re-staged inside the tile loop.
//
// Grid (persistent, XCD-aware).  Work-groups are dispatched round-robin over
// the 8 XCDs (block b lands on XCD b % 8).  Block b takes panel group
// pg = (b/8) % ngroups and tile stream (b/8)/ngroups * 8 + b % 8, so the
// ngroups blocks that need the same element tile sit on the same XCD and walk
// the same tile sequence: the tile is fetched from HBM once and re-read from
// that XCD's L2 by the other groups.
//
// Unaligned rows.  When nunit is not a multiple of the 16-byte vector (or u is
// not 16-byte aligned) a wave copies its contiguous slab of element data into
// a wave-private LDS area with aligned 16-byte loads and reads its fragments
// from there.
#include "common.hpp"

namespace dg {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
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

struct FwdArgs {
    const void* D;
    const void* u;
    void* out;
    int64_t nelem;
    int64_t ntiles;
    int nmat;
    int nunit;
    int mblk;          // 16-row panels per operator: ceil(nunit/16)
    int panels_total;  // nmat * mblk
    int ppg;           // panels per resident group
    int ngroups;       // ceil(panels_total / ppg)
    int nstreams;      // tile streams: 8 * (blocks per XCD per group)
    int vec_in;        // u rows may be read as 16-byte vectors
    int u_aligned;     // u itself is 16-byte aligned
    int use_slab;      // unaligned rows go through the wave-private LDS slab
    int vec_out;       // out rows may be written as 16-byte vectors
    int nt_store;      // streaming (non-temporal) output stores
};

__device__ inline int round_up_dev(int x, int v) { return (x + v - 1) / v * v; }

template <typename T, int KQ>
__device__ inline void stage_panels(const T* __restrict__ D, T* dl, int p0, int np,
                                    int nunit, int mblk) {
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + Mma<T>::V;
    const int total = np * 16 * KP;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int j = idx % KP;
        const int rr = idx / KP;  // operator row within the staged group
        const int rn = rr % 16;   // node offset 4g + r within its panel
        const int panel = p0 + rr / 16;
        const int m = panel / mblk;
        const int i = (panel % mblk) * 16 + rn;
        T v = T(0);
        if (i < nunit && j < nunit) v = D[((int64_t)m * nunit + i) * nunit + j];
        // Place node 4g + r at the panel row whose accumulator lands in
        // register r of lane group g, so every lane ends up with four
        // consecutive nodes of its element.
        const int rho = Mma<T>::acc_row(rn >> 2, rn & 3);
        dl[(rr - rn + rho) * LD + j] = v;
    }
}

// B fragments of one 16-element column block straight from global memory:
// KQ contiguous nodes of the lane's element from node g*KQ; zero beyond nunit
// or nelem.  Requires 16-byte aligned rows (vec_in).
template <typename T, int KQ>
__device__ inline void load_b_global(const T* __restrict__ u, int64_t e, int g, const FwdArgs& a,
                                     T (&b)[KQ]) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    const bool ev = e < a.nelem;
    const T* src = u + (ev ? e : 0) * a.nunit + g * KQ;
#pragma unroll
    for (int s = 0; s < KQ; s += V) {
        vec_t v = vec_t(T(0));
        if (ev && g * KQ + s < a.nunit) v = *reinterpret_cast<const vec_t*>(src + s);
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
// at element ew0, whose start is 16-byte aligned) into wave-private LDS.
template <typename T>
__device__ inline void stage_slab(const T* __restrict__ u, int64_t ew0, int nel, int nunit,
                                  bool aligned, T* slab, int lane) {
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    const int len = nel * nunit;
    const T* src = u + ew0 * nunit;
    // ew0 is a multiple of 16, so the slab starts 16-byte aligned iff u does
    const int nvec = aligned ? len / V : 0;
    for (int q = lane; q < nvec; q += 64)
        reinterpret_cast<vec_t*>(slab)[q] = reinterpret_cast<const vec_t*>(src)[q];
    for (int f = nvec * V + lane; f < len; f += 64) slab[f] = src[f];
}

template <typename T, int KQ, int CB>
__global__ void __launch_bounds__(256) dg_fwd_kernel(FwdArgs a) {
    typedef typename Mma<T>::acc_t acc_t;
    typedef typename Mma<T>::vec_t vec_t;
    constexpr int V = Mma<T>::V;
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + V;  // one vector of row padding against bank conflicts

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T* dl = reinterpret_cast<T*>(smem);
    const T* __restrict__ D = static_cast<const T*>(a.D);
    const T* __restrict__ u = static_cast<const T*>(a.u);
    T* __restrict__ out = static_cast<T*>(a.out);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int c = lane & 15;  // MFMA column: the element within a 16-block
    const int g = lane >> 4;  // MFMA k index: which quarter of the nodes
    const int nunit = a.nunit;

    // XCD-aware placement: see the file comment.
    const int xcd = blockIdx.x & 7;
    const int k = blockIdx.x >> 3;
    const int pg = k % a.ngroups;
    const int64_t stream = (int64_t)(k / a.ngroups) * 8 + xcd;
    const int p_lo = pg * a.ppg;
    const int np = min(a.ppg, a.panels_total - p_lo);

    stage_panels<T, KQ>(D, dl, p_lo, np, nunit, a.mblk);
    // wave-private slab for unaligned element rows, after the operator panels
    T* slab = dl + (size_t)a.ppg * 16 * LD + (size_t)wave * round_up_dev(16 * CB * nunit, V);
    __syncthreads();

    const int64_t tile_elems = (int64_t)nw * 16 * CB;
    for (int64_t tile = stream; tile < a.ntiles; tile += a.nstreams) {
        const int64_t e0 = tile * tile_elems + (int64_t)wave * 16 * CB;
        if (e0 >= a.nelem) continue;  // whole wave past the end (no block-level sync below)

        T b[CB][KQ];
        if (a.vec_in) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) load_b_global<T, KQ>(u, e0 + cb * 16 + c, g, a, b[cb]);
        } else if (!a.use_slab) {
            // unaligned rows too long for a wave slab: masked scalar loads
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                const T* row = u + (e < a.nelem ? e : 0) * nunit + g * KQ;
#pragma unroll
                for (int s = 0; s < KQ; ++s)
                    b[cb][s] = (e < a.nelem && g * KQ + s < nunit) ? row[s] : T(0);
            }
        } else {
            const int nel = (int)min<int64_t>(16 * CB, a.nelem - e0);
            stage_slab<T>(u, e0, nel, nunit, a.u_aligned, slab, lane);
            wave_lds_sync();
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int el = cb * 16 + c;
                const T* row = slab + el * nunit + g * KQ;
#pragma unroll
                for (int s = 0; s < KQ; ++s)
                    b[cb][s] = (el < nel && g * KQ + s < nunit) ? row[s] : T(0);
            }
            wave_lds_sync();  // slab reads done before the next tile overwrites it
        }

        for (int pp = 0; pp < np; ++pp) {
            const int panel = p_lo + pp;
            const int m = panel / a.mblk;
            const int i0 = (panel % a.mblk) * 16;
            acc_t acc[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[cb] = acc_t(T(0));
            const T* arow = dl + (pp * 16 + c) * LD + g * KQ;
#pragma unroll
            for (int s = 0; s < KQ; s += V) {
                const vec_t av = *reinterpret_cast<const vec_t*>(arow + s);
#pragma unroll
                for (int t = 0; t < V; ++t)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[cb] = Mma<T>::step(av[t], b[cb][s + t], acc[cb]);
            }
            // Lane holds the results for nodes i0+4g .. i0+4g+3 of element column c.
            const int i = i0 + 4 * g;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t e = e0 + cb * 16 + c;
                if (e >= a.nelem) continue;
                T* dst = out + ((int64_t)m * a.nelem + e) * nunit + i;
                if (a.vec_out) {
                    if (i < nunit) {
                        if constexpr (V == 4) {
                            if (a.nt_store)
                                __builtin_nontemporal_store(acc[cb], reinterpret_cast<f32x4*>(dst));
                            else
                                *reinterpret_cast<f32x4*>(dst) = acc[cb];
                        } else {
                            f64x2 lo = {acc[cb][0], acc[cb][1]};
                            f64x2 hi = {acc[cb][2], acc[cb][3]};
                            reinterpret_cast<f64x2*>(dst)[0] = lo;
                            reinterpret_cast<f64x2*>(dst)[1] = hi;
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (i + r < nunit) dst[r] = acc[cb][r];
                }
            }
        }
    }
}

typedef void (*fwd_fn)(FwdArgs);

// KQ values instantiated: every multiple of 4 a node count up to 512 needs is
// covered by the next listed value (KQ >= ceil(nunit/4) rounded to 4).
#define DG_KQ_LIST(X) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64) \
    X(72) X(80) X(88) X(96) X(112) X(128)

static const int kKQ[] = {
#define X(k) k,
    DG_KQ_LIST(X)
#undef X
};

template <typename T, int CB>
fwd_fn pick_kernel(int kq) {
#define X(k)                                                   \
    if constexpr (CB < 4 || k * sizeof(T) <= 32 * 4) {         \
        if (kq == k) return dg_fwd_kernel<T, k, CB>;           \
    }
    DG_KQ_LIST(X)
#undef X
    return nullptr;
}

int kq_for(int nunit) {
    int need = (int)round_up(ceil_div(nunit, 4), 4);
    for (int k : kKQ)
        if (k >= need) return k;
    return -1;
}

constexpr size_t kLdsBudget = 64 * 1024;   // default staging budget: 2 groups per CU
constexpr size_t kLdsMax = 160 * 1024;     // gfx950 LDS per CU

template <typename T>
dg_status launch_t(int nmat, int64_t nelem, int nunit, const void* D, const void* u, void* out,
                   const dg_tile* tile, hipStream_t s) {
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;

    int waves = (tile && tile->waves) ? tile->waves : 4;
    int epw = (tile && tile->elems_per_wave) ? tile->elems_per_wave : 0;
    if (waves < 1 || waves > 4) return fail(DG_EINVAL, "tile.waves must be in 1..4");
    int cb;
    const bool rows_aligned = (nunit % Mma<T>::V == 0) && (reinterpret_cast<uintptr_t>(u) % 16 == 0);
    if (epw == 0) {
        // measured defaults (FP32, 2^21 elements): aligned short rows favour one
        // column block per wave (more waves in flight); otherwise more column
        // blocks per wave, as registers allow
        const int w = kq * (int)sizeof(T) / 4;  // KQ in 32-bit registers
        if (rows_aligned && w <= 16) cb = 1;
        else if (w <= 32) cb = 4;
        else if (w <= 64) cb = 2;
        else cb = 1;
    }
    else if (epw == 16) cb = 1;
    else if (epw == 32) cb = 2;
    else if (epw == 64 && kq * (int)sizeof(T) <= 32 * 4) cb = 4;
    else return fail(DG_EINVAL, "tile.elems_per_wave must be 16 or 32 (or 64 for nunit <= 128 in FP32)");

    const int mblk = (int)ceil_div(nunit, 16);
    const int panels_total = nmat * mblk;
    const size_t panel_bytes = (size_t)16 * (4 * kq + Mma<T>::V) * sizeof(T);
    const bool vec_in = (nunit % Mma<T>::V == 0) && (reinterpret_cast<uintptr_t>(u) % 16 == 0);
    size_t slab_bytes =
        vec_in ? 0 : (size_t)waves * round_up(16 * cb * nunit, Mma<T>::V) * sizeof(T);
    const bool use_slab = slab_bytes > 0 && slab_bytes + panel_bytes <= kLdsMax / 2;
    if (!use_slab) slab_bytes = 0;
    int ppg;
    if (tile && tile->d_panels > 0) {
        ppg = std::min(tile->d_panels, panels_total);
    } else {
        // Whole stack if it fits the default budget; else the fewest groups
        // (balanced) whose panels fit the LDS next to the slabs.
        const size_t budget = kLdsBudget > slab_bytes ? kLdsBudget - slab_bytes : 0;
        if ((size_t)panels_total * panel_bytes <= budget) {
            ppg = panels_total;
        } else {
            const size_t room = kLdsMax - slab_bytes;
            const int fit = std::max<int>(1, (int)(room / panel_bytes));
            const int groups = (int)ceil_div(panels_total, fit);
            ppg = (int)ceil_div(panels_total, groups);
        }
    }
    const int ngroups = (int)ceil_div(panels_total, ppg);
    const size_t smem = (size_t)ppg * panel_bytes + slab_bytes;
    if (smem > kLdsMax) return fail(DG_EINVAL, "tile.d_panels exceeds the 160 KB LDS");

    fwd_fn fn = (cb == 4) ? pick_kernel<T, 4>(kq) : (cb == 2) ? pick_kernel<T, 2>(kq) : pick_kernel<T, 1>(kq);
    if (!fn) return fail(DG_EUNSUPPORTED, "no DG kernel instance for this nunit");
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));

    const int block = 64 * waves;
    const int64_t tile_elems = (int64_t)16 * cb * waves;
    const int64_t ntiles = ceil_div(nelem, tile_elems);
    int per_cu = (tile && tile->groups_per_cu > 0) ? tile->groups_per_cu : 0;
    if (per_cu == 0) {
        DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(fn), block, smem));
        if (per_cu < 1) per_cu = 1;
    }
    // blocks per XCD per group: fill the resident capacity, but no more
    // streams than tiles.
    const int64_t cap = std::max<int64_t>(1, (int64_t)per_cu * dev.num_cu / (8 * ngroups));
    const int64_t slots = std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(ntiles, 8)));
    const int64_t grid = 8 * ngroups * slots;

    FwdArgs a;
    a.D = D;
    a.u = u;
    a.out = out;
    a.nelem = nelem;
    a.ntiles = ntiles;
    a.nmat = nmat;
    a.nunit = nunit;
    a.mblk = mblk;
    a.panels_total = panels_total;
    a.ppg = ppg;
    a.ngroups = ngroups;
    a.nstreams = (int)(8 * slots);
    a.vec_in = vec_in;
    a.u_aligned = reinterpret_cast<uintptr_t>(u) % 16 == 0;
    a.use_slab = use_slab;
    a.vec_out = (nunit % 4 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    a.nt_store = (tile && (tile->flags & DG_TILE_NT_STORE)) ? 1 : 0;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), smem, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace

dg_status launch_dg_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                               const void* u, void* out, const dg_tile* tile, hipStream_t s) {
    if (t == DG_F32) return launch_t<float>(nmat, nelem, nunit, D, u, out, tile, s);
    if (t == DG_F64) return launch_t<double>(nmat, nelem, nunit, D, u, out, tile, s);
    return fail(DG_EUNSUPPORTED, "launch_dg_forward_fp: dtype");
}

}  // namespace dg
