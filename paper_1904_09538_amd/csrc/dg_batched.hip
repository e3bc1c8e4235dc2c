// Mixed-order DG differentiation in one persistent launch (FP32).
//
// Elements of hexahedral order p = 1..7 (nunit = (p+1)^3) are stored ragged
// and element-major: element e's nodes at u_packed[off[e] .. off[e]+n_e), its
// outputs at out_packed[m*total + off[e] + i] (total = sum_e n_e), with its
// own operator stack D^(p_e) [3][n_e][n_e].  Per element the operation is the
// plain one, out[m][i] = sum_j D^(p)[m][i][j] u[j].
//
// Plan (host, once): a counting sort groups the element ids by order; for
// each order a launch shape (column blocks per wave, operator panels resident
// per work-group) is chosen -- by the caller, or by ranking the candidates
// with the calibrated performance model (the paper's intended use: rank
// equivalent variants and prune the tuning space).  The work-groups of the
// persistent grid are then split across orders in proportion to each
// order's predicted time, so that all orders finish together.
//
// Kernel: a work-group finds its order from the block ranges, then runs the
// same contraction as the plain kernel (operator panels resident in LDS, XCD
// aware tile streams within the order's block range) on a gathered list of
// element ids.  Rows start at arbitrary 4-byte offsets in the packed layout;
// element data are still read, and results written, as 16-byte vectors
// (unaligned vector accesses, with value-by-value row tails).  Order 1 takes
// one element per thread, orders 6 and 7 a GEMM tiling (see below).
#include <algorithm>
#include <cmath>
#include <set>
#include <vector>

#include "dg_kernel.hpp"

namespace dg {

struct BOrder {
    const float* D;     // [3][n][n] (filled in at launch)
    int64_t count;      // elements of this order
    int64_t ids;        // start of this order's ids in the sorted id list
    int64_t ntiles;
    int nunit, mblk, panels_total, ppg, ngroups, nstreams;
    int variant;        // kernel body (order, column blocks)
    int cb;
};

struct BArgs {
    const float* u;
    float* out;
    const int64_t* perm;  // element ids sorted by order
    const int64_t* off;   // [nelem+1] node offsets
    int64_t total;        // sum of nunit over elements
    int nmat;
    int waves;
    int64_t blk_lo[9];    // block range of order p: [blk_lo[p], blk_lo[p+1])
    BOrder ord[8];
    int* ctr;             // [9]: GEMM tile pool cursor per XCD, finished work-groups
    int pool;             // some order runs on the GEMM body
};

namespace {

using namespace kern;

// Four consecutive values of a row that starts at any 4-byte boundary:
// `avail` values from p on belong to the row; the rest read as zero.  A
// full in-range vector is one 16-byte load (the 16-byte copy from a 4-byte
// aligned address is left to the compiler, which issues a single vector load
// on this target); row tails are loaded value by value.
__device__ inline f32x4 load4(const float* p, bool ok, int avail) {
    f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
    if (!ok || avail <= 0) return v;
    if (avail >= 4) {
        __builtin_memcpy(&v, p, 16);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (q < avail) v[q] = p[q];
    }
    return v;
}

__device__ inline void store4(float* p, f32x4 v, int avail) {
    if (avail >= 4) {
        __builtin_memcpy(p, &v, 16);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (q < avail) p[q] = v[q];
    }
}

template <int KQ, int CB>
__device__ void batched_body(const BArgs& a, const BOrder& o, int64_t lb, float* dl) {
    typedef f32x4 vec_t;
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int n = o.nunit;
    const int xcd = (int)(lb & 7);
    const int64_t kb = lb >> 3;
    const int pg = (int)(kb % o.ngroups);
    const int64_t stream = (kb / o.ngroups) * 8 + xcd;
    const int p_lo = pg * o.ppg;
    const int np = min(o.ppg, o.panels_total - p_lo);

    // stage this group's operator panels (rows (m, i), columns j)
    const int total_slots = np * 16 * KP;
    for (int idx = threadIdx.x; idx < total_slots; idx += blockDim.x) {
        const int j = idx % KP;
        const int rr = idx / KP;
        const int panel = p_lo + rr / 16;
        const int m = panel / o.mblk;
        const int i = (panel % o.mblk) * 16 + (rr % 16);
        dl[rr * LD + j] = (i < n && j < n) ? o.D[((int64_t)m * n + i) * n + j] : 0.0f;
    }
    __syncthreads();

    const int64_t tile_elems = (int64_t)a.waves * 16 * CB;
    for (int64_t tile = stream; tile < o.ntiles; tile += o.nstreams) {
        const int64_t k0 = tile * tile_elems + (int64_t)wave * 16 * CB;  // position in the id list
        if (k0 >= o.count) continue;
        // lane (c, g) reads nodes g*KQ .. g*KQ+KQ-1 of element column c as
        // 16-byte loads from wherever the row starts
        int64_t base[CB];
        bool ok[CB];
        float bv[CB][KQ];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const int64_t k = k0 + q * 16 + c;
            ok[q] = k < o.count;
            base[q] = ok[q] ? a.off[a.perm[o.ids + k]] : 0;
#pragma unroll
            for (int t = 0; t < KQ; t += 4) {
                const f32x4 v = load4(a.u + base[q] + g * KQ + t, ok[q], n - g * KQ - t);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) bv[q][t + s4] = v[s4];
            }
        }
        for (int pp = 0; pp < np; ++pp) {
            f32x4 acc[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
            const float* arow = dl + (pp * 16 + c) * LD + g * KQ;
#pragma unroll
            for (int t = 0; t < KQ; t += 4) {
                const vec_t av = *reinterpret_cast<const vec_t*>(arow + t);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                    for (int q = 0; q < CB; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s4], bv[q][t + s4], acc[q], 0, 0, 0);
            }
            // lane holds output nodes i .. i+3 of element column c
            const int panel = p_lo + pp;
            const int m = panel / o.mblk;
            const int i = (panel % o.mblk) * 16 + 4 * g;
#pragma unroll
            for (int q = 0; q < CB; ++q)
                if (ok[q] && i < n) store4(a.out + (int64_t)m * a.total + base[q] + i, acc[q], n - i);
        }
    }
}

constexpr int GBM = 128, GBN = 128, GBK = 16, GLD = GBK + 4;
constexpr int kGemmVariant = 20, kValu8Variant = 21;
constexpr size_t kGemmLds = (size_t)2 * (GBM + GBN) * GLD * 4;
constexpr int kGemmMinNunit = 343;

// One GEMM tile: element block eb (GBN elements of the order's id list) x
// operator row block rb (GBM stacked rows), the contraction double-buffered
// through LDS in chunks of GBK nodes.
__device__ void gemm_tile(const BArgs& a, const BOrder& o, int64_t eb, int rb, float* sm) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const int n = o.nunit;
    const int R = a.nmat * n;  // stacked operator rows
    const int nk = (n + GBK - 1) / GBK;
    float* As = sm;                    // [2][GBM][GLD]
    float* Bs = sm + 2 * GBM * GLD;    // [2][GBN][GLD]
    const int64_t e0 = eb * GBN;
    const int r0 = rb * GBM;
    // staging coordinates: A row ar, columns ah .. ah+7; B elements be and
    // be+64, nodes bq .. bq+3
    const int ar = tid >> 1, ah = (tid & 1) * 8;
    const int be = tid >> 2, bq = (tid & 3) * 4;
    const bool a_ok = r0 + ar < R;
    const float* arow = o.D + (int64_t)(a_ok ? r0 + ar : 0) * n;
    bool b_ok[2];
    const float* brow[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t kb_ = e0 + be + 64 * h;
        b_ok[h] = kb_ < o.count;
        brow[h] = a.u + (b_ok[h] ? a.off[a.perm[o.ids + kb_]] : 0);
    }
    float ra[8], rbv[2][4];
    auto load = [&](int kc) {
        const int k0 = kc * GBK;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = k0 + ah + 4 * h;
            const f32x4 v = load4(arow + j, a_ok, n - j);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) ra[4 * h + q4] = v[q4];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f32x4 v = load4(brow[h] + k0 + bq, b_ok[h], n - k0 - bq);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) rbv[h][q4] = v[q4];
        }
    };
    auto store = [&](int buf) {
        float* ad = As + (buf * GBM + ar) * GLD + ah;
        *reinterpret_cast<f32x4*>(ad) = f32x4{ra[0], ra[1], ra[2], ra[3]};
        *reinterpret_cast<f32x4*>(ad + 4) = f32x4{ra[4], ra[5], ra[6], ra[7]};
#pragma unroll
        for (int h = 0; h < 2; ++h)
            *reinterpret_cast<f32x4*>(Bs + (buf * GBN + be + 64 * h) * GLD + bq) =
                f32x4{rbv[h][0], rbv[h][1], rbv[h][2], rbv[h][3]};
    };
    load(0);
    store(0);
    __syncthreads();
    f32x4 acc[4][4];
#pragma unroll
    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) load(kc + 1);
        f32x4 av[4], bv[4];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
            av[tm] = *reinterpret_cast<const f32x4*>(As + (buf * GBM + wm * 64 + tm * 16 + c) * GLD + 4 * g);
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
            bv[tn] = *reinterpret_cast<const f32x4*>(Bs + (buf * GBN + wn * 64 + tn * 16 + c) * GLD + 4 * g);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int tn = 0; tn < 4; ++tn)
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[tm][s4], bv[tn][s4], acc[tm][tn], 0,
                                                                       0, 0);
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    // lane holds stacked rows r0 + wm*64 + tm*16 + 4g + r of element column
    // wn*64 + tn*16 + c
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        const int64_t kpos = e0 + wn * 64 + tn * 16 + c;
        if (kpos >= o.count) continue;
        const int64_t eoff = a.off[a.perm[o.ids + kpos]];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
            const int row = r0 + wm * 64 + tm * 16 + 4 * g;
            if (row >= R) continue;
            const int m = row / n;
            const int i = row - m * n;
            if (i + 4 <= n) {
                // four nodes of one operator slab: one 16-byte store (the
                // stacked rows past R are zero padding: i + 4 <= n keeps them out)
                store4(a.out + (int64_t)m * a.total + eoff + i, acc[tm][tn], 4);
            } else {
                // the four rows cross into the next slab (or past R)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = row + r;
                    if (rr >= R) break;
                    const int mr = rr / n;
                    a.out[(int64_t)mr * a.total + eoff + (rr - mr * n)] = acc[tm][tn][r];
                }
            }
        }
    }
}

// Tiles of XCD pool x for a GEMM order: its element blocks eb = x (mod 8),
// each with all RB operator row blocks.
__device__ inline int64_t pool_tiles(const BOrder& o, int nmat, int x, int& RB) {
    RB = (nmat * o.nunit + GBM - 1) / GBM;
    const int64_t EB = (o.count + GBN - 1) / GBN;
    return EB > x ? ((EB - x + 7) / 8) * RB : 0;
}

// The GEMM orders' tiles form one pool per XCD (highest order first).  Every
// work-group drains its own XCD's pool, then the others', claiming one tile
// at a time with an atomic cursor; the work-groups whose static share ran out
// early thereby take over the remaining GEMM work, and the split needs no
// exact cost estimate.  The last work-group to finish resets the cursors for
// the next launch.
__device__ void gemm_pool(const BArgs& a, float* sm) {
    __shared__ int64_t claim;
    const int x0 = (int)(blockIdx.x & 7);
    for (int xi = 0; xi < 8; ++xi) {
        const int x = (x0 + xi) & 7;
        int64_t total = 0;
        for (int p = 7; p >= 1; --p) {
            const BOrder& o = a.ord[p];
            if (o.variant != kGemmVariant || o.count == 0) continue;
            int RB;
            total += pool_tiles(o, a.nmat, x, RB);
        }
        while (true) {
            // another XCD's drained pool is seen by a plain load, without
            // one more atomic on its cursor
            if (threadIdx.x == 0) {
                const int seen =
                    xi == 0 ? 0 : __hip_atomic_load(&a.ctr[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                claim = seen >= total ? total : atomicAdd(&a.ctr[x], 1);
            }
            __syncthreads();
            int64_t t = claim;
            __syncthreads();
            if (t >= total) break;
            for (int p = 7; p >= 1; --p) {
                const BOrder& o = a.ord[p];
                if (o.variant != kGemmVariant || o.count == 0) continue;
                int RB;
                const int64_t nt = pool_tiles(o, a.nmat, x, RB);
                if (t < nt) {
                    gemm_tile(a, o, x + 8 * (t / RB), (int)(t % RB), sm);
                    break;
                }
                t -= nt;
            }
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.ctr[8], 1) == (int)gridDim.x - 1) {
            for (int x = 0; x < 9; ++x) atomicExch(&a.ctr[x], 0);
            __threadfence();
        }
    }
}

// Order 1 (nunit 8): the operator stack is tiny (3 x 8 x 8) and the work
// per element a few hundred flops, so the order is bound by moving element
// data.  One thread takes one element:
// it reads the element's row with 16-byte loads, applies the operators with
// the node loops fully unrolled (operator entries are wave-uniform loads),
// and writes each output row with 16-byte stores.  A wave keeps 64 element
// rows in flight.
template <int N>
__device__ void valu_body(const BArgs& a, const BOrder& o, int64_t lb) {
    constexpr int NV = (N + 3) / 4;
    const float* __restrict__ D = o.D;
    for (int64_t blk = lb; blk * 256 < o.count; blk += o.nstreams) {
        const int64_t k = blk * 256 + threadIdx.x;
        if (k >= o.count) continue;
        const int64_t eoff = a.off[a.perm[o.ids + k]];
        float x[4 * NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const f32x4 t = load4(a.u + eoff + 4 * v, true, N - 4 * v);
#pragma unroll
            for (int q = 0; q < 4; ++q) x[4 * v + q] = t[q];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float* dst = a.out + (int64_t)m * a.total + eoff;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 4 * v + q;
                    if (i < N) {
                        float acc = 0.0f;
#pragma unroll
                        for (int j = 0; j < N; ++j) acc = __builtin_fmaf(D[(m * N + i) * N + j], x[j], acc);
                        y[q] = acc;
                    }
                }
                store4(dst + 4 * v, y, N - 4 * v);
            }
        }
    }
}

// kernel bodies instantiated: (order, column blocks per wave)
#define DG_BATCHED_VARIANTS(X) \
    X(0, 4, 1) X(1, 4, 2) X(2, 8, 1) X(3, 8, 2) X(4, 16, 1) X(5, 16, 2) X(6, 32, 1) X(7, 32, 2) \
    X(8, 56, 1)

__global__ void __launch_bounds__(256) dg_batched_kernel(BArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float* dl = reinterpret_cast<float*>(smem);
    int p = 1;
    while (p < 7 && (int64_t)blockIdx.x >= a.blk_lo[p + 1]) ++p;
    const BOrder& o = a.ord[p];
    const int64_t lb = (int64_t)blockIdx.x - a.blk_lo[p];
    switch (o.variant) {
#define X(V, KQ, CB)                          \
    case V:                                   \
        batched_body<KQ, CB>(a, o, lb, dl);   \
        break;
        DG_BATCHED_VARIANTS(X)
#undef X
        case kValu8Variant:
            valu_body<8>(a, o, lb);
            break;
        default:  // GEMM orders: all their tiles come from the pool
            break;
    }
    if (a.pool) {
        __syncthreads();  // the static part's LDS use ends before the pool's begins
        gemm_pool(a, dl);
    }
}

int variant_of(int kq, int cb) {
#define X(V, KQ, CB) \
    if (kq == KQ && cb == CB) return V;
    DG_BATCHED_VARIANTS(X)
#undef X
    return -1;
}

}  // namespace

// ------------------------------------------------------------------ plan

struct PlanOrder {
    int present = 0;
    int64_t count = 0;
    dg_tile tile = {};
    double predicted_s = 0;  // standalone full-GPU prediction of this order's work
    int64_t blocks = 0;
    BOrder b = {};
};

struct BatchPlan {
    int64_t nelem = 0, total = 0;
    int nmat = 3;
    int waves = 4;
    size_t smem = 0;
    int64_t grid = 0;
    int64_t* d_perm = nullptr;
    int64_t* d_off = nullptr;
    int* d_ctr = nullptr;  // GEMM tile pool cursors (zero between launches)
    PlanOrder ord[8];
    double predicted_s = 0;
};

constexpr size_t kBatchLds = 80 * 1024;  // per work-group: two work-groups per CU

static double eval_model(const int64_t* f, const double* cost, const int32_t* group, double edge) {
    double c[3] = {0, 0, 0};
    for (int k = 0; k < PF_COUNT; ++k) c[group ? group[k] : 0] += cost[k] * (double)f[k];
    if (!group) return c[0];
    const double d = c[1] - c[2];
    return c[0] + c[2] + d * 0.5 * (std::tanh(edge * d) + 1.0);
}

// Work-groups an order's share would have alone on the GPU with the
// planner's rule (two work-groups per CU, a whole number of streams per
// operator group, no more streams than tiles): the share its candidates are
// priced at.
static int64_t standalone_share(const dg_tile& t, int64_t count, int n, int nmat, int num_cu) {
    int64_t unit = 8, ntiles;
    if (t.flags & DG_TILE_BATCH_GEMM) {
        ntiles = ceil_div((int64_t)nmat * n, (int64_t)GBM) * ceil_div(count, (int64_t)GBN);
    } else if (t.elems_per_wave == 256) {
        ntiles = ceil_div(count, (int64_t)256);
    } else {
        const int64_t panels = (int64_t)nmat * ceil_div(n, 16);
        unit = 8 * ceil_div(panels, (int64_t)std::max(1, t.d_panels));
        ntiles = ceil_div(count, (int64_t)t.elems_per_wave * 4);
    }
    int64_t blocks = std::max<int64_t>(unit, (2 * (int64_t)num_cu / unit) * unit);
    return std::min<int64_t>(blocks, unit * std::max<int64_t>(1, ceil_div(ntiles, 8)));
}

dg_status batch_plan_create(int64_t nelem, const int8_t* order, int nmat, const dg_tile* tiles,
                            const double* cost, const int32_t* group, double edge, BatchPlan** out) {
    if (nelem < 0 || !order || !out) return fail(DG_EINVAL, "dgdiff_plan_create: bad arguments");
    if (nmat != 3) return fail(DG_EUNSUPPORTED, "dgdiff_plan_create: nmat must be 3");
    DeviceInfo dev;
    dg_status st = current_device(&dev);
    if (st != DG_OK) return st;
    auto* P = new BatchPlan();
    P->nelem = nelem;
    P->nmat = nmat;
    // counting sort by order (stable: ids ascending within an order)
    std::vector<int64_t> off(nelem + 1, 0), perm(std::max<int64_t>(nelem, 1));
    int64_t cnt[9] = {0};
    for (int64_t e = 0; e < nelem; ++e) {
        const int p = order[e];
        if (p < 1 || p > 7) {
            delete P;
            return fail(DG_EINVAL, "dgdiff_plan_create: orders must be in 1..7");
        }
        ++cnt[p];
        const int64_t ne = (int64_t)(p + 1) * (p + 1) * (p + 1);
        off[e + 1] = off[e] + ne;
    }
    P->total = off[nelem];
    int64_t start[9] = {0};
    for (int p = 2; p <= 8; ++p) start[p] = start[p - 1] + cnt[p - 1];
    {
        int64_t pos[9];
        std::copy(start, start + 9, pos);
        for (int64_t e = 0; e < nelem; ++e) perm[pos[order[e]]++] = e;
    }
    // per-order launch shape
    for (int p = 1; p <= 7; ++p) {
        PlanOrder& po = P->ord[p];
        po.count = cnt[p];
        po.present = cnt[p] > 0;
        if (!po.present) continue;
        const int n = (p + 1) * (p + 1) * (p + 1);
        const int kq = kern::kq_for(n);
        const int mblk = (int)ceil_div(n, 16);
        const int panels = nmat * mblk;
        const size_t panel_bytes = (size_t)16 * (4 * kq + 4) * 4;
        // operator panels that fit the per-group LDS budget
        auto max_ppg_for = [&](int) { return (int)std::min<size_t>(panels, kBatchLds / panel_bytes); };
        // kernel body of this order: one element per thread (order 1), GEMM
        // tiling (orders 6, 7, or when asked for) or resident operator panels
        const bool force_gemm = tiles && (tiles[p].flags & DG_TILE_BATCH_GEMM);
        const bool force_panels = tiles && tiles[p].elems_per_wave && !force_gemm;
        const bool use_valu = n == 8 && !force_gemm && !force_panels;
        const bool use_gemm = !use_valu && (n >= kGemmMinNunit || force_gemm);
        std::vector<dg_tile> cands;
        if (use_valu) {
            cands.push_back(dg_tile{256, 4, 2, 0, 0});
        } else if (use_gemm) {
            cands.push_back(dg_tile{GBN, 4, 1, GBM / 16, DG_TILE_BATCH_GEMM});
        } else if (tiles && tiles[p].elems_per_wave) {
            dg_tile t = tiles[p];
            if (t.elems_per_wave != 16 && t.elems_per_wave != 32) {
                delete P;
                return fail(DG_EINVAL, "dgdiff_plan_create: tile elems_per_wave must be 16 or 32");
            }
            // operator panels per work-group: as many as the per-group LDS allows
            // unless given (balanced over the groups either way)
            const int max_ppg = max_ppg_for(t.elems_per_wave / 16);
            if (max_ppg < 1) {
                delete P;
                return fail(DG_EUNSUPPORTED, "dgdiff_plan_create: tile does not fit the LDS");
            }
            const int want = t.d_panels > 0 ? std::min(t.d_panels, max_ppg) : max_ppg;
            t.d_panels = (int)ceil_div(panels, ceil_div(panels, want));
            t.waves = 4;
            if (t.groups_per_cu <= 0) t.groups_per_cu = 2;
            t.flags = 0;
            cands.push_back(t);
        } else {
            // operator-group counts reachable within the LDS budget (a few of
            // the smallest), each with balanced groups
            for (int cb : {1, 2}) {
                if (variant_of(kq, cb) < 0) continue;
                std::set<int> ngs;
                for (int ppg = max_ppg_for(cb); ppg >= 1 && ngs.size() < 5; --ppg)
                    ngs.insert((int)ceil_div(panels, ppg));
                for (int ng : ngs) {
                    const int ppg = (int)ceil_div(panels, ng);
                    dg_tile t = {};
                    t.elems_per_wave = 16 * cb;
                    t.waves = 4;
                    t.d_panels = ppg;
                    t.groups_per_cu = 2;
                    cands.push_back(t);
                }
            }
        }
        // Each candidate is priced as the body that runs it, standalone on the
        // whole GPU: the share it would get alone (two work-groups per CU, no
        // more streams than tiles).  A fitted model may predict a negative
        // time for a tiny launch, so the first scored candidate is taken as
        // found whatever its sign.
        double best = 0;
        bool found = false;
        for (const dg_tile& t : cands) {
            double pred = 0;
            if (cost) {
                perf_kernel_desc d = {};
                d.kernel = DG_K_BATCHED;
                d.dtype = DG_F32;
                d.n0 = po.count;
                d.nunit = n;
                d.nmat = nmat;
                d.tile = t;
                d.num_cu = dev.num_cu;
                d.workgroups = standalone_share(t, po.count, n, nmat, dev.num_cu);
                int64_t f[PF_COUNT];
                if (perf_features_count(&d, f) != DG_OK) continue;
                if (t.flags & DG_TILE_BATCH_GEMM) {
                    perf_kernel_desc q = {};
                    q.kernel = DG_K_BATCHED_POOL;
                    q.dtype = DG_F32;
                    q.n0 = d.workgroups;
                    int64_t fq[PF_COUNT];
                    if (perf_features_count(&q, fq) != DG_OK) continue;
                    for (int k = 0; k < PF_COUNT; ++k) f[k] += fq[k];
                }
                pred = eval_model(f, cost, group, edge);
            } else {
                // no model: the smallest number of operator groups, one column block
                pred = t.d_panels > 0 ? (double)ceil_div(panels, t.d_panels) + (t.elems_per_wave == 16 ? 0 : 0.5)
                                      : 0.0;
            }
            if (!found || pred < best) {
                best = pred;
                po.tile = t;
                found = true;
            }
        }
        if (!found) {
            delete P;
            return fail(DG_EUNSUPPORTED, "dgdiff_plan_create: no launch shape for an order");
        }
        po.predicted_s = cost ? best : 0.0;
        const int cb = po.tile.elems_per_wave / 16;
        BOrder& b = po.b;
        b.count = po.count;
        b.ids = start[p];
        b.nunit = n;
        b.mblk = mblk;
        b.panels_total = panels;
        size_t lds;
        if (use_valu) {
            // order 1: one element per thread
            b.ppg = 1;
            b.ngroups = 1;
            b.cb = 1;
            b.variant = kValu8Variant;
            b.ntiles = ceil_div(po.count, (int64_t)256);
            lds = 0;
        } else if (use_gemm) {
            // large orders: GEMM tiling (GBM operator rows x GBN elements)
            b.ppg = 1;
            b.ngroups = 1;
            b.cb = 1;
            b.variant = kGemmVariant;
            b.ntiles = ceil_div((int64_t)nmat * n, (int64_t)GBM) * ceil_div(po.count, (int64_t)GBN);
            lds = kGemmLds;
        } else {
            b.ppg = std::max(1, std::min(po.tile.d_panels, panels));
            b.ngroups = (int)ceil_div(panels, b.ppg);
            b.cb = cb;
            b.variant = variant_of(kq, cb);
            b.ntiles = ceil_div(po.count, (int64_t)16 * cb * 4);
            lds = (size_t)b.ppg * panel_bytes;
        }
        if (b.variant < 0 || lds > 160 * 1024) {
            delete P;
            return fail(DG_EUNSUPPORTED, "dgdiff_plan_create: launch shape not available");
        }
        P->smem = std::max(P->smem, lds);
    }
    // work-group split: resident capacity shared in proportion to predicted time
    int per_cu = 1;
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(dg_batched_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P->smem));
    DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(dg_batched_kernel), 64 * P->waves, P->smem));
    per_cu = std::max(per_cu, 1);
    const double capacity = (double)per_cu * dev.num_cu;
    // an order's weight: its predicted time (floored, since a fitted model
    // can go negative outside the sizes it was calibrated on), else a
    // roofline estimate at the rates the bodies sustain on this GPU, about
    // 80 TFLOP/s and 2.5 TB/s (flops alone would starve the memory-bound low
    // orders)
    // Orders on the GEMM body draw their tiles from the pool, which every
    // work-group joins once its own share is done, so the split only has to
    // keep the other orders from finishing last: their shares are sized 1.25x
    // their estimate (the excess flows into the pool).
    auto weight = [&](int p) {
        const PlanOrder& po = P->ord[p];
        const double nn = std::pow((double)(p + 1), 3.0);
        const double w = cost ? std::max(po.predicted_s, 1e-7)
                              : std::max(6.0 * nn * nn * po.count / 80e12, 16.0 * nn * po.count / 2.5e12);
        return po.b.variant == kGemmVariant ? w : 1.25 * w;
    };
    double wsum = 0;
    for (int p = 1; p <= 7; ++p)
        if (P->ord[p].present) wsum += weight(p);
    int64_t lo = 0;
    double pred_total = 0;
    for (int p = 1; p <= 7; ++p) {
        PlanOrder& po = P->ord[p];
        P->ord[p].b.D = nullptr;
        if (!po.present) {
            po.blocks = 0;
            continue;
        }
        const double w = weight(p);
        const int64_t unit = 8 * po.b.ngroups;
        int64_t blocks = (int64_t)std::llround(capacity * w / wsum / unit) * unit;
        blocks = std::max<int64_t>(unit, blocks);
        // no more tile streams than tiles
        blocks = std::min<int64_t>(blocks, unit * std::max<int64_t>(1, ceil_div(po.b.ntiles, 8)));
        po.blocks = blocks;
        po.b.nstreams = (int)(8 * (blocks / unit));
        pred_total += po.predicted_s;
        lo += blocks;
    }
    P->grid = lo;
    P->predicted_s = pred_total;
    // device copies of the id list and the offsets
    DG_HIP_CHECK(hipMalloc(&P->d_ctr, sizeof(int) * 9));
    DG_HIP_CHECK(hipMemset(P->d_ctr, 0, sizeof(int) * 9));
    if (nelem > 0) {
        DG_HIP_CHECK(hipMalloc(&P->d_perm, sizeof(int64_t) * nelem));
        DG_HIP_CHECK(hipMalloc(&P->d_off, sizeof(int64_t) * (nelem + 1)));
        DG_HIP_CHECK(hipMemcpy(P->d_perm, perm.data(), sizeof(int64_t) * nelem, hipMemcpyHostToDevice));
        DG_HIP_CHECK(hipMemcpy(P->d_off, off.data(), sizeof(int64_t) * (nelem + 1),
                               hipMemcpyHostToDevice));
    }
    *out = P;
    return DG_OK;
}

void batch_plan_destroy(BatchPlan* P) {
    if (!P) return;
    if (P->d_perm) (void)hipFree(P->d_perm);
    if (P->d_off) (void)hipFree(P->d_off);
    if (P->d_ctr) (void)hipFree(P->d_ctr);
    delete P;
}

dg_status batch_apply(const BatchPlan* P, const void* const* D_sets, const void* u, void* out,
                      hipStream_t s) {
    if (P->nelem == 0) return DG_OK;
    BArgs a = {};
    a.u = static_cast<const float*>(u);
    a.out = static_cast<float*>(out);
    a.perm = P->d_perm;
    a.off = P->d_off;
    a.total = P->total;
    a.nmat = P->nmat;
    a.waves = P->waves;
    a.ctr = P->d_ctr;
    a.pool = 0;
    for (int p = 1; p <= 7; ++p)
        if (P->ord[p].present && P->ord[p].b.variant == kGemmVariant) a.pool = 1;
    int64_t lo = 0;
    for (int p = 1; p <= 7; ++p) {
        a.blk_lo[p] = lo;
        a.ord[p] = P->ord[p].b;
        if (P->ord[p].present) {
            if (!D_sets[p]) return fail(DG_EINVAL, "dgdiff_apply_batched: missing operator set");
            a.ord[p].D = static_cast<const float*>(D_sets[p]);
        }
        lo += P->ord[p].blocks;
    }
    a.blk_lo[8] = lo;
    a.blk_lo[0] = 0;
    DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(dg_batched_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)P->smem));
    hipLaunchKernelGGL(dg_batched_kernel, dim3((unsigned)P->grid), dim3(64 * P->waves), P->smem, s, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg

using namespace dg;

struct dg_plan {
    BatchPlan* p;
};

extern "C" {

dg_status dgdiff_plan_create(int64_t nelem, const int8_t* order, int32_t nmat, const dg_tile* tiles,
                             const double* model_cost, const int32_t* model_group, double model_edge,
                             dg_plan** out) {
    set_error("");
    if (!out) return fail(DG_EINVAL, "dgdiff_plan_create: out is NULL");
    *out = nullptr;
    BatchPlan* P = nullptr;
    dg_status st = batch_plan_create(nelem, order, nmat, tiles, model_cost, model_group, model_edge, &P);
    if (st != DG_OK) return st;
    *out = new dg_plan{P};
    return DG_OK;
}

int64_t dgdiff_plan_total_nodes(const dg_plan* plan) { return plan ? plan->p->total : -1; }

dg_status dgdiff_plan_info(const dg_plan* plan, int32_t p, dg_tile* tile, int64_t* count,
                           int64_t* workgroups, double* predicted_s) {
    set_error("");
    if (!plan || p < 1 || p > 7) return fail(DG_EINVAL, "dgdiff_plan_info: bad arguments");
    const PlanOrder& po = plan->p->ord[p];
    if (tile) *tile = po.tile;
    if (count) *count = po.count;
    if (workgroups) *workgroups = po.blocks;
    if (predicted_s) *predicted_s = po.predicted_s;
    return DG_OK;
}

dg_status dgdiff_apply_batched(const dg_plan* plan, const void* const* D_sets, const void* u_packed,
                               void* out_packed, dg_stream_t stream) {
    set_error("");
    if (!plan || !D_sets) return fail(DG_EINVAL, "dgdiff_apply_batched: NULL argument");
    if (plan->p->nelem > 0 && (!u_packed || !out_packed))
        return fail(DG_EINVAL, "dgdiff_apply_batched: NULL array");
    const size_t nu = (size_t)plan->p->total * 4, no = nu * plan->p->nmat;
    if (overlaps(out_packed, no, u_packed, nu))
        return fail(DG_EINVAL, "dgdiff_apply_batched: out overlaps u");
    return batch_apply(plan->p, D_sets, u_packed, out_packed, reinterpret_cast<hipStream_t>(stream));
}

void dgdiff_plan_destroy(dg_plan* plan) {
    if (!plan) return;
    batch_plan_destroy(plan->p);
    delete plan;
}

}  // extern "C"
