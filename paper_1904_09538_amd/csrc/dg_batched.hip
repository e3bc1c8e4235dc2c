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
// element ids.  Rows are not 16-byte aligned in the packed layout, so element
// data are read and outputs written with masked scalar accesses.
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
};

namespace {

using namespace kern;

// Panels a work-group may hold for a given KQ (the 80 KB per-group budget).
constexpr int max_panels(int kq) {
    const int pb = 16 * (4 * kq + 4) * 4;
    const int m = (80 * 1024) / pb;
    return m < 1 ? 1 : m;
}

template <int KQ, int CB>
__device__ void batched_body(const BArgs& a, const BOrder& o, int64_t lb, float* dl) {
    typedef f32x4 vec_t;
    constexpr int KP = 4 * KQ;
    constexpr int LD = KP + 4;
    // Large orders walk the contraction in chunks of 32 nodes per lane group
    // and keep the accumulators of all their resident panels (at most
    // max_panels) live across chunks: 32 element values per column block in
    // registers instead of KQ.
    constexpr int KC = KQ <= 32 ? KQ : 32;
    constexpr int NCH = (KQ + KC - 1) / KC;
    constexpr int MAXP = NCH == 1 ? 1 : max_panels(KQ);
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
        int64_t eid[CB], base[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const int64_t k = k0 + q * 16 + c;
            eid[q] = k < o.count ? a.perm[o.ids + k] : -1;
            base[q] = eid[q] >= 0 ? a.off[eid[q]] : 0;
        }
        for (int pp0 = 0; pp0 < np; pp0 += MAXP) {
            f32x4 acc[MAXP][CB];
#pragma unroll
            for (int pq = 0; pq < MAXP; ++pq)
#pragma unroll
                for (int q = 0; q < CB; ++q) acc[pq][q] = f32x4{0.f, 0.f, 0.f, 0.f};
            // NCH == 1: one chunk per panel, panels one after another
            for (int pq1 = 0; pq1 < (NCH == 1 ? min(MAXP, np - pp0) : 1); ++pq1) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int k_lo = ch * KC;
                    float b[CB][KC];
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        const float* row = a.u + base[q] + g * KQ + k_lo;
#pragma unroll
                        for (int t = 0; t < KC; ++t)
                            b[q][t] = (eid[q] >= 0 && k_lo + t < KQ && g * KQ + k_lo + t < n) ? row[t]
                                                                                               : 0.0f;
                    }
#pragma unroll
                    for (int pq = 0; pq < MAXP; ++pq) {
                        const int pp = pp0 + (NCH == 1 ? pq1 : pq);
                        if ((NCH == 1 && pq > 0) || pp >= np) continue;
                        const float* arow = dl + (pp * 16 + c) * LD + g * KQ + k_lo;
#pragma unroll
                        for (int t = 0; t < KC; t += 4) {
                            if (k_lo + t >= KQ) continue;
                            const vec_t av = *reinterpret_cast<const vec_t*>(arow + t);
#pragma unroll
                            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                                for (int q = 0; q < CB; ++q)
                                    acc[pq][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        av[s4], b[q][t + s4], acc[pq][q], 0, 0, 0);
                        }
                    }
                }
                if constexpr (NCH == 1) {
                    const int pp = pp0 + pq1;
                    const int panel = p_lo + pp;
                    const int m = panel / o.mblk;
                    const int i = (panel % o.mblk) * 16 + 4 * g;
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        if (eid[q] < 0) continue;
                        float* dst = a.out + (int64_t)m * a.total + base[q] + i;
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (i + r < n) dst[r] = acc[0][q][r];
                        acc[0][q] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
                }
            }
            if constexpr (NCH > 1) {
#pragma unroll
                for (int pq = 0; pq < MAXP; ++pq) {
                    const int pp = pp0 + pq;
                    if (pp >= np) continue;
                    const int panel = p_lo + pp;
                    const int m = panel / o.mblk;
                    const int i = (panel % o.mblk) * 16 + 4 * g;  // four consecutive output nodes
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        if (eid[q] < 0) continue;
                        float* dst = a.out + (int64_t)m * a.total + base[q] + i;
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (i + r < n) dst[r] = acc[pq][q][r];
                    }
                }
            }
        }
    }
}

// kernel bodies instantiated: (order, column blocks per wave)
#define DG_BATCHED_VARIANTS(X) \
    X(0, 4, 1) X(1, 4, 2) X(2, 8, 1) X(3, 8, 2) X(4, 16, 1) X(5, 16, 2) X(6, 32, 1) X(7, 32, 2) \
    X(8, 56, 1) X(10, 88, 1) X(11, 128, 1)

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
        default:
            break;
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
        const int max_ppg = std::max<int>(1, (int)std::min<size_t>(panels, kBatchLds / panel_bytes));
        std::vector<dg_tile> cands;
        if (tiles && tiles[p].elems_per_wave) {
            dg_tile t = tiles[p];
            if (t.elems_per_wave != 16 && t.elems_per_wave != 32) {
                delete P;
                return fail(DG_EINVAL, "dgdiff_plan_create: tile elems_per_wave must be 16 or 32");
            }
            // operator panels per work-group: as many as the per-group LDS allows
            // unless given (balanced over the groups either way)
            const int want = t.d_panels > 0 ? std::min(t.d_panels, max_ppg) : max_ppg;
            t.d_panels = (int)ceil_div(panels, ceil_div(panels, want));
            t.waves = 4;
            if (t.groups_per_cu <= 0) t.groups_per_cu = 2;
            cands.push_back(t);
        } else {
            // operator-group counts reachable within the LDS budget (a few of
            // the smallest), each with balanced groups
            std::set<int> ngs;
            for (int ppg = max_ppg; ppg >= 1 && ngs.size() < 5; --ppg)
                ngs.insert((int)ceil_div(panels, ppg));
            for (int cb : {1, 2}) {
                if (variant_of(kq, cb) < 0) continue;
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
        // a fitted model may predict a negative time for a tiny launch, so the
        // first scored candidate is taken as found whatever its sign
        double best = 0;
        bool found = false;
        for (const dg_tile& t : cands) {
            double pred = 0;
            if (cost) {
                perf_kernel_desc d = {};
                d.kernel = DG_K_DGDIFF;
                d.dtype = DG_F32;
                d.n0 = po.count;
                d.nunit = n;
                d.nmat = nmat;
                d.tile = t;
                d.num_cu = dev.num_cu;
                int64_t f[PF_COUNT];
                if (perf_features_count(&d, f) != DG_OK) continue;
                pred = eval_model(f, cost, group, edge);
            } else {
                // no model: the smallest number of operator groups, one column block
                pred = (double)ceil_div(panels, t.d_panels) + (t.elems_per_wave == 16 ? 0 : 0.5);
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
        b.ppg = std::max(1, std::min(po.tile.d_panels, panels));
        b.ngroups = (int)ceil_div(panels, b.ppg);
        b.cb = cb;
        b.variant = variant_of(kq, cb);
        b.ntiles = ceil_div(po.count, (int64_t)16 * cb * 4);
        if (b.variant < 0 || (size_t)b.ppg * panel_bytes > 160 * 1024) {
            delete P;
            return fail(DG_EUNSUPPORTED, "dgdiff_plan_create: launch shape not available");
        }
        P->smem = std::max(P->smem, (size_t)b.ppg * panel_bytes);
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
    // can go negative outside the sizes it was calibrated on), else its flops
    auto weight = [&](int p) {
        const PlanOrder& po = P->ord[p];
        return cost ? std::max(po.predicted_s, 1e-7)
                    : (double)po.count * std::pow((double)(p + 1), 6.0);
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
