// Closed-form operation counts of the library's kernels: the input features of
// the paper's black-box model (Sections "Gathering Kernel Statistics" and
// "Kernel Features").
//
// The paper counts, per statement, the integer points of the loop domain
// projected onto the statement's loops, times the operations per execution
// (its per-statement count formula), with a granularity per operation kind.
// Our kernels are hand-written, so each count is that sum worked out by hand
// for the kernel's documented schedule (the launch plan below is the one the
// launcher uses), including ragged tails.  Readings of the counting rules:
//   - global loads/stores: bytes moved by the lanes that execute them
//     (a 16-byte vector load of one lane counts 16);
//   - LDS: bytes moved by the lanes that execute the access (stores of the
//     operator staging, reads of MFMA operands, slab copies, wave shuffles);
//   - matrix cores: flops of the executed MFMA instructions (2*M*N*K each,
//     padding included) per data type;
//   - VALU flops: per lane that computes them;
//   - barriers: per work-item (the paper's rule), multiplied by work-groups;
//   - work-groups and kernel launches.
// Memory accesses are tagged by access pattern, as the paper does: DG element
// data on the 16-byte vector path vs. the unaligned-row paths, output rows
// stored as vectors vs. scalars, and loads of an element tile by the second
// and later operator groups (L2 re-reads, not HBM traffic).  The number of
// element tiles a wave processes (summed over operator groups) carries the
// fixed per-tile latency; the longest chain of loop iterations one work-group
// walks (its element tiles, k-chunks or strip rows) carries the latency of
// launches too small to fill the GPU.
// A brute-force enumerator of the same schedule in the test oracle must give
// identical int64 counts.
#include "dg_kernel.hpp"

namespace dg {

int stencil5_rows_per_strip(int64_t n);

namespace {

using kern::Plan;

dg_status count_dg_fp(const perf_kernel_desc* d, int64_t* c) {
    const size_t sz = d->dtype == DG_F64 ? 8 : 4;
    const int V = (int)(16 / sz);
    const int64_t E = d->n0;
    const int n = d->nunit, M = d->nmat;
    const int kq = kern::kq_for(n);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large");
    int cb;
    dg_status st = kern::forward_cb(sz, kq, n % V == 0, d->tile.elems_per_wave, &cb);
    if (st != DG_OK) return st;
    Plan P;
    st = kern::make_plan(sz, 1, M, E, n, kq, cb, d->tile.waves, d->tile.d_panels,
                         d->tile.groups_per_cu, d->num_cu, n % V == 0, &P);
    if (st != DG_OK) return st;
    const int64_t KP = 4 * kq;
    const int64_t nwt = ceil_div(E, (int64_t)16 * cb);  // wave-tiles that start before E
    c[PF_LAUNCH] = 1;
    c[PF_WORKGROUPS] = P.grid;
    c[PF_BARRIER_X_WG] = P.grid;  // one barrier after the operator staging
    c[PF_GLD_DG_D] = 8 * P.slots * (int64_t)M * n * n * (int64_t)sz;
    // element rows read per operator group: the pipelined loads take whole
    // wave-tiles (rows past the end clamp to the last element)
    const int64_t urows = kern::pipelined_loads(sz, n, kq, cb, n % 4 == 0, P) ? nwt * 16 * cb : E;
    c[P.vec_in ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] = urows * n * (int64_t)sz;
    c[PF_GLD_DG_U_L2] = (int64_t)(P.ngroups - 1) * urows * n * (int64_t)sz;
    // unaligned rows read through the wave slab are also written through it:
    // contiguous stores (plus one LDS write and read per output value)
    const bool stage_out = P.use_slab && n % 4 != 0;
    c[(n % 4 == 0 || stage_out) ? PF_GST_DG_OUT : PF_GST_DG_OUT_UNAL] = E * M * n * (int64_t)sz;
    c[PF_WAVE_TILES] = nwt * P.ngroups;
    c[PF_SERIAL_STEPS] = ceil_div(P.ntiles, 8 * P.slots);  // tiles of the busiest stream
    c[PF_LAT_STEPS] = c[PF_SERIAL_STEPS] * 64 / ((int64_t)d->tile.groups_per_cu * d->tile.waves);
    c[PF_LDS_BYTES] = 8 * P.slots * P.panels_total * 16 * KP * (int64_t)sz  // staging stores
                      + nwt * P.panels_total * 64 * kq * (int64_t)sz      // operand reads
                      + (P.use_slab ? (int64_t)P.ngroups * 2 * E * n * (int64_t)sz : 0)
                      + (stage_out ? 2 * E * M * n * (int64_t)sz : 0);
    c[sz == 8 ? PF_MFMA_F64 : PF_MFMA_F32] = nwt * P.panels_total * kq * (int64_t)cb * 2048;
    return DG_OK;
}

dg_status count_dg_lowp(const perf_kernel_desc* d, int64_t* c) {
    const int fmt = lp_format(d->dtype, &d->tile);
    LpPlan P;
    dg_status st = make_lp_plan(fmt, d->nmat, d->n0, d->nunit, &d->tile, d->tile.groups_per_cu,
                                d->num_cu, &P);
    if (st != DG_OK) return st;
    const int64_t E = d->n0;
    const int n = d->nunit, M = d->nmat;
    const int64_t eg = d->dtype == DG_BF16 ? 2 : 1;  // bytes per value in HBM
    const int64_t KP = 32 * P.ks;
    const int64_t nwt = ceil_div(E, (int64_t)16 * P.cb);
    c[PF_LAUNCH] = 1;
    c[PF_WORKGROUPS] = P.grid;
    c[PF_BARRIER_X_WG] = P.grid;
    c[PF_GLD_DG_D] = 8 * P.slots * (int64_t)M * n * n * eg;
    c[n % 8 == 0 ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] = E * n * eg;
    c[PF_GLD_DG_U_L2] = (int64_t)(P.ngroups - 1) * E * n * eg;
    c[n % 4 == 0 ? PF_GST_DG_OUT : PF_GST_DG_OUT_UNAL] = E * M * n * 4;
    c[PF_WAVE_TILES] = nwt * P.ngroups;
    c[PF_SERIAL_STEPS] = ceil_div(P.ntiles, 8 * P.slots);
    c[PF_LAT_STEPS] = c[PF_SERIAL_STEPS] * 64 / ((int64_t)d->tile.groups_per_cu * P.waves);
    c[PF_LDS_BYTES] = 8 * P.slots * P.panels_total * 16 * KP * P.lds_esz +
                      nwt * P.panels_total * P.ks * 64 * 8 * P.lds_esz;
    c[fmt == 1 ? PF_MFMA_FP8 : PF_MFMA_BF16] = nwt * P.panels_total * P.ks * (int64_t)P.cb * 16384;
    return DG_OK;
}

dg_status count_stencil(const perf_kernel_desc* d, int64_t* c) {
    const int64_t n = d->n0;
    const size_t sz = d->dtype == DG_F64 ? 8 : 4;
    c[PF_LAUNCH] = 1;
    // the fast path is taken for FP32 with n % 4 == 0 (leading dimensions
    // padded to multiples of 4, aligned arrays, as the harness allocates them)
    if (d->dtype == DG_F32 && n % 4 == 0) {
        const int64_t R = stencil5_rows_per_strip(n);
        const int64_t gx = ceil_div(n, 1024), gy = ceil_div(n, R);
        const int64_t A = n / 4;                               // active lanes per strip row
        const int64_t SH = A / 64 + (((A - 1) % 64) != 63 ? 1 : 0);  // lanes loading their halo
        const int64_t rows_loaded = n + 2 * gy;                // over all strips
        c[PF_WORKGROUPS] = gx * gy;
        c[PF_GLD_ST_U] = rows_loaded * (A * 16 + SH * 8);
        c[PF_GST_ST_RES] = n * A * 16;
        c[PF_LDS_BYTES] = rows_loaded * gx * 256 * 2 * 4;      // two shuffles per lane and row
        c[PF_VALU_F32] = n * gx * 256 * 20;                    // 4 outputs x 5 flops, every lane
        c[PF_SERIAL_STEPS] = std::min(R, n);                   // rows of one strip
    } else {
        c[PF_WORKGROUPS] = ceil_div(n, 64) * ceil_div(n, 4);
        c[PF_GLD_ST_U] = n * n * 5 * (int64_t)sz;
        c[PF_GST_ST_RES] = n * n * (int64_t)sz;
        c[sz == 8 ? PF_VALU_F64 : PF_VALU_F32] = n * n * 5;
        c[PF_SERIAL_STEPS] = 1;
    }
    return DG_OK;
}

dg_status count_matmul(const perf_kernel_desc* d, int64_t* c) {
    const int64_t n = d->n0;
    const int64_t grid = ceil_div(n, 128);
    const int64_t wg = grid * grid;
    const int64_t nk = ceil_div(n, 16);
    c[PF_LAUNCH] = 1;
    c[PF_WORKGROUPS] = wg;
    c[PF_BARRIER_X_WG] = wg * (1 + nk);
    c[PF_GLD_MM_AB] = 8 * n * n * grid;   // each a row / b column read once per block column / row
    c[PF_GST_MM_C] = 4 * n * n;
    c[PF_LDS_BYTES] = wg * nk * 256 * (64 + 128);  // chunk stores + operand reads
    c[PF_MFMA_F32] = wg * nk * 4 * 64 * 2048;
    // k-chunks walked by the busiest compute unit: the work-groups are dealt
    // evenly over num_cu units (one work-group's chain when num_cu is 0).
    // The tiles are MFMA-bound, so work-groups sharing a unit share its
    // matrix cores and the busiest unit's chain sets the time.
    c[PF_SERIAL_STEPS] = (d->num_cu > 0 ? ceil_div(wg, (int64_t)d->num_cu) : 1) * nk;
    return DG_OK;
}

const char* kNames[PF_COUNT] = {
    "launch", "workgroups", "barrier_x_wg", "gld_dg_u", "gld_dg_u_l2", "gld_dg_d", "gst_dg_out",
    "gld_st_u", "gst_st_res", "gld_mm_ab", "gst_mm_c", "lds_bytes", "mfma_f64", "mfma_f32",
    "mfma_bf16", "mfma_fp8", "valu_f32", "valu_f64", "gld_dg_u_unal", "gst_dg_out_unal",
    "wave_tiles", "serial_steps", "lat_steps"};

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" {

int32_t perf_feature_count(void) { return PF_COUNT; }

const char* perf_feature_name(int32_t k) { return (k >= 0 && k < PF_COUNT) ? kNames[k] : ""; }

dg_status perf_features_count(const perf_kernel_desc* d, int64_t* counts) {
    set_error("");
    if (!d || !counts) return fail(DG_EINVAL, "perf_features_count: NULL argument");
    for (int k = 0; k < PF_COUNT; ++k) counts[k] = 0;
    if (d->n0 < 0) return fail(DG_EINVAL, "perf_features_count: negative size");
    switch (d->kernel) {
        case DG_K_DGDIFF:
            if (d->nunit < 1 || d->nunit > 512 || d->nmat < 1 || d->nmat > 8)
                return fail(DG_EUNSUPPORTED, "perf_features_count: DG sizes");
            if (d->tile.waves < 1 || d->tile.waves > 8 || d->tile.elems_per_wave == 0 ||
                d->tile.groups_per_cu < 1 || d->tile.d_panels < 1 || d->num_cu < 1)
                return fail(DG_EINVAL, "perf_features_count: DG needs a resolved tile and num_cu");
            if (d->n0 == 0) return DG_OK;
            if (d->dtype == DG_F32 || d->dtype == DG_F64) return count_dg_fp(d, counts);
            if (d->dtype == DG_BF16 || d->dtype == DG_FP8E4M3) return count_dg_lowp(d, counts);
            return fail(DG_EUNSUPPORTED, "perf_features_count: DG dtype");
        case DG_K_STENCIL5:
            if (d->dtype != DG_F32 && d->dtype != DG_F64) return fail(DG_EUNSUPPORTED, "stencil dtype");
            if (d->n0 == 0) return DG_OK;
            return count_stencil(d, counts);
        case DG_K_MATMUL:
            if (d->dtype != DG_F32) return fail(DG_EUNSUPPORTED, "matmul dtype");
            if (d->n0 == 0) return DG_OK;
            return count_matmul(d, counts);
        case DG_K_EMPTY:
            counts[PF_LAUNCH] = 1;
            counts[PF_WORKGROUPS] = d->n0;
            return DG_OK;
    }
    return fail(DG_EINVAL, "perf_features_count: unknown kernel");
}

dg_status dgdiff_resolve_tile(dg_dtype in_t, int32_t nmat, int64_t nelem, int32_t nunit,
                              dg_tile* tile) {
    set_error("");
    if (!tile || nmat < 1 || nmat > 8 || nunit < 1 || nunit > 512 || nelem < 1)
        return fail(DG_EINVAL, "dgdiff_resolve_tile: bad arguments");
    if (in_t == DG_F32 || in_t == DG_F64) return resolve_forward_fp(in_t, nmat, nelem, nunit, tile);
    if (in_t == DG_BF16 || in_t == DG_FP8E4M3)
        return resolve_forward_lowp(in_t, nmat, nelem, nunit, tile);
    return fail(DG_EUNSUPPORTED, "dgdiff_resolve_tile: dtype");
}

}  // extern "C"
