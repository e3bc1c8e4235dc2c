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

// One launch of the contraction kernel (dg_kernel.hpp) with nseg contraction
// segments and out_slabs output slabs: the forward (nseg 1, out_slabs nmat)
// and grad_u on it (transposed operator, nseg nmat, one output slab).
// Counts are added to c.  acc: the launch adds to the output (reads it).
dg_status count_contraction(size_t sz, int nseg, int out_slabs, int64_t E, int n, int cb,
                            const dg_tile& tile, int num_cu, bool vec_in, bool allow_pipe, bool acc,
                            int64_t* c) {
    const int kq = kern::kq_for(n);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large");
    Plan P;
    dg_status st = kern::make_plan(sz, nseg, out_slabs, E, n, kq, cb, tile.waves, tile.d_panels,
                                   tile.groups_per_cu, num_cu, vec_in, &P);
    if (st != DG_OK) return st;
    const int64_t KP = 4 * kq;
    const int64_t nwt = ceil_div(E, (int64_t)16 * cb);  // wave-tiles that start before E
    c[PF_LAUNCH] += 1;
    c[PF_WORKGROUPS] += P.grid;
    c[PF_BARRIER_X_WG] += P.grid;  // one barrier after the operator staging
    c[PF_GLD_DG_D] += 8 * P.slots * (int64_t)out_slabs * nseg * n * n * (int64_t)sz;
    // element rows read per operator group: the pipelined loads take whole
    // wave-tiles (rows past the end clamp to the last element)
    const bool piped = allow_pipe && kern::pipelined_loads(sz, n, kq, cb, n % 4 == 0, P);
    const int64_t urows = piped ? nwt * 16 * cb : E;
    c[P.vec_in ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] += urows * n * (int64_t)sz * nseg;
    c[PF_GLD_DG_U_L2] += (int64_t)(P.ngroups - 1) * urows * n * (int64_t)sz * nseg;
    // unaligned rows read through the wave slab are also written through it:
    // contiguous stores (plus one LDS write and read per output value)
    const bool stage_out = P.use_slab && n % 4 != 0;
    const int64_t out_bytes = E * out_slabs * n * (int64_t)sz;
    c[(n % 4 == 0 || stage_out) ? PF_GST_DG_OUT : PF_GST_DG_OUT_UNAL] += out_bytes;
    if (cb == 2) c[PF_DG_OUT_W32] += out_bytes;
    if (cb == 4) c[PF_DG_OUT_W64] += out_bytes;
    if (acc) c[PF_GLD_WS] += E * out_slabs * n * (int64_t)sz;
    c[PF_WAVE_TILES] += nwt * P.ngroups;
    const int64_t serial = ceil_div(P.ntiles, 8 * P.slots);  // tiles of the busiest stream
    c[PF_SERIAL_STEPS] += serial;
    c[PF_LAT_STEPS] += serial * 64 / ((int64_t)tile.groups_per_cu * tile.waves);
    c[PF_LDS_BYTES] += 8 * P.slots * P.panels_total * 16 * nseg * KP * (int64_t)sz  // staging stores
                       + nwt * P.panels_total * 64 * kq * (int64_t)sz * nseg    // operand reads
                       + (P.use_slab ? (int64_t)P.ngroups * 2 * E * n * (int64_t)sz * nseg : 0)
                       + (stage_out ? 2 * E * out_slabs * n * (int64_t)sz : 0);
    c[sz == 8 ? PF_MFMA_F64 : PF_MFMA_F32] += nwt * P.panels_total * kq * (int64_t)cb * 2048 * nseg;
    c[PF_STAGE_CHAIN] += (int64_t)P.ppg * 16 * nseg * KP * (int64_t)sz;   // the first group's panels
    return DG_OK;
}

dg_status count_dg_fp(const perf_kernel_desc* d, int64_t* c) {
    const size_t sz = d->dtype == DG_F64 ? 8 : 4;
    const int V = (int)(16 / sz);
    const int n = d->nunit;
    const int kq = kern::kq_for(n);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large");
    int cb;
    dg_status st = kern::forward_cb(sz, kq, n % V == 0, d->tile.elems_per_wave, &cb);
    if (st != DG_OK) return st;
    return count_contraction(sz, 1, d->nmat, d->n0, n, cb, d->tile, d->num_cu, n % V == 0, true, false, c);
}

// grad_u = sum_m D_m^T g_m as a 128 x 128-tile GEMM (output nodes x elements,
// contraction over (m, i) in chunks of 16 nodes of one operator), FP32.
void count_bwd_u_gemm(int64_t E, int n, int M, int64_t* c) {
    const int64_t T = kern::kBwdTile;
    const int64_t ntile_e = ceil_div(E, T), ntile_j = ceil_div(n, T);
    const int64_t active = ntile_e * ntile_j;        // blocks past the last tile return at once
    const int64_t nchunk = (int64_t)M * ceil_div(n, 16);
    c[PF_LAUNCH] += 1;
    c[PF_WORKGROUPS] += ceil_div(ntile_e, 8) * 8 * ntile_j;
    c[PF_BARRIER_X_WG] += active * (1 + nchunk);
    c[PF_GLD_DG_D] += ntile_e * M * (int64_t)n * n * 4;
    // g rows: the first output-node tile reads them from memory, later ones
    // (rows over 128 nodes) from the XCD's L2
    c[n % 4 == 0 ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] += E * M * (int64_t)n * 4;
    c[PF_GLD_DG_U_L2] += (ntile_j - 1) * E * M * (int64_t)n * 4;
    c[n % 4 == 0 ? PF_GST_DG_OUT : PF_GST_DG_OUT_UNAL] += E * (int64_t)n * 4;
    c[PF_LDS_BYTES] += active * nchunk * 256 * (64 + 128);  // chunk stores + operand reads
    c[PF_MFMA_F32] += active * nchunk * 4 * 64 * 2048;
    c[PF_SERIAL_STEPS] += nchunk;
}

dg_status count_bwd_u(const perf_kernel_desc* d, int64_t* c) {
    const size_t sz = d->dtype == DG_F64 ? 8 : 4;
    const int V = (int)(16 / sz);
    const int64_t E = d->n0;
    const int n = d->nunit, M = d->nmat;
    if (d->tile.flags & DG_TILE_BATCH_GEMM) {
        if (sz != 4 || n < 97) return fail(DG_EINVAL, "grad_u GEMM body: FP32 rows of 97 or more nodes only");
        count_bwd_u_gemm(E, n, M, c);
        return DG_OK;
    }
    if (d->tile.elems_per_wave != 16) return fail(DG_EINVAL, "grad_u contraction: elems_per_wave 16");
    const int kq = kern::kq_for(n);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large");
    const int nseg = kern::grad_u_segments(sz, M, kq);
    if (nseg == M) {
        const bool vec = n % V == 0 && (nseg == 1 || (E * n) % V == 0);
        return count_contraction(sz, nseg, 1, E, n, 1, d->tile, d->num_cu, vec, false, false, c);
    }
    for (int m = 0; m < M; ++m) {
        dg_status st = count_contraction(sz, 1, 1, E, n, 1, d->tile, d->num_cu, n % V == 0, false, m > 0, c);
        if (st != DG_OK) return st;
    }
    return DG_OK;
}

// grad_D: split partial tiles (kernel 1), group sums (kernel 2), final sums (kernel 3).
dg_status count_bwd_d(const perf_kernel_desc* d, int64_t* c) {
    const int64_t sz = d->dtype == DG_F64 ? 8 : 4;
    const int V = (int)(16 / sz);
    const int64_t E = d->n0;
    const int n = d->nunit, M = d->nmat;
    const int64_t count = (int64_t)M * n * n;
    const int fl = sz == 8 ? PF_VALU_F64 : PF_VALU_F32;
    if (E == 0) {  // the empty sum: one launch writes zeros
        c[PF_LAUNCH] += 1;
        c[PF_WORKGROUPS] += ceil_div(count, 256);
        c[PF_GST_DG_OUT_UNAL] += count * sz;
        return DG_OK;
    }
    kern::SplitPlan sp;
    if (!kern::bwd_split_plan(M, E, n, d->tile.groups_per_cu, d->num_cu, (size_t)sz, 0, &sp))
        return fail(DG_EINVAL, "grad_D split plan");
    const int64_t ntile = ceil_div(n, kern::kBwdTile);
    const int64_t tiles = M * ntile * ntile;
    const int64_t chunks = tiles * ceil_div(E, kern::kBwdChunk);  // (work-group, chunk) pairs
    c[PF_LAUNCH] += 3;
    c[PF_WORKGROUPS] += tiles * sp.nsplit + ceil_div(count, 256) * sp.ngroups + ceil_div(count, 256);
    c[PF_BARRIER_X_WG] += tiles * sp.nsplit + chunks;
    // every element's g and u rows, once per output tile row / column
    c[n % V == 0 ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] += E * sz * M * 2 * ntile * n;
    c[PF_LDS_BYTES] += chunks * (256 * 16 + 4 * 64 * 32) * sz;   // chunk stores + operand reads
    c[sz == 8 ? PF_MFMA_F64 : PF_MFMA_F32] += chunks * 4 * 64 * 2048;
    c[PF_GST_WS] += sp.nsplit * count * sz + sp.ngroups * count * sz;
    c[PF_GLD_WS] += sp.nsplit * count * sz + sp.ngroups * count * sz;
    c[fl] += sp.nsplit * count + sp.ngroups * count;
    c[PF_GST_DG_OUT_UNAL] += count * sz;
    c[PF_SERIAL_STEPS] += ceil_div(std::min(sp.split_len, E), (int64_t)kern::kBwdChunk);
    return DG_OK;
}

// dgdiff_quantize: the launch shape of quant_plan; code stores are 4-value
// vectors of codes where the row layout allows (cols % 4 == 0).
dg_status count_quant(const perf_kernel_desc* d, int64_t* c) {
    const int fp8 = d->dtype == DG_FP8E4M3 ? 1 : 0;
    const int64_t rows = d->n0, cols = d->nunit, esz = fp8 ? 1 : 2;
    const int per_row = d->nmat ? 1 : 0;
    if (rows == 0 || cols == 0) return DG_OK;
    const QuantPlan P = quant_plan(fp8, rows, cols, per_row);
    if (P.kind == QuantPlan::kGlobal) {
        const int64_t N = rows * cols, tail = N % 4, waves = 4 * P.blocks;
        c[PF_LAUNCH] += 4;
        c[PF_WORKGROUPS] += 2 + 2 * P.blocks;
        c[PF_GST_WS] += 4 + 4 * P.blocks;       // cleared maximum; one atomic maximum per work-group
        c[PF_GLD_WS] += 4 * waves + 4;          // the maximum, read once per encode wave and at the end
        c[PF_LDS_BYTES] += 32 * P.blocks;       // four wave maxima stored and read back per work-group
        c[PF_BARRIER_X_WG] += P.blocks;
        c[PF_GLD_DG_U] += 2 * 4 * (N - tail);   // maximum pass and encode pass, 16-byte vectors
        c[PF_GLD_DG_U_UNAL] += 2 * 4 * tail;
        c[PF_GST_DG_OUT] += N - tail;           // four codes per store
        c[PF_GST_DG_OUT_UNAL] += tail + 4;      // tail codes; the inverse scale
        c[PF_VALU_F32] += N;                    // x * s
        c[PF_SERIAL_STEPS] += ceil_div(N / 4, 256 * P.blocks);
        // wave-steps of the two vector loops: with T threads, wave w runs
        // nv / T trips plus one while its first vector 64 w is below nv % T
        const int64_t T = 256 * P.blocks, nv = N / 4;
        c[PF_WAVE_TILES] += 2 * ((T / 64) * (nv / T) + ceil_div(nv % T, 64));
        return DG_OK;
    }
    const int64_t vec = cols % 4 == 0;
    c[PF_LAUNCH] += 1 + (per_row ? 0 : 1);
    c[PF_WORKGROUPS] += P.blocks + (per_row ? 0 : 1);
    const int64_t nwaves = 4 * P.blocks;
    if (P.kind == QuantPlan::kShortRows) {
        c[vec ? PF_GLD_DG_U : PF_GLD_DG_U_UNAL] += rows * cols * 4;
        c[vec ? PF_GST_DG_OUT : PF_GST_DG_OUT_UNAL] += rows * cols * esz;
        if (fp8) c[PF_VALU_F32] += rows * 4 * ceil_div(cols, 4);   // x * s on whole 4-value vectors
        // wave-steps of four slots (a slot: 64 / sw consecutive rows): wave w
        // takes slots w, w + W, w + 2W, w + 3W, then w + 4W ...: slots / 4W
        // steps plus one while w < slots % 4W
        const int64_t slots = ceil_div(rows, 64 / P.sw);
        c[PF_SERIAL_STEPS] += ceil_div(slots, 4 * nwaves);
        c[PF_WAVE_TILES] += nwaves * (slots / (4 * nwaves)) + std::min<int64_t>(nwaves, slots % (4 * nwaves));
    } else {
        c[PF_GLD_DG_U_UNAL] += rows * cols * 4 * (fp8 ? 2 : 1);  // FP8 reads the row twice
        c[PF_GST_DG_OUT_UNAL] += rows * cols * esz;
        if (fp8) c[PF_VALU_F32] += rows * cols;
        c[PF_SERIAL_STEPS] += ceil_div(rows, nwaves);
        c[PF_WAVE_TILES] += rows;   // one row per wave-step
    }
    c[PF_GST_DG_OUT_UNAL] += per_row ? rows * 4 : 4;  // inverse scales (always requested)
    return DG_OK;
}

// The staged low-precision body (dg_lowp_staged_kernel): per work-group with
// tiles (one row group of one slab, K tiles of its stream), the group's
// operator rows loaded once, K + 2 tile loads (each tile once, the last one
// twice more: the loads run two tiles ahead), K + 1 LDS copies of loaded
// tiles (cb 16-byte chunks and one scale per thread; the last copy is the
// last tile again), K multiplies (B fragments, products, scaled results into
// the LDS rows), K writes (2 cb 16-byte LDS reads per thread, the tile's rows
// stored), K + 1 barriers, and the element buffers' padding rows zeroed once.
// Element loads of group 0's first pass are HBM reads, all others L2
// re-reads; the FP8 path reads one element scale per thread and load, and one
// operator scale per wave.
static dg_status count_dg_lowp_staged(const perf_kernel_desc* d, const LpPlan& P, int64_t* c) {
    const int64_t E = d->n0;
    const int n = d->nunit, M = d->nmat;
    const bool fp8 = d->dtype == DG_FP8E4M3;
    const int64_t eg = fp8 ? 1 : 2;             // operator bytes per value
    const int64_t ue = P.fmt == 3 ? 4 : eg;     // element-data bytes per value (FP32 when fused)
    const int64_t TE = 16 * P.cb, T = 64 * P.waves, ns = 8 * P.slots;
    const int64_t streams = std::min<int64_t>(ns, P.ntiles);   // streams with tiles
    const int64_t wgs = streams * P.ngroups;                    // work-groups with tiles
    // elements of each stream's last tile, summed over the streams with tiles
    const int64_t last_el = (streams - 1) * TE + (E - (P.ntiles - 1) * TE);
    c[PF_LAUNCH] = 1;
    c[PF_WORKGROUPS] = P.grid;
    c[PF_BARRIER_X_WG] = P.ngroups * P.ntiles + wgs;
    c[PF_WAVE_TILES] = P.ngroups * P.ntiles;
    c[PF_GLD_DG_D] = streams * M * (int64_t)n * n * eg + (fp8 ? wgs * P.waves * 4 : 0);
    c[PF_GLD_DG_U] = E * n * ue;
    c[PF_GLD_DG_U_L2] = ((int64_t)(P.ngroups - 1) * E + 2 * (int64_t)P.ngroups * last_el) * n * ue;
    if (fp8) c[PF_GLD_DG_U_UNAL] = 4 * (T / TE) * (P.ngroups * E + 2 * (int64_t)P.ngroups * last_el);
    c[PF_GST_DG_OUT] = E * M * (int64_t)n * 4;
    // per row group: its rows, its valid 16-row blocks, the waves holding one
    int64_t lds_tile = 0, mfma_tile = 0, valu_tile = 0;   // per tile, summed over the groups
    for (int rg = 0; rg < P.nrg; ++rg) {
        const int64_t rows = std::min<int64_t>((int64_t)P.rb * 16, n - (int64_t)rg * P.rb * 16);
        const int64_t blocks = ceil_div(rows, 16);
        const int64_t active = ceil_div(blocks, (int64_t)P.pw);
        lds_tile += active * (P.ks * P.cb * 64 * 16 + P.cb * 64 * 4) + rows * 64 * P.cb;
        mfma_tile += blocks * P.ks * P.cb * 16384;
        valu_tile += (int64_t)P.cb * 64 * (active + 4 * blocks);
    }
    const int64_t zrows = 4 * P.ks - n / 8;
    c[PF_LDS_BYTES] = wgs * 2 * zrows * TE * 16                          // padding rows zeroed
                      + (P.ngroups * P.ntiles + wgs) * T * (ls_chunks_in(P.cb) * 16 + 4)  // copies + scales
                      + M * P.ntiles * lds_tile                           // multiplies
                      + P.ngroups * P.ntiles * T * ls_chunks_out(P.cb) * 16;  // result rows read back
    c[PF_MFMA_BF16] = M * P.ntiles * mfma_tile;
    c[PF_VALU_F32] = M * P.ntiles * valu_tile;
    c[PF_SERIAL_STEPS] = ceil_div(P.ntiles, ns);
    c[PF_LAT_STEPS] = c[PF_SERIAL_STEPS] * 64 / ((int64_t)d->tile.groups_per_cu * P.waves);
    return DG_OK;
}

dg_status count_dg_lowp(const perf_kernel_desc* d, int64_t* c) {
    if ((d->tile.flags & DG_TILE_QUANT_U) && d->dtype != DG_BF16)
        return fail(DG_EINVAL, "DG_TILE_QUANT_U is for BF16 input");
    const int fmt = lp_format(d->dtype, &d->tile);
    LpPlan P;
    dg_status st = make_lp_plan(fmt, d->nmat, d->n0, d->nunit, &d->tile, d->tile.groups_per_cu,
                                d->num_cu, &P);
    if (st != DG_OK) return st;
    if (P.staged) return count_dg_lowp_staged(d, P, c);
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
    // operator panels staged, then read as MFMA operands; the operator scales
    // (eight per work-group) are staged too and read once per panel, or per
    // panel pair, of every wave-tile
    const bool pair = lp_pair_ok(P, n, n % 4 == 0);
    int64_t scale_reads = 0, pairs = 0;   // per wave-tile, over the groups
    for (int pg = 0; pg < P.ngroups; ++pg) {
        const int np = std::min(P.ppg, P.panels_total - pg * P.ppg);
        const int pr = pair ? np / 2 : 0;
        pairs += pr;
        scale_reads += pr + (np - 2 * pr);
    }
    c[PF_LDS_BYTES] = 8 * P.slots * P.panels_total * 16 * KP * P.lds_esz +
                      nwt * P.panels_total * P.ks * 64 * 8 * P.lds_esz +
                      P.grid * 8 * 4 + nwt * scale_reads * 64 * 4;
    c[fmt == 1 ? PF_MFMA_FP8 : PF_MFMA_BF16] = nwt * P.panels_total * P.ks * (int64_t)P.cb * 16384;
    // de-scaling: per lane and column block, one product of the two scales and
    // four multiplies per panel (a pair: one product, eight multiplies, every
    // lane); a single panel only on lanes whose element exists
    c[PF_VALU_F32] = nwt * pairs * P.cb * 64 * 9 + (P.panels_total - 2 * pairs) * 4 * E * 5;
    if (d->dtype == DG_FP8E4M3) {
        // scales: nmat operator scales per work-group; the element's scale by
        // each of its four lanes, in every operator group
        c[PF_GLD_DG_D] += P.grid * M * 4;
        c[PF_GLD_DG_U_UNAL] += (int64_t)P.ngroups * E * 4 * 4;
    }
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

// One order's share of a batched launch (dg_batched.hip), by body:
//   one element per thread (elems_per_wave 256; order 1): operator entries
//     are wave-uniform loads, 192 per wave and sweep;
//   resident operator panels (elems_per_wave 16 / 32): the plain kernel's
//     schedule over a gathered element list, rows at any 4-byte offset;
//   GEMM tiles (DG_TILE_BATCH_GEMM): 128 stacked operator rows x 128
//     elements, drawn from the pool (all of the order's tiles, in any order).
// Element ids and offsets are loaded by every lane that uses them (8 + 8 bytes).
dg_status count_batched(const perf_kernel_desc* d, int64_t* c) {
    const int64_t cnt = d->n0, G = d->workgroups;
    const int n = d->nunit;
    const int M = d->nmat;
    if (G < 1) return fail(DG_EINVAL, "batched: workgroups of the order's share needed");
    c[PF_LAUNCH] += 1;
    c[PF_WORKGROUPS] += G;
    if (cnt == 0) return DG_OK;
    if (d->tile.flags & DG_TILE_BATCH_GEMM) {
        const int64_t R = (int64_t)M * n, RB = ceil_div(R, 128), EB = ceil_div(cnt, 128);
        const int64_t nk = ceil_div(n, 16), tiles = RB * EB;
        c[PF_BARRIER_X_WG] += tiles * (3 + nk);         // claim (2) + staging (1) + chunks
        c[PF_GLD_DG_D] += EB * R * n * 4;
        c[PF_GLD_DG_U_UNAL] += cnt * (int64_t)n * 4;    // first row block of each element block
        c[PF_GLD_DG_U_L2] += (RB - 1) * cnt * (int64_t)n * 4;
        c[PF_GLD_IDX] += RB * cnt * 192;
        c[PF_GST_DG_OUT_UNAL] += R * cnt * 4;
        // chunk stores and operand reads; each claim of a tile passes the
        // tile index through LDS (one 8-byte store, read by every thread)
        c[PF_LDS_BYTES] += tiles * nk * 256 * (64 + 128) + tiles * (8 + 256 * 8);
        c[PF_MFMA_F32] += tiles * nk * 4 * 64 * 2048;
        c[PF_SERIAL_STEPS] += nk;
        return DG_OK;
    }
    if (d->tile.elems_per_wave == 256) {
        if (n != 8) return fail(DG_EINVAL, "batched: one element per thread is for nunit 8");
        const int64_t sweeps = ceil_div(cnt, 256);                  // 256-element blocks
        const int64_t full = cnt / 64, part = cnt % 64 ? 1 : 0;     // waves with work
        c[PF_GLD_IDX] += cnt * 16;
        c[PF_GLD_DG_U_UNAL] += cnt * 32;
        c[PF_GST_DG_OUT_UNAL] += cnt * 96;
        c[PF_GLD_DG_D] += (full + part) * 192 * 4;
        c[PF_VALU_F32] += cnt * 3 * 64 * 2;
        c[PF_SERIAL_STEPS] += ceil_div(sweeps, G);
        return DG_OK;
    }
    const int cb = d->tile.elems_per_wave / 16;
    if (cb != 1 && cb != 2) return fail(DG_EINVAL, "batched: elems_per_wave 16, 32, 128 or 256");
    const int kq = kern::kq_for(n);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large");
    const int64_t mblk = ceil_div(n, 16), panels = M * mblk;
    const int64_t ppg = std::max<int64_t>(1, std::min<int64_t>(d->tile.d_panels, panels));
    const int64_t ngroups = ceil_div(panels, ppg);
    if (G % (8 * ngroups)) return fail(DG_EINVAL, "batched: workgroups not a multiple of 8 x groups");
    const int64_t nstreams = 8 * (G / (8 * ngroups));
    const int64_t ntiles = ceil_div(cnt, (int64_t)16 * cb * 4);
    const int64_t nwt = ceil_div(cnt, (int64_t)16 * cb);
    c[PF_BARRIER_X_WG] += G;
    c[PF_GLD_DG_D] += nstreams * M * (int64_t)n * n * 4;
    c[PF_GLD_IDX] += ngroups * cnt * 64;
    c[PF_GLD_DG_U_UNAL] += cnt * (int64_t)n * 4;
    c[PF_GLD_DG_U_L2] += (ngroups - 1) * cnt * (int64_t)n * 4;
    c[PF_GST_DG_OUT_UNAL] += cnt * M * (int64_t)n * 4;
    c[PF_WAVE_TILES] += nwt * ngroups;
    c[PF_LDS_BYTES] += nstreams * panels * 16 * 4 * kq * 4     // staging stores
                       + nwt * panels * 256 * kq;               // operand reads
    c[PF_MFMA_F32] += nwt * panels * kq * (int64_t)cb * 2048;
    const int64_t serial = ceil_div(ntiles, nstreams);
    c[PF_SERIAL_STEPS] += serial;
    c[PF_LAT_STEPS] += serial * 64 / (std::max(1, d->tile.groups_per_cu) * 4);
    c[PF_STAGE_CHAIN] += ppg * 16 * 4 * kq * 4;
    return DG_OK;
}

// A work-removed twin: the original's global accesses, launches, work-groups
// and schedule; no LDS, matrix-core work or barriers; one add per loaded value.
void remove_work(int64_t* c) {
    c[PF_LDS_BYTES] = c[PF_BARRIER_X_WG] = 0;
    c[PF_MFMA_F64] = c[PF_MFMA_F32] = c[PF_MFMA_BF16] = c[PF_MFMA_FP8] = 0;
    c[PF_VALU_F64] = 0;
    int64_t loaded = 0;
    for (int k : {PF_GLD_DG_U, PF_GLD_DG_U_L2, PF_GLD_DG_D, PF_GLD_ST_U, PF_GLD_MM_AB, PF_GLD_DG_U_UNAL})
        loaded += c[k];
    c[PF_VALU_F32] = loaded / 4;
}

dg_status count_ubench(const dg_ubench_desc* d, int64_t* c) {
    const int64_t n = d->n;
    c[PF_LAUNCH] = 1;
    switch (d->kind) {
        case DG_UB_STREAM: {
            const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), kUbStreamBlocks));
            c[PF_WORKGROUPS] = blocks;
            c[PF_GLD_UB] = (int64_t)d->a * 16 * n;
            c[PF_GST_UB] = 16 * n;
            c[PF_VALU_F32] = (int64_t)(d->a - 1) * 4 * n;
            c[PF_SERIAL_STEPS] = ceil_div(n, 256 * blocks);
            return DG_OK;
        }
        case DG_UB_STRIDED:
            c[PF_WORKGROUPS] = ceil_div(n, 256);
            c[PF_GLD_UB_STRIDED] = 4 * n;
            c[PF_GST_UB] = 4 * n;
            c[PF_SERIAL_STEPS] = 1;
            return DG_OK;
        case DG_UB_FMA:
            // initial values (one product, 32 adds), a trip's 64 fused multiply-adds, the 31-add sum
            c[PF_WORKGROUPS] = n;
            c[PF_VALU_F32] = 256 * n * (33 + 128 * (int64_t)d->a + 31);
            c[PF_GST_UB] = 256 * n * 4;
            c[PF_SERIAL_STEPS] = d->a;
            return DG_OK;
        case DG_UB_MFMA:
            c[PF_WORKGROUPS] = n;
            c[d->dtype == DG_BF16 ? PF_MFMA_BF16 : PF_MFMA_F32] =
                4 * n * (int64_t)d->a * 8 * (d->dtype == DG_BF16 ? 16384 : 2048);
            c[PF_VALU_F32] = 256 * n * 7 * 4;   // the eight accumulators summed
            c[PF_GST_UB] = 256 * n * 16;
            c[PF_SERIAL_STEPS] = d->a;
            return DG_OK;
        case DG_UB_LDS:
            c[PF_WORKGROUPS] = n;
            c[PF_GLD_UB] = 256 * n * 4 * d->b;
            c[PF_GST_UB] = 256 * n * 4 * d->b;
            c[PF_LDS_BYTES] = 256 * n * 4 * d->b * (2 * (int64_t)d->a + 2);
            c[PF_SERIAL_STEPS] = d->a;
            return DG_OK;
        case DG_UB_BARRIER:
            c[PF_WORKGROUPS] = n;
            c[PF_BARRIER_X_WG] = n * d->a;
            c[PF_GST_UB] = 256 * n * 4;
            c[PF_SERIAL_STEPS] = d->a;
            return DG_OK;
        case DG_UB_OVERLAP: {
            const int64_t blocks = ceil_div(n, 256);
            c[PF_WORKGROUPS] = blocks;
            c[PF_GLD_UB] = 16 * n;
            c[PF_GST_UB] = 16 * n;
            c[PF_LDS_BYTES] = 256 * blocks * (int64_t)d->a * 32;
            c[PF_SERIAL_STEPS] = d->a;
            return DG_OK;
        }
        case DG_UB_TILE_READ: {
            const int64_t trips = n / 16;
            c[PF_WORKGROUPS] = trips * trips;
            c[d->a == 1 ? PF_GLD_UB_STRIDED : PF_GLD_UB] = n * n * trips * 4;
            c[PF_GST_UB] = n * n * 4;
            c[PF_VALU_F32] = n * n * trips;
            c[PF_SERIAL_STEPS] = trips;
            return DG_OK;
        }
        case DG_UB_TWIN_DG: {
            perf_kernel_desc f = {};
            f.kernel = DG_K_DGDIFF;
            f.dtype = DG_F32;
            f.n0 = n;
            f.nunit = d->a;
            f.nmat = d->b;
            f.tile = d->tile;
            f.num_cu = d->num_cu;
            c[PF_LAUNCH] = 0;
            dg_status st = count_dg_fp(&f, c);
            if (st != DG_OK) return st;
            remove_work(c);
            return DG_OK;
        }
        case DG_UB_TWIN_STENCIL:
        case DG_UB_TWIN_MATMUL: {
            perf_kernel_desc f = {};
            f.kernel = d->kind == DG_UB_TWIN_STENCIL ? DG_K_STENCIL5 : DG_K_MATMUL;
            f.dtype = DG_F32;
            f.n0 = n;
            f.num_cu = d->num_cu;
            for (int k = 0; k < PF_COUNT; ++k) c[k] = 0;
            dg_status st = d->kind == DG_UB_TWIN_STENCIL ? count_stencil(&f, c) : count_matmul(&f, c);
            if (st != DG_OK) return st;
            remove_work(c);
            return DG_OK;
        }
    }
    return fail(DG_EINVAL, "perf_ubench_count: unknown kind");
}

const char* kNames[PF_COUNT] = {
    "launch", "workgroups", "barrier_x_wg", "gld_dg_u", "gld_dg_u_l2", "gld_dg_d", "gst_dg_out",
    "gld_st_u", "gst_st_res", "gld_mm_ab", "gst_mm_c", "lds_bytes", "mfma_f64", "mfma_f32",
    "mfma_bf16", "mfma_fp8", "valu_f32", "valu_f64", "gld_dg_u_unal", "gst_dg_out_unal",
    "wave_tiles", "serial_steps", "lat_steps", "gld_ws", "gst_ws", "gld_idx", "gld_ub", "gst_ub",
    "gld_ub_strided", "dg_out_w32", "dg_out_w64", "stage_chain"};

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
            if (d->tile.waves < 1 || d->tile.waves > 16 || d->tile.elems_per_wave == 0 ||
                d->tile.groups_per_cu < 1 || d->tile.d_panels < 1 || d->num_cu < 1)
                return fail(DG_EINVAL, "perf_features_count: DG needs a resolved tile and num_cu");
            if (d->n0 == 0) return DG_OK;
            if (d->dtype == DG_F32 || d->dtype == DG_F64) {
                if (d->tile.waves > 8) return fail(DG_EINVAL, "tile.waves must be in 1..8");
                return count_dg_fp(d, counts);
            }
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
        case DG_K_BWD_U:
        case DG_K_BWD_D:
            if (d->dtype != DG_F32 && d->dtype != DG_F64) return fail(DG_EUNSUPPORTED, "adjoint dtype");
            if (d->nunit < 1 || d->nunit > 512 || d->nmat < 1 || d->nmat > 8)
                return fail(DG_EUNSUPPORTED, "perf_features_count: adjoint sizes");
            if (d->num_cu < 1 || d->tile.groups_per_cu < 1)
                return fail(DG_EINVAL, "perf_features_count: adjoint needs dgdiff_resolve_backward's tile and num_cu");
            if (d->kernel == DG_K_BWD_D) return count_bwd_d(d, counts);
            if (d->n0 == 0) return DG_OK;
            if (!(d->tile.flags & DG_TILE_BATCH_GEMM) && (d->tile.waves < 1 || d->tile.d_panels < 1))
                return fail(DG_EINVAL, "perf_features_count: grad_u needs a resolved tile");
            return count_bwd_u(d, counts);
        case DG_K_QUANT:
            if (d->dtype != DG_BF16 && d->dtype != DG_FP8E4M3) return fail(DG_EUNSUPPORTED, "quantiser target");
            if (d->nunit < 0) return fail(DG_EINVAL, "quantiser cols");
            return count_quant(d, counts);
        case DG_K_BATCHED:
            if (d->dtype != DG_F32 || d->nmat != 3 || d->nunit < 1 || d->nunit > 512)
                return fail(DG_EUNSUPPORTED, "perf_features_count: batched orders are FP32, nmat 3");
            return count_batched(d, counts);
        case DG_K_BATCHED_POOL:
            // every work-group joins the pool: one barrier before it, and the
            // claim that finds each of the eight pools drained (two barriers)
            counts[PF_BARRIER_X_WG] = 17 * d->n0;
            counts[PF_LDS_BYTES] = 8 * d->n0 * (8 + 256 * 8);   // the eight claims that find a pool drained
            return DG_OK;
    }
    return fail(DG_EINVAL, "perf_features_count: unknown kernel");
}

dg_status perf_ubench_count(const dg_ubench_desc* d, int64_t* counts) {
    set_error("");
    if (!d || !counts) return fail(DG_EINVAL, "perf_ubench_count: NULL argument");
    for (int k = 0; k < PF_COUNT; ++k) counts[k] = 0;
    dg_status st = check_ubench(d);
    if (st != DG_OK) return st;
    if (d->n == 0) return DG_OK;
    return count_ubench(d, counts);
}

dg_status dgdiff_resolve_backward(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit,
                                  dg_tile* tile_u, dg_tile* tile_d) {
    set_error("");
    if ((t != DG_F32 && t != DG_F64) || nmat < 1 || nmat > 8 || nunit < 1 || nunit > 512 || nelem < 1)
        return fail(DG_EINVAL, "dgdiff_resolve_backward: bad arguments");
    return resolve_backward(t, nmat, nelem, nunit, tile_u, tile_d);
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
