/*
 * Brute-force operation counts — TEST INFRASTRUCTURE ONLY (oracle).
 *
 * The paper obtains a kernel's operation counts by counting, for every
 * statement, the integer points of the loop domain projected onto the loops
 * that enclose it, times the operations one execution performs (its
 * per-statement count algorithm).  Here that sum is taken literally: every
 * work-group, wave, element tile, lane and loop iteration of a kernel's
 * documented schedule is walked, and each executed statement adds the bytes
 * or flops it moves.  No closed form is used anywhere in this file; the
 * library's closed forms must reproduce these counts exactly.
 *
 * Counting rules (the paper's granularities, as read here):
 *   global and LDS traffic in bytes of the lanes that execute the access;
 *   matrix-core flops of every executed MFMA instruction (2*16*16*K);
 *   VALU flops per computing lane; barriers per work-item, times work-groups.
 *
 * The launch-shape rules restated below (operator panel groups, XCD slots,
 * paths taken) describe the schedule that is counted; they are part of the
 * kernels' documented interface, not shared code.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* feature slots, in the order of the library's interface */
enum { F_LAUNCH, F_WG, F_BAR, F_U, F_U_L2, F_D, F_OUT, F_ST_U, F_ST_RES, F_MM_AB, F_MM_C, F_LDS,
       F_MFMA_F64, F_MFMA_F32, F_MFMA_BF16, F_MFMA_FP8, F_VALU_F32, F_VALU_F64, F_U_UNAL, F_OUT_UNAL,
       F_WAVE_TILES, F_SERIAL, F_LAT, F_WS_LD, F_WS_ST, F_IDX, F_UB_LD, F_UB_ST, F_UB_LD_STRIDED,
       F_OUT_W32, F_OUT_W64, F_STAGE, F_N };

enum { K_DG = 0, K_STENCIL = 1, K_MATMUL = 2, K_EMPTY = 3, K_BWD_U = 4, K_BWD_D = 5, K_QUANT = 6,
       K_BATCHED = 7, K_BATCHED_POOL = 8 };
enum { T_F64 = 0, T_F32 = 1, T_BF16 = 2, T_FP8 = 3 };

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t mini(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t maxi(int64_t a, int64_t b) { return a > b ? a : b; }

/* smallest k in the kernel's instantiated list with k >= ceil(n/4) rounded up to 4 */
static int kq_of(int n) {
    static const int list[] = {4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64, 72, 80, 88, 96, 112, 128};
    int need = (int)(cdiv(cdiv(n, 4), 4) * 4);
    for (unsigned k = 0; k < sizeof(list) / sizeof(list[0]); ++k)
        if (list[k] >= need) return list[k];
    return -1;
}

/* ---------------------------------------------------------------- DG forward */

/* One launch of the contraction kernel.  nseg contraction segments (grad_u:
   the nmat slabs of g, operator transposed), M output slabs; allow_pipe: the
   forward's paired-store launch (pipelined element loads may apply); acc:
   the launch adds to its output (reads each value it writes). */
static int dg_walk(int dtype, int64_t E, int n, int nseg, int M, int epw, int waves, int per_cu,
                   int d_panels, int flags, int num_cu, int allow_pipe, int acc, int64_t* c) {
    const int lowp = dtype == T_BF16 || dtype == T_FP8;
    const int native = dtype == T_FP8 && (flags & 2);
    const int64_t sz = dtype == T_F64 ? 8 : 4;      /* FP element size */
    const int64_t eg = dtype == T_BF16 ? 2 : 1;     /* low-precision element size in HBM */
    const int64_t el = native ? 1 : 2;              /* low-precision element size in LDS */
    const int cb = epw / 16;
    /* the FP kernel's output stores by wave tiles of 32 or 64 elements carry
       their own pattern tag as well */
    const int wide_tag = lowp ? -1 : cb == 2 ? F_OUT_W32 : cb == 4 ? F_OUT_W64 : -1;
    int KQ, KP, V = 0, KS = 0;
    if (lowp) {
        KS = (int)cdiv(n, 32);
        KQ = 8 * KS;
        KP = 32 * KS;
    } else {
        KQ = kq_of(n);
        if (KQ < 0) return 1;
        KP = 4 * KQ;
        V = (int)(16 / sz);
    }
    /* launch shapes the library documents as unavailable: an element tile
       of 64 per wave needs the wave's element fragments within 128 bytes per
       lane (FP32 nunit <= 128, FP64 nunit <= 64; low precision nunit <= 256),
       waves per work-group 1..8, and the staged operator panels (plus a wave
       slab) within the 160 KB LDS */
    if (waves < 1 || waves > 8) return 1;
    if (epw != 16 && epw != 32 && epw != 64) return 1;
    if (epw == 64 && (lowp ? KS > 8 : KQ * sz > 128)) return 1;
    if (lowp && KS > 16) return 1;
    const int mblk = (int)cdiv(n, 16);
    const int P = M * mblk;
    const int ppg = (int)mini(d_panels, P);
    const int NG = (int)cdiv(P, ppg);
    const int64_t Te = 16LL * cb * waves;
    const int64_t ntiles = cdiv(E, Te);
    const int64_t cap = maxi(1, (int64_t)per_cu * num_cu / (8 * NG));
    const int64_t slots = maxi(1, mini(cap, cdiv(ntiles, 8)));
    const int64_t G = 8 * NG * slots;
    const int64_t nstreams = 8 * slots;
    /* paths */
    const int vec_in = lowp ? (n % 8 == 0) : (n % V == 0);
    int use_slab = 0;
    if (!lowp && !vec_in) {
        int64_t panel_bytes = 16 * (nseg * 4LL * KQ + V) * sz;
        int64_t slab = (int64_t)waves * nseg * cdiv(16LL * cb * n, V) * V * sz;
        use_slab = slab + panel_bytes <= 80 * 1024;
    }
    {
        const int64_t panel = lowp ? 16 * (32LL * KS * el + 16) : 16 * (nseg * 4LL * KQ + V) * sz;
        const int64_t slab = use_slab ? (int64_t)waves * nseg * cdiv(16LL * cb * n, V) * V * sz : 0;
        if (ppg * panel + slab > 160 * 1024) return 1;
    }
    const int vec_out = n % 4 == 0;
    /* unaligned rows that come through the wave slab leave through it too */
    const int stage_out = !lowp && use_slab && !vec_out;
    /* FP32 rows of a multiple of 32 nodes in even panel groups are stored in
       panel pairs; with small fragments (KQ * cb <= 32) their element loads are
       issued a tile ahead, every lane of a wave-tile loading all its vectors
       (rows past the end read the last element) */
    const int piped = allow_pipe && !lowp && sz == 4 && vec_in && vec_out && n % 32 == 0 &&
                      mblk % 2 == 0 && ppg % 2 == 0 && KQ * cb <= 32;

    c[F_LAUNCH] += 1;
    c[F_WG] += G;
    int64_t serial = 0, stage_max = 0;
    for (int64_t b = 0; b < G; ++b) {
        const int64_t xcd = b % 8, kb = b / 8;
        const int pg = (int)(kb % NG);
        const int64_t stream = (kb / NG) * 8 + xcd;
        const int p_lo = pg * ppg;
        const int np = (int)mini(ppg, P - p_lo);
        /* operator staging: one lane-iteration per LDS slot */
        const int KS2 = lowp ? KP : nseg * KP;   /* staged columns per row */
        int64_t staged = 0;
        for (int64_t idx = 0; idx < (int64_t)np * 16 * KS2; ++idx) {
            const int k = (int)(idx % KS2) % KP;
            const int rr = (int)(idx / KS2);
            const int panel = p_lo + rr / 16;
            const int o = (panel % mblk) * 16 + rr % 16;
            if (o < n && k < n) c[F_D] += lowp ? eg : sz;
            c[F_LDS] += lowp ? el : sz;
            staged += lowp ? el : sz;
        }
        if (!lowp && staged > stage_max) stage_max = staged;
        if (lowp) {
            /* threads 0..7 stage the operator scales (1 where none are given):
               FP8 reads the nmat given ones */
            for (int t = 0; t < 8; ++t) {
                c[F_LDS] += 4;
                if (dtype == T_FP8 && t < M) c[F_D] += 4;
            }
        }
        c[F_BAR] += 1;
        /* element-data tag: re-reads by groups > 0, else by access path */
        const int tag = pg != 0 ? F_U_L2 : vec_in ? F_U : F_U_UNAL;
        int64_t steps = 0;
        for (int64_t tile = stream; tile < ntiles; tile += nstreams) {
            ++steps;
            for (int w = 0; w < waves; ++w) {
                const int64_t e0 = tile * Te + (int64_t)w * 16 * cb;
                if (e0 >= E) continue;
                c[F_WAVE_TILES] += 1;
                /* element data */
                if (lowp) {
                    for (int q = 0; q < cb; ++q)
                        for (int lane = 0; lane < 64; ++lane) {
                            const int cc = lane & 15, g = lane >> 4;
                            const int64_t e = e0 + q * 16 + cc;
                            if (dtype == T_FP8 && e < E) c[F_U_UNAL] += 4;   /* the element's scale */
                            for (int s = 0; s < KS; ++s) {
                                if (vec_in) {
                                    if (e < E && g * KQ + 8 * s < n) c[tag] += 8 * eg;
                                } else {
                                    for (int t = 0; t < 8; ++t)
                                        if (e < E && g * KQ + 8 * s + t < n) c[tag] += eg;
                                }
                            }
                        }
                } else {
                    for (int sg = 0; sg < nseg; ++sg) {   /* each contraction segment's rows */
                        if (piped) {
                            for (int q = 0; q < cb; ++q)
                                for (int lane = 0; lane < 64; ++lane)
                                    for (int s = 0; s < KQ; s += V) c[tag] += 16;
                        } else if (vec_in) {
                            for (int q = 0; q < cb; ++q)
                                for (int lane = 0; lane < 64; ++lane) {
                                    const int cc = lane & 15, g = lane >> 4;
                                    const int64_t e = e0 + q * 16 + cc;
                                    if (e >= E) continue;
                                    for (int s = 0; s < KQ; s += V)
                                        if (g * KQ + s < n) c[tag] += 16;
                                }
                        } else if (!use_slab) {
                            for (int q = 0; q < cb; ++q)
                                for (int lane = 0; lane < 64; ++lane) {
                                    const int cc = lane & 15, g = lane >> 4;
                                    const int64_t e = e0 + q * 16 + cc;
                                    for (int t = 0; t < KQ; ++t)
                                        if (e < E && g * KQ + t < n) c[tag] += sz;
                                }
                        } else {
                            const int64_t nel = mini(16LL * cb, E - e0);
                            const int64_t len = nel * n;
                            for (int64_t f = 0; f < len; ++f) {   /* slab copy: load + LDS store */
                                c[tag] += sz;
                                c[F_LDS] += sz;
                            }
                            for (int q = 0; q < cb; ++q)
                                for (int lane = 0; lane < 64; ++lane) {
                                    const int cc = lane & 15, g = lane >> 4;
                                    const int elx = q * 16 + cc;
                                    for (int t = 0; t < KQ; ++t)
                                        if (elx < nel && g * KQ + t < n) c[F_LDS] += sz;
                                }
                        }
                    }
                }
                const int64_t nel_w = mini(16LL * cb, E - e0);
                /* panels */
                for (int pp = 0; pp < np; ++pp) {
                    const int panel = p_lo + pp;
                    const int i0 = (panel % mblk) * 16;
                    if (lowp) {
                        for (int s = 0; s < KS; ++s) {
                            c[F_LDS] += 64 * 8 * el;                    /* operand read */
                            for (int q = 0; q < cb; ++q) c[native ? F_MFMA_FP8 : F_MFMA_BF16] += 16384;
                        }
                        /* de-scaling: panel pairs (rows of a multiple of 32 nodes,
                           even panel groups) read the operator scale once and scale
                           both panels on every lane; single panels on lanes whose
                           element exists (one product of scales, four multiplies) */
                        const int lp_pair = vec_out && n % 32 == 0 && mblk % 2 == 0 && ppg % 2 == 0;
                        if (lp_pair && pp % 2 == 0 && pp + 1 < np) {
                            c[F_LDS] += 64 * 4;
                            for (int q = 0; q < cb; ++q) c[F_VALU_F32] += 64 * 9;
                        } else if (!(lp_pair && pp % 2 == 1)) {
                            c[F_LDS] += 64 * 4;
                            for (int q = 0; q < cb; ++q)
                                for (int lane = 0; lane < 64; ++lane)
                                    if (e0 + q * 16 + (lane & 15) < E) c[F_VALU_F32] += 5;
                        }
                    } else {
                        for (int sg = 0; sg < nseg; ++sg)
                            for (int s = 0; s < KQ; s += V) {
                                c[F_LDS] += 64 * 16;                    /* 16-byte operand read */
                                for (int t = 0; t < V; ++t)
                                    for (int q = 0; q < cb; ++q)
                                        c[sz == 8 ? F_MFMA_F64 : F_MFMA_F32] += 2048;
                            }
                    }
                    if (stage_out) {
                        /* each lane puts its four results into the slab ... */
                        for (int q = 0; q < cb; ++q)
                            for (int lane = 0; lane < 64; ++lane) {
                                const int cc = lane & 15, g = lane >> 4;
                                if (q * 16 + cc >= nel_w) continue;
                                for (int r = 0; r < 4; ++r)
                                    if (i0 + 4 * g + r < n) c[F_LDS] += sz;
                            }
                        /* ... and after the last panel of this output slab in the
                           group, the wave copies the staged rows out */
                        const int m = panel / mblk;
                        const int pf = (int)maxi(p_lo, (int64_t)m * mblk);
                        const int pl = (int)mini(p_lo + np, (int64_t)(m + 1) * mblk);
                        if (panel + 1 == pl) {
                            const int64_t rows = mini((int64_t)(pl - m * mblk) * 16, n) - (pf - m * mblk) * 16;
                            for (int64_t f = 0; f < nel_w * rows; ++f) {
                                c[F_LDS] += sz;
                                c[F_OUT] += sz;
                                if (wide_tag >= 0) c[wide_tag] += sz;
                                if (acc) c[F_WS_LD] += sz;   /* the value added to */
                            }
                        }
                        continue;
                    }
                    for (int q = 0; q < cb; ++q)
                        for (int lane = 0; lane < 64; ++lane) {
                            const int cc = lane & 15, g = lane >> 4;
                            const int64_t e = e0 + q * 16 + cc;
                            if (e >= E) continue;
                            const int i = i0 + 4 * g;
                            const int64_t osz = lowp ? 4 : sz;
                            if (acc)
                                for (int r = 0; r < 4; ++r)
                                    if (i + r < n) c[F_WS_LD] += osz;   /* the value added to */
                            if (vec_out) {
                                if (i < n) {
                                    c[F_OUT] += 4 * osz;
                                    if (wide_tag >= 0) c[wide_tag] += 4 * osz;
                                }
                            } else {
                                for (int r = 0; r < 4; ++r)
                                    if (i + r < n) {
                                        c[F_OUT_UNAL] += osz;
                                        if (wide_tag >= 0) c[wide_tag] += osz;
                                    }
                            }
                        }
                }
            }
        }
        if (steps > serial) serial = steps;
    }
    /* latency left unhidden: the busiest stream's steps over resident waves
       per SIMD (per_cu work-groups of `waves` waves on 4 SIMDs), x 64 */
    c[F_SERIAL] += serial;
    c[F_LAT] += serial * 64 / ((int64_t)per_cu * waves);
    c[F_STAGE] += stage_max;   /* the most any one work-group staged before its first tile */
    return 0;
}

/* ---------------------------------------------------------------- stencil */

static int stencil_rows(int64_t n) {
    if (n >= 8192) return 32;
    if (n >= 4096) return 16;
    if (n >= 2048) return 8;
    return 4;
}

static void stencil_walk(int dtype, int64_t n, int64_t* c) {
    c[F_LAUNCH] += 1;
    if (dtype == T_F32 && n % 4 == 0) {
        const int64_t R = stencil_rows(n), gx = cdiv(n, 1024), gy = cdiv(n, R);
        c[F_WG] += gx * gy;
        for (int64_t by = 0; by < gy; ++by)
            for (int64_t bx = 0; bx < gx; ++bx)
                for (int t = 0; t < 256; ++t) {
                    const int lane = t & 63, wave = t >> 6;
                    const int64_t j0 = (bx * 4 + wave) * 256 + 4 * lane;
                    const int active = j0 < n;
                    const int self_halo = lane == 63 || j0 + 4 >= n;
                    const int64_t i_lo = by * R, i_hi = mini(n, i_lo + R);
                    if (i_hi - i_lo > c[F_SERIAL]) c[F_SERIAL] = i_hi - i_lo;
                    /* rows i_lo .. i_hi+1 are loaded once each (the other lanes'
                       right halo comes by a wave shuffle, which moves no LDS bytes) */
                    for (int64_t r = i_lo; r < i_hi + 2; ++r) {
                        if (active) c[F_ST_U] += 16;
                        if (active && self_halo) c[F_ST_U] += 8;
                    }
                    for (int64_t i = i_lo; i < i_hi; ++i) {
                        c[F_VALU_F32] += 4 * 5;
                        if (active) c[F_ST_RES] += 16;
                    }
                }
    } else {
        const int64_t sz = dtype == T_F64 ? 8 : 4;
        const int64_t gx = cdiv(n, 64), gy = cdiv(n, 4);
        c[F_WG] += gx * gy;
        for (int64_t by = 0; by < gy; ++by)
            for (int64_t bx = 0; bx < gx; ++bx)
                for (int t = 0; t < 256; ++t) {
                    const int64_t j = bx * 64 + (t & 63), i = by * 4 + (t >> 6);
                    if (i >= n || j >= n) continue;
                    c[F_SERIAL] = 1;
                    c[F_ST_U] += 5 * sz;
                    c[F_ST_RES] += sz;
                    c[dtype == T_F64 ? F_VALU_F64 : F_VALU_F32] += 5;
                }
    }
}

/* ---------------------------------------------------------------- matmul */

/* num_cu > 0: the serial chain is that of the compute unit with the most
   k-chunks when work-group w (in dispatch order) runs on unit w mod num_cu;
   0: the chain of one work-group */
static void matmul_walk(int64_t n, int num_cu, int64_t* c) {
    const int64_t g = cdiv(n, 128), nk = cdiv(n, 16);
    const int vec = n % 16 == 0;
    int64_t* unit = num_cu > 0 ? calloc((size_t)num_cu, sizeof(int64_t)) : NULL;
    c[F_LAUNCH] += 1;
    c[F_WG] += g * g;
    for (int64_t by = 0; by < g; ++by)
        for (int64_t bx = 0; bx < g; ++bx) {
            const int64_t row0 = by * 128, col0 = bx * 128;
            c[F_BAR] += 1 + nk;   /* barriers one work-item meets, once per work-group */
            {
                int64_t steps = 0;
                for (int64_t kc = 0; kc < nk; ++kc) ++steps;
                if (unit) {
                    int64_t* u = &unit[(by * g + bx) % num_cu];
                    *u += steps;
                    steps = *u;
                }
                if (steps > c[F_SERIAL]) c[F_SERIAL] = steps;
            }
            for (int t = 0; t < 256; ++t) {
                for (int64_t kc = 0; kc < nk; ++kc) {
                    const int64_t k0 = kc * 16;
                    const int64_t ar = row0 + (t >> 1), ak = k0 + 8 * (t & 1);
                    const int64_t bk = k0 + (t >> 4), bc = col0 + 8 * (t & 15);
                    for (int h = 0; h < 2; ++h) {
                        if (vec) {
                            if (ar < n) c[F_MM_AB] += 16;
                            if (bc + 4 * h < n) c[F_MM_AB] += 16;
                        } else {
                            for (int q = 0; q < 4; ++q) {
                                if (ar < n && ak + 4 * h + q < n) c[F_MM_AB] += 4;
                                if (bk < n && bc + 4 * h + q < n) c[F_MM_AB] += 4;
                            }
                        }
                    }
                    c[F_LDS] += 2 * 16 + 8 * 4;   /* chunk stores */
                    c[F_LDS] += 8 * 16;           /* operand reads */
                }
                /* output: 4 x 4 blocks of 4 consecutive columns per lane */
                const int lane = t & 63, wave = t >> 6, cl = lane & 15, gg = lane >> 4;
                for (int i = 0; i < 4; ++i) {
                    const int64_t r = row0 + (wave >> 1) * 64 + i * 16 + cl;
                    if (r >= n) continue;
                    for (int j = 0; j < 4; ++j) {
                        const int64_t col = col0 + (wave & 1) * 64 + j * 16 + 4 * gg;
                        if (vec) {
                            if (col < n) c[F_MM_C] += 16;
                        } else {
                            for (int q = 0; q < 4; ++q)
                                if (col + q < n) c[F_MM_C] += 4;
                        }
                    }
                }
            }
            for (int w = 0; w < 4; ++w) c[F_MFMA_F32] += nk * 64 * 2048;
        }
    free(unit);
}

/* ---------------------------------------------------------------- adjoint */

static int64_t clamp04(int64_t a) { return a < 0 ? 0 : a > 4 ? 4 : a; }

/* grad_D: kernel 1, work-group (m, tile row ti, tile column tj, split) multiplies
   its 128 x 128 tile over the split's elements in chunks of 16 (thread t
   stages element t/16 of a chunk, nodes 8(t%16) .. +7 of its g and u rows,
   four at a time); kernel 2 sums the partials of every entry in groups of 16
   splits; kernel 3 sums the group sums.  The split plan (one round of
   resident work-groups, at most one split per 256 elements, splits a
   multiple of 16 elements long) is the documented schedule. */
static int bwdd_walk(int dtype, int64_t E, int n, int M, int per_cu, int num_cu, int64_t* c) {
    const int64_t sz = dtype == T_F64 ? 8 : 4;
    const int V = (int)(16 / sz);
    const int64_t count = (int64_t)M * n * n;
    const int fl = sz == 8 ? F_VALU_F64 : F_VALU_F32;
    if (per_cu < 1 || num_cu < 1) return 1;
    if (E == 0) {
        c[F_LAUNCH] += 1;
        c[F_WG] += cdiv(count, 256);
        for (int64_t idx = 0; idx < count; ++idx) c[F_OUT_UNAL] += sz;
        return 0;
    }
    const int ntile = (int)cdiv(n, 128);
    const int64_t tiles = (int64_t)M * ntile * ntile;
    int64_t ns = maxi(1, (int64_t)per_cu * num_cu / tiles);
    ns = mini(ns, maxi(1, cdiv(E, 256)));
    const int64_t len = cdiv(cdiv(E, ns), 16) * 16;
    const int64_t nsplit = maxi(1, cdiv(E, len)), ngroups = cdiv(nsplit, 16);
    const int tag = n % V == 0 ? F_U : F_U_UNAL;
    c[F_LAUNCH] += 3;
    int64_t serial = 0;
    for (int m = 0; m < M; ++m)
        for (int ti = 0; ti < ntile; ++ti)
            for (int tj = 0; tj < ntile; ++tj)
                for (int64_t sp = 0; sp < nsplit; ++sp) {
                    const int i0 = ti * 128, j0 = tj * 128;
                    const int64_t e_lo = sp * len, e_hi = mini(E, e_lo + len);
                    const int64_t nchunk = e_hi > e_lo ? cdiv(e_hi - e_lo, 16) : 0;
                    c[F_WG] += 1;
                    c[F_BAR] += 1 + nchunk;
                    if (nchunk > serial) serial = nchunk;
                    for (int t = 0; t < 256; ++t) {
                        const int el = t >> 4, xs = (t & 15) * 8;
                        for (int64_t kc = 0; kc < nchunk; ++kc) {
                            const int64_t e = e_lo + kc * 16 + el;
                            if (e < e_hi)
                                for (int h = 0; h < 2; ++h) {
                                    c[tag] += sz * clamp04(n - (i0 + xs + 4 * h));   /* g row */
                                    c[tag] += sz * clamp04(n - (j0 + xs + 4 * h));   /* u row */
                                }
                            c[F_LDS] += 2 * 8 * sz;   /* the chunk's two rows into LDS */
                        }
                    }
                    for (int w = 0; w < 4; ++w)
                        for (int64_t kc = 0; kc < nchunk; ++kc) {
                            c[F_LDS] += 64 * 32 * sz;     /* 16 g and 16 u values per lane */
                            for (int k = 0; k < 64; ++k) c[sz == 8 ? F_MFMA_F64 : F_MFMA_F32] += 2048;
                        }
                    for (int t = 0; t < 256; ++t) {
                        const int lane = t & 63, wave = t >> 6, wr = wave >> 1, wc = wave & 1;
                        const int cc = lane & 15, g = lane >> 4;
                        for (int pi = 0; pi < 4; ++pi)
                            for (int qj = 0; qj < 4; ++qj)
                                for (int r = 0; r < 4; ++r) {
                                    const int row = sz == 8 ? g + 4 * r : 4 * g + r;
                                    const int i = i0 + wr * 64 + pi * 16 + row;
                                    const int j = j0 + wc * 64 + qj * 16 + cc;
                                    if (i < n && j < n) c[F_WS_ST] += sz;
                                }
                    }
                }
    c[F_WG] += cdiv(count, 256) * ngroups + cdiv(count, 256);
    for (int64_t idx = 0; idx < count; ++idx) {
        for (int64_t y = 0; y < ngroups; ++y) {
            for (int64_t k = 16 * y; k < mini(nsplit, 16 * y + 16); ++k) {
                c[F_WS_LD] += sz;
                c[fl] += 1;
            }
            c[F_WS_ST] += sz;
        }
        for (int64_t y = 0; y < ngroups; ++y) {
            c[F_WS_LD] += sz;
            c[fl] += 1;
        }
        c[F_OUT_UNAL] += sz;
    }
    c[F_SERIAL] += serial;
    return 0;
}

/* grad_u as a GEMM (FP32): block b sits on XCD b % 8 and takes element tile
   (b / 8 / ntile_j) * 8 + b % 8 and output-node tile (b / 8) % ntile_j; the
   contraction over (m, i) runs in chunks of 16 nodes of one operator (thread t
   stages operator rows t/32 and t/32 + 8 at output nodes 4(t%32) .. +3, and
   elements t/4 and t/4 + 64 at contraction nodes 4(t%4) .. +3). */
static void bwdu_gemm_walk(int64_t E, int n, int M, int64_t* c) {
    const int64_t ntile_e = cdiv(E, 128), ntile_j = cdiv(n, 128);
    const int64_t blocks = cdiv(ntile_e, 8) * 8 * ntile_j;
    const int kpm = (int)cdiv(n, 16);
    const int nchunk = M * kpm;
    int any = 0;
    c[F_LAUNCH] += 1;
    c[F_WG] += blocks;
    for (int64_t b = 0; b < blocks; ++b) {
        const int64_t xcd = b & 7, kb = b >> 3;
        const int64_t te = (kb / ntile_j) * 8 + xcd;
        if (te >= ntile_e) continue;
        any = 1;
        const int j0 = (int)(kb % ntile_j) * 128;
        const int64_t e0 = te * 128;
        const int gtag = j0 > 0 ? F_U_L2 : n % 4 == 0 ? F_U : F_U_UNAL;
        const int otag = n % 4 == 0 ? F_OUT : F_OUT_UNAL;
        c[F_BAR] += 1 + nchunk;
        for (int t = 0; t < 256; ++t) {
            const int ka = t >> 5, ja = (t & 31) * 4, eb = t >> 2, kq = (t & 3) * 4;
            for (int kc = 0; kc < nchunk; ++kc) {
                const int i0 = (kc % kpm) * 16;
                for (int h = 0; h < 2; ++h) {
                    const int i = i0 + ka + 8 * h, j = j0 + ja;
                    if (i < n) c[F_D] += 4 * clamp04(n - j);
                    const int64_t e = e0 + eb + 64 * h;
                    if (e < E) c[gtag] += 4 * clamp04(n - (i0 + kq));
                }
                c[F_LDS] += 4 * 16;   /* two operator and two element vectors into LDS */
            }
        }
        for (int w = 0; w < 4; ++w)
            for (int kc = 0; kc < nchunk; ++kc) {
                c[F_LDS] += 64 * (16 * 4 + 4 * 16);   /* operand reads */
                for (int k = 0; k < 64; ++k) c[F_MFMA_F32] += 2048;
            }
        for (int t = 0; t < 256; ++t) {
            const int lane = t & 63, wave = t >> 6, wm = wave >> 1, wn = wave & 1;
            const int cc = lane & 15, g = lane >> 4;
            for (int q = 0; q < 4; ++q) {
                const int64_t e = e0 + wn * 64 + q * 16 + cc;
                if (e >= E) continue;
                for (int p = 0; p < 4; ++p) {
                    const int j = j0 + wm * 64 + p * 16 + 4 * g;
                    if (j + 4 <= n) {
                        c[otag] += 16;
                    } else {
                        for (int r = 0; r < 3; ++r)
                            if (j + r < n) c[otag] += 4;
                    }
                }
            }
        }
    }
    if (any) c[F_SERIAL] += nchunk;
}

/* grad_u: the GEMM for FP32 rows of 97 nodes or more (flags bit 4 set by the
   resolver), else the contraction kernel with the operator transposed: the
   nmat slabs of g as segments of one launch where such an instance exists
   (nmat <= 3 and nmat * KQ * size <= 768 bytes of fragments), else one
   launch per operator, the later ones adding to grad_u. */
static int bwdu_walk(int dtype, int64_t E, int n, int M, int epw, int waves, int per_cu, int d_panels,
                     int flags, int num_cu, int64_t* c) {
    const int64_t sz = dtype == T_F64 ? 8 : 4;
    if (flags & 4) {
        if (sz != 4 || n < 97) return 1;
        bwdu_gemm_walk(E, n, M, c);
        return 0;
    }
    if (epw != 16) return 1;
    const int KQ = kq_of(n);
    if (KQ < 0) return 1;
    const int one = M <= 3 && (M == 1 || M * KQ * sz <= 768);
    if (one) return dg_walk(dtype, E, n, M, 1, 16, waves, per_cu, d_panels, 0, num_cu, 0, 0, c);
    for (int m = 0; m < M; ++m)
        if (dg_walk(dtype, E, n, 1, 1, 16, waves, per_cu, d_panels, 0, num_cu, 0, m > 0, c)) return 1;
    return 0;
}

/* ---------------------------------------------------------------- quantiser */

/* dgdiff_quantize.  Rows of at most 1024 values: the short-row kernel (lane
   l holds 4-value vectors 4(l + 64k), k < NV; four rows per wave and step,
   rows r0, r0 + W, r0 + 2W, r0 + 3W for W launched waves); longer rows: one
   wave per row, value by value (FP8 reads the row twice: maximum, then
   encode); FP8 with one scale for the whole array: clear, grid-wide
   maximum, encode (16-byte vectors while they fit, then the tail value by
   value), final.  BF16 without per-row scales writes its single scale
   (1) in a launch of its own.  Inverse scales are always requested. */
static int quant_walk(int dtype, int64_t rows, int64_t cols, int per_row, int64_t* c) {
    const int fp8 = dtype == T_FP8;
    const int64_t esz = fp8 ? 1 : 2;
    if (dtype != T_FP8 && dtype != T_BF16) return 1;
    if (rows == 0 || cols == 0) return 0;
    if (!per_row && fp8) {
        const int64_t N = rows * cols;
        const int64_t blocks = maxi(1, mini(cdiv(N, 1024), 1024)), T = blocks * 256;
        const int64_t nv = N / 4;
        c[F_LAUNCH] += 4;
        c[F_WG] += 1 + blocks + blocks + 1;
        c[F_WS_ST] += 4;                                   /* clear the maximum */
        for (int pass = 0; pass < 2; ++pass) {             /* maximum, encode */
            if (pass == 0)
                for (int64_t b = 0; b < blocks; ++b) {
                    c[F_LDS] += 4 * 4 + 4 * 4;                 /* four wave maxima stored, read once */
                    c[F_WS_ST] += 4;                           /* one atomic maximum per work-group */
                    c[F_BAR] += 1;
                }
            for (int64_t w = 0; w < T / 64; ++w) {
                if (pass == 1) c[F_WS_LD] += 4;                /* the maximum, wave-uniform */
                /* the wave's vector-loop trips (its first lane has the most) */
                for (int64_t v = 64 * w; v < nv; v += T) c[F_WAVE_TILES] += 1;
            }
            for (int64_t gid = 0; gid < T; ++gid) {
                for (int64_t v = gid; v < nv; v += T) {
                    c[F_U] += 16;
                    if (pass) {
                        c[F_VALU_F32] += 4;
                        c[F_OUT] += 4;
                    }
                }
                for (int64_t i = 4 * nv + gid; i < N; i += T) {
                    c[F_U_UNAL] += 4;
                    if (pass) {
                        c[F_VALU_F32] += 1;
                        c[F_OUT_UNAL] += 1;
                    }
                }
            }
        }
        c[F_WS_LD] += 4;                                   /* final: read the maximum ... */
        c[F_OUT_UNAL] += 4;                                /* ... write 1/s */
        c[F_SERIAL] += cdiv(nv, T);
        return 0;
    }
    int64_t serial = 0;
    if (cols <= 1024) {
        const int NV = cols <= 256 ? 1 : cols <= 512 ? 2 : 4;
        /* lanes per row: 64, or for rows of up to 256 values the smallest
           power of two SW with 4 SW >= cols; a slot is 64 / SW rows */
        int SW = 64;
        if (NV == 1)
            while (SW > 1 && 4 * (SW / 2) >= cols) SW /= 2;
        const int RPW = 64 / SW;
        const int64_t nslots = cdiv(rows, RPW);
        const int64_t waves = mini(cdiv(nslots, 4), fp8 ? 65536 : 262144);
        const int64_t blocks = cdiv(waves, 4), W = blocks * 4;
        const int vec = cols % 4 == 0;
        c[F_LAUNCH] += 1;
        c[F_WG] += blocks;
        for (int64_t w = 0; w < W; ++w) {
            int64_t steps = 0;
            for (int64_t b0 = w; b0 < nslots; b0 += 4 * W) {
                ++steps;
                c[F_WAVE_TILES] += 1;   /* one wave-step: four slots in flight */
                for (int j = 0; j < 4; ++j) {
                    for (int lane = 0; lane < 64; ++lane) {
                        const int64_t r = (b0 + j * W) * RPW + lane / SW;
                        const int t = lane % SW;
                        if (r >= rows) continue;
                        for (int k = 0; k < NV; ++k) {
                            const int64_t avail = cols - 4 * (t + 64 * k);
                            if (avail >= 4) c[vec ? F_U : F_U_UNAL] += 16;
                            else if (avail > 0) c[vec ? F_U : F_U_UNAL] += 4 * avail;
                            if (avail <= 0) continue;
                            if (fp8) c[F_VALU_F32] += 4;
                            c[vec ? F_OUT : F_OUT_UNAL] += (avail >= 4 ? 4 : avail) * esz;
                        }
                        if (per_row && t == 0) c[F_OUT_UNAL] += 4;
                    }
                }
            }
            if (steps > serial) serial = steps;
        }
    } else {
        const int64_t waves = mini(rows, 65536);
        const int64_t blocks = cdiv(waves, 4), W = blocks * 4;
        c[F_LAUNCH] += 1;
        c[F_WG] += blocks;
        for (int64_t w = 0; w < W; ++w) {
            int64_t steps = 0;
            for (int64_t r = w; r < rows; r += W) {
                ++steps;
                c[F_WAVE_TILES] += 1;   /* one wave-step: one row */
                for (int lane = 0; lane < 64; ++lane) {
                    for (int64_t cc = lane; cc < cols; cc += 64) {
                        c[F_U_UNAL] += 4;
                        if (fp8) {   /* encode pass */
                            c[F_U_UNAL] += 4;
                            c[F_VALU_F32] += 1;
                        }
                        c[F_OUT_UNAL] += esz;
                    }
                }
                if (per_row) c[F_OUT_UNAL] += 4;
            }
            if (steps > serial) serial = steps;
        }
    }
    if (!per_row) {   /* BF16's single scale */
        c[F_LAUNCH] += 1;
        c[F_WG] += 1;
        c[F_OUT_UNAL] += 4;
    }
    c[F_SERIAL] += serial;
    return 0;
}

/* ---------------------------------------------------------------- batched */

/* One order's share of the batched launch: G work-groups of 4 waves; element
   ids and offsets (8 + 8 bytes) loaded by every lane that uses them. */
static int batched_walk(int64_t cnt, int n, int M, int epw, int ppg_in, int per_cu, int flags, int64_t G,
                        int64_t* c) {
    if (G < 1 || M != 3) return 1;
    c[F_LAUNCH] += 1;
    c[F_WG] += G;
    if (cnt == 0) return 0;
    if (flags & 4) {
        /* GEMM tiles: pool x holds element blocks eb = x (mod 8), each with
           every row block of the 3n stacked operator rows */
        const int64_t R = (int64_t)M * n, RB = cdiv(R, 128), EB = cdiv(cnt, 128), nk = cdiv(n, 16);
        for (int x = 0; x < 8; ++x) {
            const int64_t nt = EB > x ? cdiv(EB - x, 8) * RB : 0;
            for (int64_t t = 0; t < nt; ++t) {
                const int64_t eb = x + 8 * (t / RB), rb = t % RB;
                const int64_t e0 = eb * 128, r0 = rb * 128;
                c[F_BAR] += 2 + 1 + nk;   /* the claim; after the first chunk; one per chunk */
                c[F_LDS] += 8 + 256 * 8;  /* the claimed index: thread 0 stores it, every thread reads it */
                for (int tid = 0; tid < 256; ++tid) {
                    const int ar = tid >> 1, ah = (tid & 1) * 8, be = tid >> 2, bq = (tid & 3) * 4;
                    const int a_ok = r0 + ar < R;
                    int b_ok[2];
                    for (int h = 0; h < 2; ++h) {
                        b_ok[h] = e0 + be + 64 * h < cnt;
                        if (b_ok[h]) c[F_IDX] += 16;
                    }
                    for (int64_t kc = 0; kc < nk; ++kc) {
                        const int64_t k0 = kc * 16;
                        for (int h = 0; h < 2; ++h)
                            if (a_ok) c[F_D] += 4 * clamp04(n - (k0 + ah + 4 * h));
                        for (int h = 0; h < 2; ++h)
                            if (b_ok[h]) c[rb == 0 ? F_U_UNAL : F_U_L2] += 4 * clamp04(n - k0 - bq);
                        c[F_LDS] += 4 * 16;
                    }
                }
                for (int w = 0; w < 4; ++w)
                    for (int64_t kc = 0; kc < nk; ++kc) {
                        c[F_LDS] += 64 * (4 * 16 + 4 * 16);
                        for (int k = 0; k < 64; ++k) c[F_MFMA_F32] += 2048;
                    }
                for (int tid = 0; tid < 256; ++tid) {
                    const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
                    const int cc = lane & 15, g = lane >> 4;
                    for (int tn = 0; tn < 4; ++tn) {
                        const int64_t kpos = e0 + wn * 64 + tn * 16 + cc;
                        if (kpos >= cnt) continue;
                        c[F_IDX] += 16;
                        for (int tm = 0; tm < 4; ++tm) {
                            const int64_t row = r0 + wm * 64 + tm * 16 + 4 * g;
                            if (row >= R) continue;
                            const int64_t i = row % n;
                            if (i + 4 <= n) {
                                c[F_OUT_UNAL] += 16;
                            } else {
                                for (int r = 0; r < 4; ++r) {
                                    if (row + r >= R) break;
                                    c[F_OUT_UNAL] += 4;
                                }
                            }
                        }
                    }
                }
            }
        }
        c[F_SERIAL] += nk;
        return 0;
    }
    if (epw == 256) {
        /* one element per thread (nunit 8): block lb sweeps 256-element blocks
           lb, lb + G, ...; operator entries are wave-uniform loads */
        if (n != 8) return 1;
        int64_t serial = 0;
        for (int64_t lb = 0; lb < G; ++lb) {
            int64_t steps = 0;
            for (int64_t blk = lb; blk * 256 < cnt; blk += G) {
                ++steps;
                for (int w = 0; w < 4; ++w) {
                    int any = 0;
                    for (int lane = 0; lane < 64; ++lane) {
                        const int64_t k = blk * 256 + w * 64 + lane;
                        if (k >= cnt) continue;
                        any = 1;
                        c[F_IDX] += 16;
                        for (int v = 0; v < 2; ++v) c[F_U_UNAL] += 16;
                        for (int m = 0; m < 3; ++m) {
                            for (int i = 0; i < 8; ++i)
                                for (int j = 0; j < 8; ++j) c[F_VALU_F32] += 2;
                            for (int v = 0; v < 2; ++v) c[F_OUT_UNAL] += 16;
                        }
                    }
                    if (any) c[F_D] += 3 * 8 * 8 * 4;
                }
            }
            if (steps > serial) serial = steps;
        }
        c[F_SERIAL] += serial;
        return 0;
    }
    /* resident operator panels (elems_per_wave 16 or 32) */
    const int cb = epw / 16;
    if (cb != 1 && cb != 2) return 1;
    const int KQ = kq_of(n);
    if (KQ < 0) return 1;
    const int KP = 4 * KQ;
    const int mblk = (int)cdiv(n, 16), P = M * mblk;
    const int ppg = (int)maxi(1, mini(ppg_in, P));
    const int NG = (int)cdiv(P, ppg);
    if (G % (8 * NG)) return 1;
    const int64_t nstreams = 8 * (G / (8 * NG));
    const int64_t ntiles = cdiv(cnt, 16LL * cb * 4);
    int64_t serial = 0, stage_max = 0;
    for (int64_t lb = 0; lb < G; ++lb) {
        const int64_t xcd = lb & 7, kb = lb >> 3;
        const int pg = (int)(kb % NG);
        const int64_t stream = (kb / NG) * 8 + xcd;
        const int p_lo = pg * ppg;
        const int np = (int)mini(ppg, P - p_lo);
        int64_t staged = 0;
        for (int64_t idx = 0; idx < (int64_t)np * 16 * KP; ++idx) {
            const int j = (int)(idx % KP), rr = (int)(idx / KP);
            const int panel = p_lo + rr / 16;
            const int i = (panel % mblk) * 16 + rr % 16;
            if (i < n && j < n) c[F_D] += 4;
            c[F_LDS] += 4;
            staged += 4;
        }
        if (staged > stage_max) stage_max = staged;
        c[F_BAR] += 1;
        int64_t steps = 0;
        for (int64_t tile = stream; tile < ntiles; tile += nstreams) {
            ++steps;
            for (int w = 0; w < 4; ++w) {
                const int64_t k0 = tile * 64 * cb + (int64_t)w * 16 * cb;
                if (k0 >= cnt) continue;
                c[F_WAVE_TILES] += 1;
                for (int q = 0; q < cb; ++q)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int cc = lane & 15, g = lane >> 4;
                        const int64_t k = k0 + q * 16 + cc;
                        if (k >= cnt) continue;
                        c[F_IDX] += 16;
                        for (int t = 0; t < KQ; t += 4)
                            c[pg ? F_U_L2 : F_U_UNAL] += 4 * clamp04(n - g * KQ - t);
                    }
                for (int pp = 0; pp < np; ++pp) {
                    const int panel = p_lo + pp;
                    const int i = (panel % mblk) * 16;
                    for (int t = 0; t < KQ; t += 4) {
                        c[F_LDS] += 64 * 16;
                        for (int s4 = 0; s4 < 4; ++s4)
                            for (int q = 0; q < cb; ++q) c[F_MFMA_F32] += 2048;
                    }
                    for (int q = 0; q < cb; ++q)
                        for (int lane = 0; lane < 64; ++lane) {
                            const int cc = lane & 15, g = lane >> 4;
                            const int64_t k = k0 + q * 16 + cc;
                            if (k < cnt && i + 4 * g < n) c[F_OUT_UNAL] += 4 * clamp04(n - i - 4 * g);
                        }
                }
            }
        }
        if (steps > serial) serial = steps;
    }
    c[F_SERIAL] += serial;
    c[F_LAT] += serial * 64 / ((int64_t)(per_cu < 1 ? 1 : per_cu) * 4);
    c[F_STAGE] += stage_max;
    return 0;
}

/* The staged low-precision body (rows of a multiple of 8 nodes, BF16 or FP8
   widened to BF16, unless flags bit 8 asks for the LDS-panel body):
   a work-group owns rb = d_panels consecutive 16-row blocks of one operator
   slab, waves x pw = rb (pw = 1 or 2 blocks per wave, held in registers);
   tiles of 16 cb elements; per thread cb 8-node element chunks and 2 cb
   16-byte result chunks per tile (fixed counts; out-of-range ones move no
   memory).  Walked: every work-group, its operator rows, and the call order
   of its loop, whose loads run two tiles ahead: load tiles 0, 1, 2, copy
   tiles 0 and 1 to LDS, multiply tile 0; then per tile k: load tile k + 3,
   write tile k, multiply tile k + 1, copy tile k + 2 (indices past the
   stream's last tile meaning that last tile). */
static int lp_staged_walk(int dtype, int64_t E, int n, int M, int epw, int waves, int per_cu, int rb,
                          int num_cu, int fused, int64_t* c) {
    const int fp8 = dtype == T_FP8;
    const int64_t eg = fp8 ? 1 : 2;          /* operator bytes per value */
    const int64_t ue = fused ? 4 : eg;       /* element data: FP32 when rounded in the kernel */
    if (fused && (dtype != T_BF16 || epw != 16)) return 1;
    const int KS = (int)cdiv(n, 32), KQ = 8 * KS;
    if (KS > 16) return 1;
    if (epw != 16 && epw != 32) return 1;
    if (waves < 1 || waves > 16 || rb < 1 || rb % waves) return 1;
    const int pw = rb / waves;
    if (pw != 1 && pw != 2) return 1;
    if (pw == 2 && KS > 8) return 1;
    const int cb = epw / 16;
    if (pw == 2 && cb == 2 && waves > 8) return 1;
    const int64_t TE = 16LL * cb, T = 64LL * waves;
    const int mblk = (int)cdiv(n, 16);
    const int nrg = (int)cdiv(mblk, rb);
    const int NG = M * nrg;
    const int nch_u = n / 8;
    /* staging limits and LDS (element buffers, result buffers, scales, dump) */
    if (TE * nch_u > T * cb || TE * mini((int64_t)rb * 16, n) / 4 > T * 2 * cb) return 1;
    {
        const int64_t upitch = TE * 16 + 16;
        const int64_t lds = 2 * 4LL * KS * upitch + 2 * TE * rb * 16 * 4 + 2 * TE * 4 + T * 16;
        if (lds > 160 * 1024) return 1;
    }
    const int64_t ntiles = cdiv(E, TE);
    const int64_t cap = maxi(1, (int64_t)per_cu * num_cu / (8LL * NG));
    const int64_t slots = maxi(1, mini(cap, cdiv(ntiles, 8)));
    const int64_t G = 8 * NG * slots, ns = 8 * slots;
    c[F_LAUNCH] += 1;
    c[F_WG] += G;
    int64_t serial = 0;
    for (int64_t b = 0; b < G; ++b) {
        const int64_t xcd = b % 8, kb = b / 8;
        const int gi = (int)(kb % NG);
        const int rg = gi % nrg;   /* slab gi / nrg: the counts do not depend on it */
        const int64_t stream = (kb / NG) * 8 + xcd;
        if (stream >= ntiles) continue;
        const int r0 = rg * rb * 16;
        const int rows_g = (int)mini((int64_t)rb * 16, n - r0);
        /* padding chunk rows of both element buffers */
        for (int64_t idx = 0; idx < 2LL * (4 * KS - nch_u) * TE; ++idx) c[F_LDS] += 16;
        /* operator rows: wave w holds blocks w pw .. w pw + pw - 1 of the group */
        int nbw[16];
        for (int w = 0; w < waves; ++w) {
            nbw[w] = 0;
            for (int q = 0; q < pw; ++q) {
                const int lb = w * pw + q;
                if (lb < rb && r0 + lb * 16 < n) nbw[w] = q + 1;
            }
            for (int lane = 0; lane < 64; ++lane) {
                const int cc = lane & 15, g = lane >> 4;
                for (int q = 0; q < nbw[w]; ++q) {
                    const int i = r0 + (w * pw + q) * 16 + cc;
                    for (int s = 0; s < KS; ++s)
                        if (i < n && g * KQ + 8 * s < n) c[F_D] += 8 * eg;
                }
            }
            if (fp8) c[F_D] += 4;   /* the slab's operator scale, one read per wave */
        }
        /* the loop's order of tile stages, writes and multiplies */
        int64_t K = 0;
        for (int64_t t = stream; t < ntiles; t += ns) ++K;
        int64_t* tiles = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * K + 4));
        if (!tiles) return 1;
        int64_t* stage_seq = tiles + K;
        K = 0;
        for (int64_t t = stream; t < ntiles; t += ns) tiles[K++] = t;
        if (K > serial) serial = K;
        /* the loads: tiles 0 .. K + 1 (past the end: the last tile) */
        int64_t nst = 0;
        for (int64_t k = 0; k < K + 2; ++k) stage_seq[nst++] = tiles[k < K ? k : K - 1];
        c[F_BAR] += K + 1;
        c[F_WAVE_TILES] += K;
        /* group 0's first load of a tile from HBM, every other from L2, with
           the element scales */
        for (int64_t q = 0; q < nst; ++q) {
            const int64_t t = stage_seq[q];
            int first = gi == 0;
            for (int64_t r = 0; r < q; ++r)
                if (stage_seq[r] == t) first = 0;
            const int64_t nel = mini(TE, E - t * TE);
            for (int64_t th = 0; th < T; ++th) {
                for (int kk = 0; kk < cb; ++kk)
                    if (th + kk * T < nel * nch_u) c[first ? F_U : F_U_L2] += 8 * ue;
                if (fp8 && th % TE < nel) c[F_U_UNAL] += 4;
            }
        }
        /* the LDS copies: tiles 0 .. K (every thread its cb chunks and a scale) */
        for (int64_t q = 0; q < K + 1; ++q)
            for (int64_t th = 0; th < T; ++th) c[F_LDS] += 16LL * cb + 4;
        /* multiplies (every tile once) and writes */
        for (int64_t k = 0; k < K; ++k) {
            const int64_t t = tiles[k];
            const int64_t nel = mini(TE, E - t * TE);
            for (int w = 0; w < waves; ++w) {
                if (nbw[w] == 0) continue;
                for (int s = 0; s < KS; ++s)
                    for (int q = 0; q < cb; ++q) {
                        c[F_LDS] += 64 * 16;
                        c[F_MFMA_BF16] += 16384LL * nbw[w];
                    }
                for (int q = 0; q < cb; ++q) {
                    c[F_LDS] += 64 * 4;                          /* element scale per lane */
                    c[F_VALU_F32] += 64 * (1 + 4 * nbw[w]);      /* scale product, de-scaling */
                    for (int lane = 0; lane < 64; ++lane)
                        for (int p = 0; p < nbw[w]; ++p)
                            if ((w * pw + p) * 16 + 4 * (lane >> 4) < rows_g) c[F_LDS] += 16;
                }
            }
            for (int64_t th = 0; th < T; ++th)
                for (int kk = 0; kk < 2 * cb; ++kk) {
                    const int64_t ch = th + kk * T;
                    c[F_LDS] += 16;
                    if (ch < nel * (rows_g / 4)) c[F_OUT] += 16;
                }
        }
        free(tiles);
    }
    c[F_SERIAL] += serial;
    c[F_LAT] += serial * 64 / ((int64_t)per_cu * waves);
    return 0;
}

/* counts[F_N] overwritten; returns 0 on success */
int orc_features(int kernel, int dtype, int64_t n0, int nunit, int nmat, int epw, int waves,
                 int per_cu, int d_panels, int flags, int num_cu, int64_t workgroups, int64_t* counts) {
    memset(counts, 0, sizeof(int64_t) * F_N);
    switch (kernel) {
        case K_DG:
            if (n0 == 0) return 0;
            if ((dtype == T_BF16 || (dtype == T_FP8 && !(flags & 2))) && nunit % 8 == 0 && !(flags & 8))
                return lp_staged_walk(dtype, n0, nunit, nmat, epw, waves, per_cu, d_panels, num_cu,
                                      (flags & 16) != 0, counts);
            if (flags & 16) return 1;   /* the fused rounding runs in the staged body only */
            return dg_walk(dtype, n0, nunit, 1, nmat, epw, waves, per_cu, d_panels, flags, num_cu, 1, 0,
                           counts);
        case K_STENCIL:
            if (n0 > 0) stencil_walk(dtype, n0, counts);
            return 0;
        case K_MATMUL:
            if (n0 > 0) matmul_walk(n0, num_cu, counts);
            return 0;
        case K_EMPTY:
            counts[F_LAUNCH] = 1;
            counts[F_WG] = n0;
            return 0;
        case K_BWD_U:
            if (n0 == 0) return 0;
            return bwdu_walk(dtype, n0, nunit, nmat, epw, waves, per_cu, d_panels, flags, num_cu, counts);
        case K_BWD_D:
            return bwdd_walk(dtype, n0, nunit, nmat, per_cu, num_cu, counts);
        case K_QUANT:
            return quant_walk(dtype, n0, nunit, nmat ? 1 : 0, counts);
        case K_BATCHED:
            return batched_walk(n0, nunit, nmat, epw, d_panels, per_cu, flags, workgroups, counts);
        case K_BATCHED_POOL:
            /* each work-group: one barrier before the pool, then per pool of the
               eight the claim that finds it drained (two barriers) */
            for (int64_t b = 0; b < n0; ++b) {
                counts[F_BAR] += 1;
                for (int x = 0; x < 8; ++x) {
                    counts[F_BAR] += 2;
                    counts[F_LDS] += 8 + 256 * 8;
                }
            }
            return 0;
    }
    return 1;
}

/* ---------------------------------------------------------------- measurement kernels */

enum { UB_STREAM, UB_STRIDED, UB_FMA, UB_MFMA, UB_LDS, UB_BARRIER, UB_OVERLAP, UB_TWIN_DG, UB_TWIN_STENCIL,
       UB_TWIN_MATMUL, UB_TILE_READ };

/* a twin: the original's global accesses and schedule, no on-chip work, one
   add per loaded value */
static void twin_of(int64_t* c) {
    c[F_LDS] = c[F_BAR] = 0;
    c[F_MFMA_F64] = c[F_MFMA_F32] = c[F_MFMA_BF16] = c[F_MFMA_FP8] = 0;
    c[F_VALU_F64] = 0;
    c[F_VALU_F32] = (c[F_U] + c[F_U_L2] + c[F_D] + c[F_ST_U] + c[F_MM_AB] + c[F_U_UNAL]) / 4;
}

int orc_ubench_features(int kind, int dtype, int64_t n, int a, int b, int epw, int waves, int per_cu,
                        int d_panels, int flags, int num_cu, int64_t* c) {
    memset(c, 0, sizeof(int64_t) * F_N);
    if (n == 0) return 0;
    c[F_LAUNCH] = 1;
    switch (kind) {
        case UB_STREAM: {
            /* grid-stride over 4-float vectors, at most 8192 work-groups of 256 */
            const int64_t blocks = maxi(1, mini(cdiv(n, 256), 8192)), T = blocks * 256;
            int64_t serial = 0;
            c[F_WG] = blocks;
            for (int64_t t = 0; t < T; ++t) {
                int64_t trips = 0;
                for (int64_t v = t; v < n; v += T) {
                    ++trips;
                    for (int k = 0; k < a; ++k) c[F_UB_LD] += 16;
                    c[F_VALU_F32] += 4 * (a - 1);
                    c[F_UB_ST] += 16;
                }
                if (trips > serial) serial = trips;
            }
            c[F_SERIAL] = serial;
            return 0;
        }
        case UB_STRIDED:
            c[F_WG] = cdiv(n, 256);
            for (int64_t t = 0; t < n; ++t) {
                c[F_UB_LD_STRIDED] += 4;
                c[F_UB_ST] += 4;
            }
            c[F_SERIAL] = 1;
            return 0;
        case UB_FMA:
            c[F_WG] = n;
            for (int64_t t = 0; t < 256 * n; ++t) {
                c[F_VALU_F32] += 1 + 32;                       /* (t % 256) * 2^-8, then + v * 2^-5 */
                for (int it = 0; it < a; ++it)
                    for (int k = 0; k < 64; ++k) c[F_VALU_F32] += 2;
                c[F_VALU_F32] += 31;                           /* the sum */
                c[F_UB_ST] += 4;
            }
            c[F_SERIAL] = a;
            return 0;
        case UB_MFMA:
            c[F_WG] = n;
            for (int64_t w = 0; w < 4 * n; ++w)
                for (int it = 0; it < a; ++it)
                    for (int k = 0; k < 8; ++k) c[dtype == T_BF16 ? F_MFMA_BF16 : F_MFMA_F32] += dtype == T_BF16 ? 16384 : 2048;
            for (int64_t t = 0; t < 256 * n; ++t) {
                c[F_VALU_F32] += 7 * 4;
                c[F_UB_ST] += 16;
            }
            c[F_SERIAL] = a;
            return 0;
        case UB_LDS:
            if (b != 1 && b != 4) return 1;
            c[F_WG] = n;
            for (int64_t t = 0; t < 256 * n; ++t) {
                c[F_UB_LD] += 4 * b;
                c[F_LDS] += 4 * b;                             /* initial store */
                for (int k = 0; k < a; ++k) c[F_LDS] += 2 * 4 * b;
                c[F_LDS] += 4 * b;                             /* final load */
                c[F_UB_ST] += 4 * b;
            }
            c[F_SERIAL] = a;
            return 0;
        case UB_BARRIER:
            c[F_WG] = n;
            for (int64_t g = 0; g < n; ++g) c[F_BAR] += a;
            for (int64_t t = 0; t < 256 * n; ++t) c[F_UB_ST] += 4;
            c[F_SERIAL] = a;
            return 0;
        case UB_OVERLAP: {
            const int64_t blocks = cdiv(n, 256);
            c[F_WG] = blocks;
            for (int64_t g = 0; g < 256 * blocks; ++g) {
                if (g < n) c[F_UB_LD] += 16;
                for (int k = 0; k < a; ++k) c[F_LDS] += 16 + 16;
                if (g < n) c[F_UB_ST] += 16;
            }
            c[F_SERIAL] = a;
            return 0;
        }
        case UB_TWIN_DG:
            c[F_LAUNCH] = 0;
            if (dg_walk(T_F32, n, a, 1, b, epw, waves, per_cu, d_panels, flags, num_cu, 1, 0, c)) return 1;
            twin_of(c);
            return 0;
        case UB_TWIN_STENCIL:
            memset(c, 0, sizeof(int64_t) * F_N);
            stencil_walk(T_F32, n, c);
            twin_of(c);
            return 0;
        case UB_TILE_READ:
            /* 16 x 16 work-groups over the n x n array, n/16 trips per thread */
            if (n % 16 || (a != 0 && a != 1)) return 1;
            c[F_WG] = (n / 16) * (n / 16);
            for (int64_t g1 = 0; g1 < n / 16; ++g1)
                for (int64_t g0 = 0; g0 < n / 16; ++g0)
                    for (int t = 0; t < 256; ++t) {
                        for (int64_t k = 0; k < n / 16; ++k) {
                            c[a ? F_UB_LD_STRIDED : F_UB_LD] += 4;
                            c[F_VALU_F32] += 1;
                        }
                        c[F_UB_ST] += 4;
                    }
            c[F_SERIAL] = n / 16;
            return 0;
        case UB_TWIN_MATMUL:
            memset(c, 0, sizeof(int64_t) * F_N);
            matmul_walk(n, num_cu, c);
            twin_of(c);
            return 0;
    }
    return 1;
}

/* The paper's worked example of point counting: the number of integer points
   (i, j) with p <= i < n and p <= j < i + 1, by enumeration. */
int64_t orc_count_triangle(int64_t p, int64_t n) {
    int64_t cnt = 0;
    for (int64_t i = p; i < n; ++i)
        for (int64_t j = p; j < i + 1; ++j) ++cnt;
    return cnt;
}

/* ------------------------------------------------------- program variants */

/* The variant kernels' schedules walked work-group by work-group, work-item
   by work-item and loop trip by loop trip.  Global accesses add the bytes of
   the work-item that issues them; vector-ALU and LDS statements add 64 lanes'
   worth once per wave, taken by the first work-item of the wave that executes
   the statement; barriers are taken by work-item 0 of each work-group (per
   work-item, times work-groups).  Slots in the order of the library's
   variant feature interface. */
enum { V_MM_PF, V_MM_NOPF, V_DG_NOPF, V_DG_PFU, V_DG_PFDM, V_DG_PFDMT, V_FD16, V_FD18 };
enum { G_LAUNCH, G_WG, G_BAR, G_VALU, G_LDS, G_UB_LD, G_UB_ST, G_UB_LD_STRIDED, G_MM_PF_A, G_MM_PF_B,
       G_MM_NOPF_A, G_MM_NOPF_B, G_MM_C, G_DG_NOPF_U, G_DG_DM, G_DG_UPF_U, G_DG_DMPF_U, G_DG_DMPF_DM,
       G_DG_DMPFT_U, G_DG_NOPF_RES, G_DG_UPF_RES, G_DG_DMPF_RES, G_DG_DMPFT_RES, G_FD16_U, G_FD16_RES,
       G_FD18_U, G_FD18_RES, G_N };

int orc_variant_features(int kind, int64_t n, int nunit, int nmat, int twin, int keep, int64_t* c) {
    memset(c, 0, sizeof(int64_t) * G_N);
    if (n < 0 || (twin != 0 && twin != 1) || keep < 0 || keep > 7 || (!twin && keep)) return 1;
    const int in0 = twin ? (keep & 1) != 0 : 1, in1 = twin ? (keep & 2) != 0 : 1;
    const int out = twin ? (keep & 4) != 0 : 1;
    const int fd = kind == V_FD16 || kind == V_FD18;
    const int L = kind == V_FD18 ? 18 : 16, B = L - 2, T = L * L;
    int64_t gx, gy;
    if (kind == V_MM_PF || kind == V_MM_NOPF) {
        if (n % 16) return 1;
        gx = gy = n / 16;
    } else if (fd) {
        if (twin && in1) return 1;
        gx = gy = cdiv(n, B);
    } else if (kind >= V_DG_NOPF && kind <= V_DG_PFDMT) {
        if (nunit < 16 || nunit > 512 || nunit % 16 || nmat < 1 || nmat > 8) return 1;
        gx = cdiv(n, 16);
        gy = nunit / 16;
    } else {
        return 1;
    }
    if (gx * gy == 0) return 0;
    c[G_LAUNCH] = 1;
    c[G_WG] = gx * gy;
    const int u_slot = kind == V_DG_NOPF ? G_DG_NOPF_U : kind == V_DG_PFU ? G_DG_UPF_U
                     : kind == V_DG_PFDM ? G_DG_DMPF_U : G_DG_DMPFT_U;
    const int res_slot = kind == V_DG_NOPF ? G_DG_NOPF_RES : kind == V_DG_PFU ? G_DG_UPF_RES
                       : kind == V_DG_PFDM ? G_DG_DMPF_RES : G_DG_DMPFT_RES;
    for (int64_t b1 = 0; b1 < gy; ++b1)
        for (int64_t b0 = 0; b0 < gx; ++b0) {
            /* first computing work-item of each wave (the stencils' inner part) */
            int first_inner[6] = {-1, -1, -1, -1, -1, -1};
            for (int t = T - 1; t >= 0; --t)
                if (t % L < B && t / L < B) first_inner[t / 64] = t;
            for (int t = 0; t < T; ++t) {
                const int l0 = t % L, l1 = t / L;
                const int lead = t % 64 == 0;     /* first work-item of its wave */
                const int bar = t == 0;
                switch (kind) {
                    case V_MM_PF:
                        for (int64_t ko = 0; ko < n / 16; ++ko) {
                            if (!twin) {
                                if (bar) c[G_BAR] += 2;
                                c[G_MM_PF_A] += 4;
                                c[G_MM_PF_B] += 4;
                                if (lead) c[G_LDS] += 2 * 256;
                                for (int ki = 0; ki < 16; ++ki)
                                    if (lead) {
                                        c[G_LDS] += 2 * 256;
                                        c[G_VALU] += 2 * 64;
                                    }
                            } else {
                                if (in0) { c[G_MM_PF_A] += 4; if (lead) c[G_VALU] += 64; }
                                if (in1) { c[G_MM_PF_B] += 4; if (lead) c[G_VALU] += 64; }
                            }
                        }
                        if (out) c[G_MM_C] += 4; else c[G_UB_ST] += 4;
                        break;
                    case V_MM_NOPF:
                        for (int64_t k = 0; k < n; ++k) {
                            if (!twin) {
                                c[G_MM_NOPF_A] += 4;
                                c[G_MM_NOPF_B] += 4;
                                if (lead) c[G_VALU] += 2 * 64;
                            } else {
                                if (in0) { c[G_MM_NOPF_A] += 4; if (lead) c[G_VALU] += 64; }
                                if (in1) { c[G_MM_NOPF_B] += 4; if (lead) c[G_VALU] += 64; }
                            }
                        }
                        if (out) c[G_MM_C] += 4; else c[G_UB_ST] += 4;
                        break;
                    case V_DG_NOPF: {
                        const int valid = 16 * b0 + l0 < n;
                        for (int m = 0; m < nmat; ++m) {
                            for (int j = 0; j < nunit; ++j) {
                                if (!twin) {
                                    c[G_DG_DM] += 4;
                                    c[u_slot] += 4;
                                    if (lead) c[G_VALU] += 2 * 64;
                                } else {
                                    if (in1) { c[G_DG_DM] += 4; if (lead) c[G_VALU] += 64; }
                                    if (in0) { c[u_slot] += 4; if (lead) c[G_VALU] += 64; }
                                }
                            }
                            if (out && valid) c[res_slot] += 4;
                        }
                        if (!out) c[G_UB_ST] += 4;
                        break;
                    }
                    case V_DG_PFU: {
                        const int valid = 16 * b0 + l0 < n;
                        for (int jo = 0; jo < nunit / 16; ++jo) {
                            if (!twin) {
                                if (bar) c[G_BAR] += 2;
                                c[u_slot] += 4;
                                if (lead) c[G_LDS] += 256;
                            } else if (in0) {
                                c[u_slot] += 4;
                                if (lead) c[G_VALU] += 64;
                            }
                            for (int ji = 0; ji < 16; ++ji) {
                                if (!twin && lead) c[G_LDS] += 256;
                                for (int m = 0; m < nmat; ++m) {
                                    if (!twin) {
                                        c[G_DG_DM] += 4;
                                        if (lead) c[G_VALU] += 2 * 64;
                                    } else if (in1) {
                                        c[G_DG_DM] += 4;
                                        if (lead) c[G_VALU] += 64;
                                    }
                                }
                            }
                        }
                        if (out && valid) c[res_slot] += 4 * nmat;
                        if (!out) c[G_UB_ST] += 4;
                        break;
                    }
                    case V_DG_PFDM:
                    case V_DG_PFDMT: {
                        const int valid = 16 * b0 + l0 < n;
                        for (int m = 0; m < nmat; ++m) {
                            for (int jo = 0; jo < nunit / 16; ++jo) {
                                if (!twin) {
                                    if (bar) c[G_BAR] += 2;
                                    c[G_DG_DMPF_DM] += 4;
                                    if (lead) c[G_LDS] += 256;
                                    for (int ji = 0; ji < 16; ++ji) {
                                        c[u_slot] += 4;
                                        if (lead) {
                                            c[G_LDS] += 256;
                                            c[G_VALU] += 2 * 64;
                                        }
                                    }
                                } else {
                                    if (in1) { c[G_DG_DMPF_DM] += 4; if (lead) c[G_VALU] += 64; }
                                    if (in0)
                                        for (int ji = 0; ji < 16; ++ji) {
                                            c[u_slot] += 4;
                                            if (lead) c[G_VALU] += 64;
                                        }
                                }
                            }
                            if (out && valid) c[res_slot] += 4;
                        }
                        if (!out) c[G_UB_ST] += 4;
                        break;
                    }
                    case V_FD16:
                    case V_FD18: {
                        const int inner = l0 < B && l1 < B;
                        const int in_range = inner && B * b1 + l1 < n && B * b0 + l0 < n;
                        const int u_fd = kind == V_FD18 ? G_FD18_U : G_FD16_U;
                        const int r_fd = kind == V_FD18 ? G_FD18_RES : G_FD16_RES;
                        if (!twin) {
                            c[u_fd] += 4;
                            if (lead) c[G_LDS] += 256;
                            if (bar) c[G_BAR] += 1;
                            if (inner && first_inner[t / 64] == t) {
                                c[G_LDS] += 5 * 256;
                                c[G_VALU] += 5 * 64;
                            }
                            if (in_range) c[r_fd] += 4;
                        } else {
                            if (in0) { c[u_fd] += 4; if (lead) c[G_VALU] += 64; }
                            if (out) { if (in_range) c[r_fd] += 4; }
                            else c[G_UB_ST] += 4;
                        }
                        break;
                    }
                }
            }
        }
    return 0;
}
