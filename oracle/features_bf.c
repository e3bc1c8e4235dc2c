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
       F_WAVE_TILES, F_SERIAL, F_LAT, F_N };

enum { K_DG = 0, K_STENCIL = 1, K_MATMUL = 2, K_EMPTY = 3 };
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

static int dg_walk(int dtype, int64_t E, int n, int M, int epw, int waves, int per_cu, int d_panels,
                   int flags, int num_cu, int64_t* c) {
    const int lowp = dtype == T_BF16 || dtype == T_FP8;
    const int native = dtype == T_FP8 && (flags & 2);
    const int64_t sz = dtype == T_F64 ? 8 : 4;      /* FP element size */
    const int64_t eg = dtype == T_BF16 ? 2 : 1;     /* low-precision element size in HBM */
    const int64_t el = native ? 1 : 2;              /* low-precision element size in LDS */
    const int cb = epw / 16;
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
        int64_t panel_bytes = 16 * (4LL * KQ + V) * sz;
        int64_t slab = (int64_t)waves * cdiv(16LL * cb * n, V) * V * sz;
        use_slab = slab + panel_bytes <= 80 * 1024;
    }
    {
        const int64_t panel = lowp ? 16 * (32LL * KS * el + 16) : 16 * (4LL * KQ + V) * sz;
        const int64_t slab = use_slab ? (int64_t)waves * cdiv(16LL * cb * n, V) * V * sz : 0;
        if (ppg * panel + slab > 160 * 1024) return 1;
    }
    const int vec_out = n % 4 == 0;
    /* unaligned rows that come through the wave slab leave through it too */
    const int stage_out = !lowp && use_slab && !vec_out;
    /* FP32 rows of a multiple of 32 nodes in even panel groups are stored in
       panel pairs; with small fragments (KQ * cb <= 32) their element loads are
       issued a tile ahead, every lane of a wave-tile loading all its vectors
       (rows past the end read the last element) */
    const int piped = !lowp && sz == 4 && vec_in && vec_out && n % 32 == 0 && mblk % 2 == 0 &&
                      ppg % 2 == 0 && KQ * cb <= 32;

    c[F_LAUNCH] += 1;
    c[F_WG] += G;
    for (int64_t b = 0; b < G; ++b) {
        const int64_t xcd = b % 8, kb = b / 8;
        const int pg = (int)(kb % NG);
        const int64_t stream = (kb / NG) * 8 + xcd;
        const int p_lo = pg * ppg;
        const int np = (int)mini(ppg, P - p_lo);
        /* operator staging: one lane-iteration per LDS slot */
        for (int64_t idx = 0; idx < (int64_t)np * 16 * KP; ++idx) {
            const int k = (int)(idx % KP);
            const int rr = (int)(idx / KP);
            const int panel = p_lo + rr / 16;
            const int o = (panel % mblk) * 16 + rr % 16;
            if (o < n && k < n) c[F_D] += lowp ? eg : sz;
            c[F_LDS] += lowp ? el : sz;
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
                            for (int s = 0; s < KS; ++s) {
                                if (vec_in) {
                                    if (e < E && g * KQ + 8 * s < n) c[tag] += 8 * eg;
                                } else {
                                    for (int t = 0; t < 8; ++t)
                                        if (e < E && g * KQ + 8 * s + t < n) c[tag] += eg;
                                }
                            }
                        }
                } else if (piped) {
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
                    } else {
                        for (int s = 0; s < KQ; s += V) {
                            c[F_LDS] += 64 * 16;                        /* 16-byte operand read */
                            for (int t = 0; t < V; ++t)
                                for (int q = 0; q < cb; ++q) c[sz == 8 ? F_MFMA_F64 : F_MFMA_F32] += 2048;
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
                            if (vec_out) {
                                if (i < n) c[F_OUT] += 4 * osz;
                            } else {
                                for (int r = 0; r < 4; ++r)
                                    if (i + r < n) c[F_OUT_UNAL] += osz;
                            }
                        }
                }
            }
        }
        if (steps > c[F_SERIAL]) c[F_SERIAL] = steps;
    }
    /* latency left unhidden: the busiest stream's steps over resident waves
       per SIMD (per_cu work-groups of `waves` waves on 4 SIMDs), x 64 */
    c[F_LAT] = c[F_SERIAL] * 64 / ((int64_t)per_cu * waves);
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
                    /* rows i_lo .. i_hi+1 are loaded once each */
                    for (int64_t r = i_lo; r < i_hi + 2; ++r) {
                        if (active) c[F_ST_U] += 16;
                        if (active && self_halo) c[F_ST_U] += 8;
                        c[F_LDS] += 2 * 4;   /* two shuffles */
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

/* counts[F_N] overwritten; returns 0 on success */
int orc_features(int kernel, int dtype, int64_t n0, int nunit, int nmat, int epw, int waves,
                 int per_cu, int d_panels, int flags, int num_cu, int64_t* counts) {
    memset(counts, 0, sizeof(int64_t) * F_N);
    switch (kernel) {
        case K_DG:
            if (n0 == 0) return 0;
            return dg_walk(dtype, n0, nunit, nmat, epw, waves, per_cu, d_panels, flags, num_cu, counts);
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
