/*
 * dgdiff.h — C ABI of libdgdiff.so: the DG differentiation kernel family of
 * Stevens & Kloeckner, "A mechanism for balancing accuracy and scope in
 * cross-machine black-box GPU performance modeling" (arXiv 1904.09538), its
 * companion calibration kernels, and the paper's black-box performance model.
 *
 * Conventions for every entry point
 *   - Array pointers are DEVICE pointers unless the comment says [host].
 *   - Arrays are dense and row-major.  The caller owns every buffer; the
 *     library never allocates or frees caller memory.
 *   - Device calls are asynchronous and ordered on the given HIP stream
 *     (0 = the null stream).  A device fault surfaces at the caller's next
 *     synchronisation.
 *   - Outputs are overwritten, never accumulated, and may not overlap any
 *     input (DG_EINVAL).
 *   - No exception crosses the ABI.  On failure the status is returned and a
 *     message is available from dg_last_error() on the calling thread.
 *   - All functions are reentrant.
 */
#ifndef DGDIFF_H
#define DGDIFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dg_stream_t; /* a hipStream_t */

typedef enum {
    DG_OK = 0,
    DG_EINVAL = 1,        /* bad argument: negative size, NULL array, overlap, bad enum */
    DG_EUNSUPPORTED = 2,  /* valid but not provided: nunit > 512, nmat > 8, dtype pair */
    DG_EHIP = 3,          /* a HIP runtime call failed; see dg_last_error() */
    DG_ENOMEM = 4
} dg_status;

typedef enum {
    DG_F64 = 0,
    DG_F32 = 1,
    DG_BF16 = 2,
    DG_FP8E4M3 = 3        /* OCP OFP8 E4M3FN: bias 7, max 448, no infinities */
} dg_dtype;

/* Launch shape of the DG kernels (all fields 0 = tuned default).
     elems_per_wave  element columns owned by one wave per tile: 16, 32 or 64
                     (1, 2 or 4 16-wide MFMA column blocks; 64 only while
                     nunit <= 128 in FP32 / nunit <= 64 in FP64)
     waves           waves (64 lanes each) per work-group: 1..8
     groups_per_cu   resident work-groups per compute unit of the persistent
                     grid; 0 = the occupancy maximum
     d_panels        16-row panels of the operator stack staged in LDS at a
                     time; 0 = as many as fit the LDS budget
     flags           DG_TILE_* bits                                          */
typedef struct {
    int32_t elems_per_wave;
    int32_t waves;
    int32_t groups_per_cu;
    int32_t d_panels;
    int32_t flags;
} dg_tile;

#define DG_TILE_NT_STORE 1   /* write outputs with non-temporal (streaming) stores (a
                                forward whose operator panels all fit one work-group
                                streams them without it) */
#define DG_TILE_FP8_NATIVE 2 /* FP8 input: multiply on the native FP8 matrix instruction,
                                whose internal 32-product sums are coarser than FP32
                                (default: widen FP8 exactly to BF16 and use the BF16
                                matrix cores, with true FP32 accumulation) */
#define DG_TILE_BATCH_GEMM 4 /* batched plans: run this order on the GEMM-tiled body
                                (128 operator rows x 128 elements per work-group) */
#define DG_TILE_LP_LDS_PANELS 8 /* BF16/FP8 input: run the body with operator panels
                                   resident in LDS and results stored from the matrix
                                   registers (default where nunit % 8 == 0 and D, u,
                                   out are 16-byte aligned: the staged body, operator
                                   rows in registers, element and result tiles
                                   staged in LDS, whole output rows written with
                                   streaming stores whatever DG_TILE_NT_STORE says) */
#define DG_TILE_QUANT_U 16    /* BF16 input only: u holds FP32 values, rounded to BF16
                                (to nearest even, as dgdiff_quantize does) while the
                                staged body copies them into LDS: the result is bit for
                                bit dgdiff_quantize(u, BF16) followed by dgdiff_apply,
                                without the separate pass over u.  Needs the staged body
                                (nunit a multiple of 8, 16-byte aligned arrays, one
                                column block per tile, no DG_TILE_LP_LDS_PANELS), else
                                DG_EUNSUPPORTED; D stays BF16 */

/* Message of the last failure on the calling thread ("" if none). */
const char* dg_last_error(void);

/* DG differentiation (Section "DG Differentiation" of the paper: the kernel
   res[m,k,i] = sum_j diff_mat[m,i,j] * u[k,j] for nmatrices operators):

       out[m][e][i] = inv_sD[m] * inv_su[e] * sum_{j<nunit} D[m][i][j] * u[e][j]

   D    [nmat][nunit][nunit] of in_t   (operator stack)
   u    [nelem][nunit]       of in_t   (element-major nodal data)
   out  [nmat][nelem][nunit] of out_t  (one contiguous slab per operator)
   inv_sD [nmat], inv_su [nelem] (FP32): inverse power-of-two scales of
        quantised inputs; NULL means 1.  Required for DG_FP8E4M3 input, must
        be NULL for FP32/FP64 input.
   Supported (in_t, out_t): (F64,F64), (F32,F32), (BF16,F32), (FP8E4M3,F32).
   Products are accumulated in out_t precision (FP32 for BF16 and FP8).
   nelem == 0 returns DG_OK without a launch.  1 <= nunit <= 512,
   1 <= nmat <= 8, else DG_EUNSUPPORTED.  tile may be NULL.               */
dg_status dgdiff_apply(dg_dtype in_t, dg_dtype out_t, int32_t nmat, int64_t nelem,
                       int32_t nunit, const void* D, const void* u, void* out,
                       const float* inv_sD, const float* inv_su,
                       const dg_tile* tile, dg_stream_t stream);

/* Mixed-order DG differentiation in one persistent launch (FP32).
   Element e has order p_e in 1..7 and n_e = (p_e+1)^3 nodes, stored ragged and
   element-major: u_packed[off_e .. off_e + n_e) with off the exclusive prefix
   sum of n_e; outputs at out_packed[m * total + off_e + i], total = sum_e n_e.
   Per element the operation is the plain one with that order's operators.

   dgdiff_plan_create: order [nelem] is a HOST array; nmat must be 3.
     tiles [8] (HOST, indexed by order; NULL = choose): launch shape per order.
     Three kernel bodies serve the orders: one element per thread (order 1,
     nunit 8, by default; reported as elems_per_wave 256), resident operator
     panels with the elements streamed through (elems_per_wave 16 or 32,
     d_panels; orders 2..5 by default, and order 1 when its tile gives
     elems_per_wave), and a GEMM tiling of 128 stacked operator rows x 128
     elements (orders 6 and 7, nunit >= 343, always, and any order whose
     tile sets DG_TILE_BATCH_GEMM; its other tile fields are then ignored).
     When tiles is NULL and model_cost [PF_COUNT] (HOST, seconds per feature
     unit; a model of DG_K_BATCHED counts) is given, every candidate shape of
     every order is priced with the model as the body that runs it
     (DG_K_BATCHED counts of the share the order would have alone on the
     GPU, plus DG_K_BATCHED_POOL's for GEMM tiles) -- linear (model_group
     NULL) or the overlap form (model_group [PF_COUNT] cost groups 0/1/2,
     model_edge) -- and the cheapest is taken; the persistent grid is split
     across orders in proportion to predicted time; GEMM-body orders are drained from a shared tile pool that every
     work-group joins after its own share, which absorbs estimate errors.
     The plan owns device copies of the sorted element ids and the offsets
     and the pool's cursors: calls that use one plan must not overlap in time
     (issue them on one stream).
   dgdiff_plan_info: order p's chosen shape, element count, work-groups and
     predicted standalone time (0 without a model).
   dgdiff_apply_batched: D_sets is a HOST array of 8 DEVICE pointers,
     D_sets[p] = [3][(p+1)^3][(p+1)^3] FP32 (needed for every order present);
     u_packed [total], out_packed [3][total] FP32.                            */
typedef struct dg_plan dg_plan;
dg_status dgdiff_plan_create(int64_t nelem, const int8_t* order, int32_t nmat, const dg_tile* tiles,
                             const double* model_cost, const int32_t* model_group, double model_edge,
                             dg_plan** out);
int64_t dgdiff_plan_total_nodes(const dg_plan* plan);
dg_status dgdiff_plan_info(const dg_plan* plan, int32_t p, dg_tile* tile, int64_t* count,
                           int64_t* workgroups, double* predicted_s);
dg_status dgdiff_apply_batched(const dg_plan* plan, const void* const* D_sets, const void* u_packed,
                               void* out_packed, dg_stream_t stream);
void dgdiff_plan_destroy(dg_plan* plan);

/* Adjoint of dgdiff_apply (not part of the paper; the addition that makes
   the operator differentiable).  With g = dL/dout [nmat][nelem][nunit]:
       grad_u[e][j]    = sum_m sum_i D[m][i][j] g[m][e][i]     [nelem][nunit]
       grad_D[m][i][j] = sum_e g[m][e][i] u[e][j]               [nmat][nunit][nunit]
   t is DG_F32 or DG_F64 (all arrays of t).  Either output may be NULL (not
   computed).  grad_D is reduced over element splits into the caller's
   workspace ws (>= dgdiff_backward_workspace(...) bytes, a size that depends
   on the current device's CU count and the kernel's occupancy there; unused
   when grad_D is NULL) and then summed in a fixed order: results are
   deterministic.
   nelem == 0 gives grad_D = 0 and touches no workspace.                     */
size_t dgdiff_backward_workspace(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit);
dg_status dgdiff_backward(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit, const void* D,
                          const void* u, const void* g, void* grad_u, void* grad_D, void* ws,
                          size_t ws_bytes, dg_stream_t stream);

/* dgdiff_backward without a workspace, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc).  Same arguments, results and errors as
   dgdiff_backward minus ws/ws_bytes; it calls no allocating routine.
   grad_D's split partials live in a fixed 24 MiB device array that the
   library holds on each GPU it runs on until the process ends (so the
   element range may be split into fewer, longer pieces than dgdiff_backward
   uses: same sum in another grouping, FP32/FP64 rounding differences only).
   Limit: 2 * nmat * nunit^2 * sizeof(t) <= 24 MiB, else DG_EUNSUPPORTED
   before any launch (every FP32 shape fits; FP64 at nunit 512 needs
   nmat <= 6).  Every call on one GPU shares that GPU's array: calls that
   overlap in time on one GPU (different streams, or threads) race and give
   wrong grad_D; issue them on one stream.  Nothing in the array needs
   clearing between calls (each call overwrites what it reads).            */
dg_status dgdiff_backward_noalloc(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit,
                                  const void* D, const void* u, const void* g, void* grad_u,
                                  void* grad_D, dg_stream_t stream);

/* Quantise an FP32 [rows][cols] array for the low-precision DG path.
     to = DG_BF16:     q (uint16 [rows][cols]) = round-to-nearest-even BF16 of x;
                       inv_scale, if not NULL, is filled with 1.
     to = DG_FP8E4M3:  q (uint8 [rows][cols]) = RNE E4M3FN of x * s, with s the
                       largest power of two such that amax * s <= 448 (amax
                       over the row if per_row_scale, else over the whole
                       array; s = 1 for amax 0 or not finite; s <= 2^127;
                       NaN entries ignored for amax), magnitudes past 448
                       saturate, NaN stays NaN; inv_scale [rows] (or [1])
                       receives 1/s (required).
   Used per operator (rows = nmat, cols = nunit^2) and per element
   (rows = nelem, cols = nunit).  rows or cols == 0 is a no-op.             */
dg_status dgdiff_quantize(dg_dtype to, int64_t rows, int64_t cols, int32_t per_row_scale,
                          const float* x, void* q, float* inv_scale, dg_stream_t stream);

/* Five-point stencil (Section "Finite Differences"):
       res[i][j] = u[i][j+1] + u[i+1][j] - 4 u[i+1][j+1] + u[i+1][j+2] + u[i+2][j+1]
   for 0 <= i, j < n.
   u   [(n+2)][ld_u] of t, ld_u >= n+2 (the input grid with its one-point halo)
   res [n][ld_res]   of t, ld_res >= n
   t is DG_F32 or DG_F64.  The fast path needs FP32, n and both leading
   dimensions multiples of 4 and 16-byte aligned arrays; any other layout takes
   a slower scalar kernel with the same result.  n == 0 is a no-op.         */
dg_status stencil5_apply(dg_dtype t, int64_t n, const void* u, int64_t ld_u, void* res,
                         int64_t ld_res, dg_stream_t stream);

/* Square matrix multiplication (Section "Kernel Creation and Transformation"):
       c[i][j] = sum_k a[i][k] b[k][j],   a, b, c [n][n] row-major FP32.
   t must be DG_F32 (DG_EUNSUPPORTED otherwise).  The fast path needs n a
   multiple of 16 and 16-byte aligned arrays; other n run a masked variant
   of the same kernel.  n == 0 is a no-op.                                  */
dg_status matmul_apply(dg_dtype t, int64_t n, const void* a, const void* b, void* c,
                       dg_stream_t stream);

/* ------------------------------------------------------------------------
   Black-box performance model (Sections "Gathering Kernel Statistics",
   "Modeling Kernel Execution Time", "Computing Model Parameters" and
   "Predicting Cost").  Host only, FP64.
   ------------------------------------------------------------------------ */

/* An empty kernel (no instructions) with the given number of 256-lane
   work-groups: isolates the launch and work-group costs of the model
   (Section "Other Features").  workgroups >= 1.                            */
dg_status dg_empty_launch(int64_t workgroups, dg_stream_t stream);

typedef enum {
    DG_K_DGDIFF = 0,   /* dgdiff_apply forward (dtype = in_t) */
    DG_K_STENCIL5 = 1, /* stencil5_apply (fast path: FP32, n % 4 == 0, padded pitches) */
    DG_K_MATMUL = 2,   /* matmul_apply */
    DG_K_EMPTY = 3,    /* dg_empty_launch */
    DG_K_BWD_U = 4,    /* dgdiff_backward's grad_u step (dtype F32/F64; tile from
                          dgdiff_resolve_backward: flags DG_TILE_BATCH_GEMM = the
                          128 x 128 GEMM body, else the contraction kernel) */
    DG_K_BWD_D = 5,    /* dgdiff_backward's grad_D step: split partials and the two
                          fixed-order reductions (tile.groups_per_cu from
                          dgdiff_resolve_backward) */
    DG_K_QUANT = 6,    /* dgdiff_quantize: dtype = target (BF16/FP8), n0 = rows,
                          nunit = cols, nmat = per_row_scale (0/1) */
    DG_K_BATCHED = 7,  /* one order's share of a dgdiff_apply_batched launch: n0 = its
                          elements, nunit = (p+1)^3, nmat = 3, tile and workgroups as
                          dgdiff_plan_info reports them (elems_per_wave 256 = one
                          element per thread; DG_TILE_BATCH_GEMM = GEMM tiles) */
    DG_K_BATCHED_POOL = 8 /* the GEMM tile pool's fixed cost in a batched launch with
                          GEMM orders: n0 = the launch's work-groups */
} dg_kernel;

typedef struct {
    dg_kernel kernel;
    dg_dtype dtype;
    int64_t n0;        /* DG: nelem; stencil and matmul: n; empty: work-groups */
    int32_t nunit;     /* DG only */
    int32_t nmat;      /* DG only */
    dg_tile tile;      /* DG only: fully resolved launch shape (dgdiff_resolve_tile) */
    int32_t num_cu;    /* DG, matmul: compute units of the target device (matmul: 0
                          counts one work-group's serial chain, not the busiest unit's) */
    int64_t workgroups; /* DG_K_BATCHED: work-groups of the order's share */
} perf_kernel_desc;

/* Feature indices of perf_features_count (counts are int64, exact):          */
enum {
    PF_LAUNCH = 0,       /* kernel launches */
    PF_WORKGROUPS,       /* work-groups */
    PF_BARRIER_X_WG,     /* barriers met by one work-item x work-groups */
    PF_GLD_DG_U,         /* DG element-data 16-byte vector loads, bytes (first operator group) */
    PF_GLD_DG_U_L2,      /* DG element-data re-loads by further operator groups (L2) */
    PF_GLD_DG_D,         /* DG operator loads while staging into LDS, bytes */
    PF_GST_DG_OUT,       /* DG output 16-byte vector stores, bytes */
    PF_GLD_ST_U,         /* stencil grid loads, bytes */
    PF_GST_ST_RES,       /* stencil result stores, bytes */
    PF_GLD_MM_AB,        /* matmul operand loads, bytes */
    PF_GST_MM_C,         /* matmul result stores, bytes */
    PF_LDS_BYTES,        /* LDS bytes moved (incl. wave shuffles) */
    PF_MFMA_F64,         /* matrix-core flops executed, per input type */
    PF_MFMA_F32,
    PF_MFMA_BF16,
    PF_MFMA_FP8,
    PF_VALU_F32,         /* vector-ALU flops */
    PF_VALU_F64,
    PF_GLD_DG_U_UNAL,    /* DG element-data loads on the unaligned-row paths, bytes */
    PF_GST_DG_OUT_UNAL,  /* DG output stores of unaligned rows (scalar), bytes */
    PF_WAVE_TILES,       /* DG element tiles processed by a wave, summed over operator groups */
    PF_SERIAL_STEPS,     /* longest chain of loop iterations one work-group walks (latency) */
    PF_LAT_STEPS,        /* DG: 64 x serial steps / resident waves per SIMD (per_cu x waves / 4):
                            the tile latency left unhidden by other waves (launch configuration) */
    PF_GLD_WS,           /* partial-result (workspace) loads, bytes */
    PF_GST_WS,           /* partial-result (workspace) stores, bytes */
    PF_GLD_IDX,          /* index and offset loads (batched element lists), bytes */
    PF_GLD_UB,           /* measurement kernels: 16-byte vector loads, consecutive lanes, bytes */
    PF_GST_UB,           /* measurement kernels: stores, bytes */
    PF_GLD_UB_STRIDED,   /* measurement kernels: 4-byte loads, lanes S floats apart, bytes */
    PF_DG_OUT_W32,       /* of the DG contraction's output bytes, those written by 32-element wave */
    PF_DG_OUT_W64,       /* tiles, and by 64-element ones: a tag of the store pattern (a wider tile
                            spreads each panel's 64-byte row pieces over more rows), not extra bytes */
    PF_STAGE_CHAIN,      /* operator-staging kernels: LDS bytes one work-group stages before its first
                            element tile (the largest over the launch's work-groups), summed over
                            launches: a latency chain like PF_SERIAL_STEPS, not a volume */
    PF_COUNT
};

int32_t perf_feature_count(void);           /* PF_COUNT */
const char* perf_feature_name(int32_t k);   /* "" when out of range */

/* Exact operation counts of one launch described by d (int64 counts[PF_COUNT],
   overwritten).  Global and LDS traffic are bytes of the lanes that execute
   the access; matrix-core work is the flops of the executed instructions
   (padding included); barriers are counted per work-item and multiplied by
   the work-group count (the paper's granularity rules).  DG descriptors need
   a resolved tile (all of elems_per_wave, waves, groups_per_cu, d_panels)
   and num_cu: counts then follow the exact schedule dgdiff_apply launches
   with that tile on a device with num_cu compute units.                     */
dg_status perf_features_count(const perf_kernel_desc* d, int64_t* counts);

/* Fill the 0 fields of *tile with the launch shape dgdiff_apply would use
   for this problem on the current device (groups_per_cu from the occupancy
   of the chosen kernel; needs a GPU).                                       */
dg_status dgdiff_resolve_tile(dg_dtype in_t, int32_t nmat, int64_t nelem, int32_t nunit,
                              dg_tile* tile);

/* The launch shapes dgdiff_backward uses for this problem on the current
   device (needs a GPU): *tile_u for the grad_u step (DG_TILE_BATCH_GEMM in
   flags when it runs as the 128 x 128 GEMM), *tile_d for grad_D
   (groups_per_cu = resident work-groups per CU of the split-partial
   kernel, which sets the split count).  Either pointer may be NULL.         */
dg_status dgdiff_resolve_backward(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit,
                                  dg_tile* tile_u, dg_tile* tile_d);

/* ------------------------------------------------------------------------
   Measurement kernels (Sections "Measurement Kernel Design", "Measurement
   Kernel Sets for Evaluation" and "Measurement Workload Synthesis by Work
   Removal Transformation"): microbenchmarks that each exercise one feature
   of the model, and work-removed twins that keep a kernel's global-memory
   accesses and drop its on-chip work.  All FP32; arrays are device arrays,
   `in` a HOST array of device pointers.
     kind                n              a              b         in / out
     DG_UB_STREAM        4-float vectors inputs 1..4     -        in[0..a-1] [4n], out [4n] = sum of inputs
     DG_UB_STRIDED       threads        stride S >= 1    -        in[0] [n*S], out[t] = in[0][t*S]
     DG_UB_FMA           work-groups    loop trips       -        out [256n]: the fma recurrence's sum
     DG_UB_MFMA          work-groups    loop trips       -        out [1024n]: eight chains of products
                                                                  (dtype DG_F32 or DG_BF16 operands)
     DG_UB_LDS           work-groups    trips            1 or 4   in[0], out [256n*b]: rotated by a lanes
     DG_UB_BARRIER       work-groups    barriers         -        out [256n] = a
     DG_UB_OVERLAP       4-float vectors LDS pairs m     -        in[0], out [4n]: rotated by m lanes
     DG_UB_TWIN_DG       nelem          nunit            nmat     in[0] = D, in[1] = u, out as dgdiff_apply
                                                                  (tile: a resolved FP32 forward tile)
     DG_UB_TWIN_STENCIL  n              ld_u             ld_res   in[0] = u, out = res (vector path layout)
     DG_UB_TWIN_MATMUL   n              -                -        in[0] = a, in[1] = b, out = c
     DG_UB_TILE_READ     n (mult. of 16) pattern 0 or 1  -        in[0] [n*n], out [n*n]: the square
                                                                  matmul's tiled operand fetches of
                                                                  Section "Global Memory Access Pattern
                                                                  Features": 16x16 work-group (g0, g1),
                                                                  thread (l0, l1) reads, at trip k < n/16,
                                                                  pattern 0 (a): x[n(16 g1 + l1) + 16k + l0],
                                                                  pattern 1 (b): x[n(16k + l1) + 16 g0 + l0],
                                                                  and stores the sum at (16 g1 + l1, 16 g0 + l0)
   The twins' outputs carry no meaning beyond covering every element the
   original writes.  perf_ubench_count gives the launch's counts (as
   perf_features_count; twins count the original's global accesses, with the
   adds of the loaded values as VALU flops).                                */
typedef enum {
    DG_UB_STREAM = 0,
    DG_UB_STRIDED = 1,
    DG_UB_FMA = 2,
    DG_UB_MFMA = 3,
    DG_UB_LDS = 4,
    DG_UB_BARRIER = 5,
    DG_UB_OVERLAP = 6,
    DG_UB_TWIN_DG = 7,
    DG_UB_TWIN_STENCIL = 8,
    DG_UB_TWIN_MATMUL = 9,
    DG_UB_TILE_READ = 10
} dg_ubench;

typedef struct {
    dg_ubench kind;
    dg_dtype dtype;
    int64_t n;
    int32_t a, b;
    dg_tile tile;      /* DG_UB_TWIN_DG only */
    int32_t num_cu;    /* DG_UB_TWIN_DG only (counts) */
} dg_ubench_desc;

dg_status dg_ubench_run(const dg_ubench_desc* d, const void* const* in, void* out, dg_stream_t stream);
dg_status perf_ubench_count(const dg_ubench_desc* d, int64_t* counts);

/* ------------------------------------------------------------------------
   Program variants (Sections "Matrix Multiplication", "DG Differentiation"
   and "Finite Differences"): equivalent formulations of each evaluation
   computation that the model is asked to rank.  FP32 vector-ALU code with
   the paper's work-group shapes (16 x 16 work-items; the 18 x 18 stencil
   324), lid(0) = threadIdx.x % L, lid(1) = threadIdx.x / L, gid(0) =
   blockIdx.x, gid(1) = blockIdx.y.  All arrays row-major device FP32.
     kind            n        operation, layout and schedule
     DG_V_MM_PF      n        c = a b, a = in0, b = in1, c = out, [n][n], n a multiple
                              of 16: per 16-wide k step a 16 x 16 tile of a and one of b
                              are staged in LDS, one value per work-item
     DG_V_MM_NOPF    n        c = a b without staging or k split: each work-item walks
                              its row of a and column of b in global memory
     DG_V_DG_NOPF    nelem    res[m][k][i] = sum_j D[m][i][j] u[k][j] (Section "DG
                              Differentiation"), u = in0 [nelem][nunit], D = in1
                              [nmat][nunit][nunit], res = out [nmat][nelem][nunit];
                              work-item (k, i) = (16 gid(0) + lid(0), 16 gid(1) + lid(1)),
                              operands from global memory, loop order m, j
     DG_V_DG_PFU     nelem    as DG_V_DG_NOPF; per 16-wide j step the 16 x 16 tile of u
                              (the work-group's 16 elements) is staged in LDS, the nmat
                              sums are kept in registers (loop order j, m)
     DG_V_DG_PFDM    nelem    as DG_V_DG_NOPF; per operator and 16-wide j step the 16 x 16
                              tile of D[m] (the work-group's 16 rows) is staged in LDS
                              (loop order m, j)
     DG_V_DG_PFDMT   nelem    DG_V_DG_PFDM on transposed element data: u [nunit][nelem],
                              res [nmat][nunit][nelem] (consecutive lid(0), consecutive
                              addresses)
     DG_V_FD16       n        res[i][j] = u[i][j+1] + u[i+1][j] - 4 u[i+1][j+1] + u[i+1][j+2]
                              + u[i+2][j+1] (Section "Finite Differences"), u = in0
                              [n+2][ld_u], res = out [n][ld_res]: a 16 x 16 work-group
                              stages a 16 x 16 tile of u (one value each), 14 x 14 of its
                              work-items compute
     DG_V_FD18       n        the same with 18 x 18 work-groups (16 x 16 compute)
   DG variants: nunit a multiple of 16 in 16..512, nmat 1..8.  Loads past the
   last element (grid point) read the last one; only result stores are
   guarded.  n == 0 (nelem == 0) is a no-op.
   work_removed = 1 runs the variant's work-removed twin (Section "Measurement
   Workload Synthesis by Work Removal Transformation"): the same loops and the
   global accesses to the arrays in keep (DG_V_KEEP_* bits) only, each load
   added to one per-work-item sum, with no LDS, barrier or other arithmetic.
   With DG_V_KEEP_OUT the sum is stored where the variant stores its result;
   otherwise out is a destination of one float per work-item,
   out[(gid(1) * gx + gid(0)) * threads + threadIdx.x] (gx, work-groups and
   threads from dg_variant_shape).  Arrays a twin does not read may be NULL.
   DG_EINVAL: sizes outside the above, keep on a full variant, DG_V_KEEP_IN1 on
   a stencil, NULL arrays, or an output overlapping a read input.            */
typedef enum {
    DG_V_MM_PF = 0,
    DG_V_MM_NOPF = 1,
    DG_V_DG_NOPF = 2,
    DG_V_DG_PFU = 3,
    DG_V_DG_PFDM = 4,
    DG_V_DG_PFDMT = 5,
    DG_V_FD16 = 6,
    DG_V_FD18 = 7
} dg_variant;

#define DG_V_KEEP_IN0 1
#define DG_V_KEEP_IN1 2
#define DG_V_KEEP_OUT 4

typedef struct {
    dg_variant kind;
    int64_t n;          /* matmul, stencil: n; DG: nelem */
    int32_t nunit;      /* DG only */
    int32_t nmat;       /* DG only */
    int64_t ld_u;       /* stencil only */
    int64_t ld_res;     /* stencil only */
    int32_t work_removed;
    int32_t keep;       /* work-removed twins only */
} dg_variant_desc;

/* Work-groups (gx * gy) and work-items per work-group of the launch.       */
dg_status dg_variant_shape(const dg_variant_desc* d, int64_t* workgroups, int32_t* threads);
dg_status dg_variant_run(const dg_variant_desc* d, const void* in0, const void* in1, void* out,
                         dg_stream_t stream);

/* Features of the variant study (perf_variant_count), in the paper's
   granularities: per launch, per work-group (barriers: per work-item x
   work-groups), per wave for vector-ALU and LDS work (a wave instruction
   counts 64 lanes, whichever lanes are active), per work-item for global
   accesses (bytes of the lanes that issue them).  One global-access feature
   per access pattern of the variants (the paper's tagged patterns); the
   microbenchmark features keep the names perf_feature_name gives them.     */
enum {
    VF_LAUNCH = 0,
    VF_WORKGROUPS,
    VF_BARRIER_X_WG,
    VF_VALU_F32_SG,      /* FP32 flops (fused multiply-add 2, add 1) x 64 per wave instruction */
    VF_LDS_SG,           /* LDS bytes, 4 x 64 per wave access of one float per lane */
    VF_GLD_UB,           /* microbenchmarks: 16-byte vector loads, bytes */
    VF_GST_UB,           /* microbenchmark stores and twin destinations: stride-1 stores, bytes */
    VF_GLD_UB_STRIDED,   /* microbenchmarks: 4-byte loads, lanes S floats apart, bytes */
    VF_GLD_MM_PF_A,      /* matmul, tiled: a tile loads */
    VF_GLD_MM_PF_B,      /*                b tile loads */
    VF_GLD_MM_NOPF_A,    /* matmul, untiled: row of a */
    VF_GLD_MM_NOPF_B,    /*                  column of b */
    VF_GST_MM_C,         /* matmul result stores (both) */
    VF_GLD_DG_NOPF_U,    /* DG untiled: u[k][j] per work-item */
    VF_GLD_DG_DM,        /* DG untiled and u-staged: D[m][i][j] per work-item */
    VF_GLD_DG_UPF_U,     /* DG u-staged: u tile loads */
    VF_GLD_DG_DMPF_U,    /* DG D-staged: u[k][j] per work-item */
    VF_GLD_DG_DMPF_DM,   /* DG D-staged (both layouts): D tile loads */
    VF_GLD_DG_DMPFT_U,   /* DG D-staged, transposed: u[j][k] per work-item */
    VF_GST_DG_NOPF_RES,  /* DG result stores, one feature per variant */
    VF_GST_DG_UPF_RES,
    VF_GST_DG_DMPF_RES,
    VF_GST_DG_DMPFT_RES,
    VF_GLD_FD16_U,       /* stencil tile loads and result stores per work-group shape */
    VF_GST_FD16_RES,
    VF_GLD_FD18_U,
    VF_GST_FD18_RES,
    VF_COUNT
};

int32_t perf_variant_feature_count(void);            /* VF_COUNT */
const char* perf_variant_feature_name(int32_t k);    /* "" when out of range */
/* Exact counts of one launch of d (int64 counts[VF_COUNT], overwritten); a
   host computation that needs no GPU.                                      */
dg_status perf_variant_count(const dg_variant_desc* d, int64_t* counts);

/* Flags of the model fits.  DG_FIT_RELATIVE: minimise the relative error
   (the paper's scale_features_by_output, Section "Computing Model
   Parameters").  DG_FIT_NONNEG: keep every cost parameter >= 0 (the paper's
   interpretability criterion, Section "Assumptions and Limitations": a cost model that
   needs negative weights is not one).                                       */
#define DG_FIT_RELATIVE 1
#define DG_FIT_NONNEG 2

/* Fit a linear model t ~ F p (F [rows][cols] row-major FP64 features, t
   [rows] seconds): the p [cols] minimising ||t - F p||_2, or with
   DG_FIT_RELATIVE the relative error ||1 - diag(1/t) F p||_2.  Columns are
   equilibrated, the system is solved by an FP64 SVD (no normal equations),
   singular values below 1e-12 of the largest are dropped and the
   minimum-norm solution is returned: a rank-deficient F is not an error
   (*rank < cols).  With DG_FIT_NONNEG, when that solution has a negative
   entry, p is instead the non-negative least-squares minimiser of the same
   equilibrated system (Lawson-Hanson active set).  *resid = residual norm at
   the solution, *cond = condition number of the kept part of the
   unconstrained system.  Each output pointer except p may be NULL.
   DG_EINVAL: rows or cols <= 0, non-finite input, unknown flags, or t <= 0
   with DG_FIT_RELATIVE.                                                     */
dg_status perf_model_fit(int32_t rows, int32_t cols, const double* F, const double* t,
                         int32_t flags, double* p, double* resid, int32_t* rank, double* cond);

/* The paper's nonlinear overlap model (Sections "Modeling Operation Overlap"
   and "Models Demonstrated").  group[j] puts feature j into the overhead (0),
   global-memory (1) or on-chip (2) cost; with c_x = sum over group x of
   p_j F[k][j]:
       t_k ~ c_0 + c_1 s(c_1 - c_2) + c_2 s(c_2 - c_1),  s(x) = (tanh(edge x) + 1) / 2.
   Fitted by Levenberg-Marquardt in FP64 on the relative (DG_FIT_RELATIVE)
   or absolute residual; every step is an augmented least-squares solve by SVD
   (no normal equations).  With DG_FIT_NONNEG each step is projected onto
   p >= 0, parameters held at zero while the gradient points out of the
   orthant.  On entry a non-zero p (e.g. a linear fit; magnitudes are taken)
   and edge > 0 seed the iteration; on exit they hold the fit.  *iters =
   iterations taken.  DG_EINVAL: bad sizes, groups outside 0..2, unknown
   flags, non-finite features or t <= 0.                                     */
dg_status perf_model_fit_overlap(int32_t rows, int32_t cols, const double* F, const int32_t* group,
                                 const double* t, int32_t flags, double* p, double* edge,
                                 double* resid, int32_t* iters);
dg_status perf_model_predict_overlap(int32_t rows, int32_t cols, const double* F,
                                     const int32_t* group, const double* p, double edge,
                                     double* t_out);

/* t_out[k] = sum_j F[k][j] p[j] (Section "Predicting Cost").               */
dg_status perf_model_predict(int32_t rows, int32_t cols, const double* F, const double* p,
                             double* t_out);

#ifdef __cplusplus
}
#endif

#endif /* DGDIFF_H */
