// Shared host/device helpers of libdgdiff (internal; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/dgdiff.h"

namespace dg {

// ------------------------------------------------------------------ errors

void set_error(const std::string& msg);
dg_status fail(dg_status st, const std::string& msg);
dg_status hip_fail(hipError_t err, const char* what);

#define DG_HIP_CHECK(expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return ::dg::hip_fail(_e, #expr); \
    } while (0)

// ------------------------------------------------------------------ device info

struct DeviceInfo {
    int device = -1;
    int num_cu = 0;
    int warp_size = 64;
    size_t lds_per_block = 0;
    char arch[64] = {0};
};

// Properties of the current device (cached per device id).
dg_status current_device(DeviceInfo* out);

// True if [a, a+na) and [b, b+nb) overlap (byte ranges).
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

inline size_t dtype_size(dg_dtype t) {
    switch (t) {
        case DG_F64: return 8;
        case DG_F32: return 4;
        case DG_BF16: return 2;
        case DG_FP8E4M3: return 1;
    }
    return 0;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// FP32 -> BF16 bits, round to nearest even; NaN stays NaN (made quiet),
// overflow rounds to infinity.  The quantiser and the fused BF16 staging of
// the low-precision DG body share it, so their codes are the same bits.
__device__ inline uint16_t round_bf16_bits(uint32_t b) {   // b: an FP32 bit pattern
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ inline uint16_t round_bf16(float f) { return round_bf16_bits(__builtin_bit_cast(uint32_t, f)); }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ------------------------------------------------------------------ launchers

// DG forward, FP32 or FP64 in and out (T chosen by dtype).  Arguments already
// validated; nelem > 0.
dg_status launch_dg_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit,
                               const void* D, const void* u, void* out,
                               const dg_tile* tile, hipStream_t s);

// Launch plan of the low-precision forward (shared with the feature counter).
//   staged body (staged = true): a work-group owns rb = waves x pw row blocks
//   of one operator slab (a row group; nrg of them per slab, ngroups = nmat x
//   nrg), keeps its operator rows in registers and stages element tiles of
//   16 cb elements and their result rows in LDS; ppg reports rb.
//   LDS-panel body (staged = false): ppg operator panels per work-group in LDS.
struct LpPlan {
    int fmt;       // 0 BF16, 1 FP8 native, 2 FP8 widened to BF16
    int ks, cb, waves, lds_esz;
    int mblk, panels_total, ppg, ngroups;
    int64_t ntiles, slots, grid;
    size_t panel_bytes, smem;
    bool staged;
    int pw, rb, nrg, upitch;
};
// Staged body: 8-node element chunks and 16-byte result chunks each thread
// handles per tile of 16 cb elements (its fixed number of loads and stores).
constexpr int ls_chunks_in(int cb) { return cb; }
constexpr int ls_chunks_out(int cb) { return 2 * cb; }
int lp_format(dg_dtype in_t, const dg_tile* tile);
bool lp_pair_ok(const LpPlan& P, int nunit, bool vec_out);
// aligned: D, u and out start on 16-byte boundaries (the staged body needs it)
dg_status make_lp_plan(int fmt, int nmat, int64_t nelem, int nunit, const dg_tile* tile, int per_cu,
                       int num_cu, LpPlan* P, bool aligned = true);
dg_status resolve_forward_lowp(dg_dtype in_t, int nmat, int64_t nelem, int nunit, dg_tile* tile);
dg_status resolve_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit, dg_tile* tile);

dg_status launch_dg_forward_lowp(dg_dtype in_t, int nmat, int64_t nelem, int nunit, const void* D,
                                 const void* u, void* out, const float* inv_sD,
                                 const float* inv_su, const dg_tile* tile, hipStream_t s);

size_t backward_workspace_bytes(dg_dtype t, int nmat, int64_t nelem, int nunit);
dg_status resolve_backward(dg_dtype t, int nmat, int64_t nelem, int nunit, dg_tile* tu, dg_tile* td);
dg_status launch_dg_backward(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                             const void* u, const void* g, void* grad_u, void* grad_D, void* ws,
                             size_t ws_bytes, hipStream_t s);
// No-allocation backward: grad_D's partials live in a fixed device array of
// kBackwardScratchBytes per device (see dgdiff_backward_noalloc).
constexpr size_t kBackwardScratchBytes = (size_t)24 << 20;
dg_status launch_dg_backward_noalloc(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                                     const void* u, const void* g, void* grad_u, void* grad_D,
                                     hipStream_t s);

// Launch shape of dgdiff_quantize (a pure function of the sizes; shared with
// the feature counter): kShortRows = rows of at most 1024 values in
// registers, nv 4-value vectors per lane, rows of up to 256 values packed
// 64 / sw to a wave (sw lanes each), four such slots per wave and step;
// kRows = one wave per longer row; kGlobal = FP8 with one scale for the
// whole array (init, grid-wide maximum, encode, final: four launches).
struct QuantPlan {
    enum Kind { kShortRows, kRows, kGlobal } kind;
    int nv;
    int sw;          // kShortRows: lanes per row (a power of two), 64 / sw rows per wave slot
    int64_t blocks;  // 256-thread work-groups of the main kernel(s)
    int64_t rows, cols;
};
QuantPlan quant_plan(int fp8, int64_t rows, int64_t cols, int per_row);
dg_status launch_quantize(dg_dtype to, int64_t rows, int64_t cols, int per_row, const float* x,
                          void* q, float* inv_scale, hipStream_t s);

// work = false: the work-removed twin of the vector path
dg_status launch_stencil5(dg_dtype t, int64_t n, const void* u, int64_t ld_u, void* res,
                          int64_t ld_res, hipStream_t s, bool work = true);
bool stencil5_vector_ok(dg_dtype t, int64_t n, const void* u, int64_t ld_u, const void* res,
                        int64_t ld_res);
int stencil5_rows_per_strip(int64_t n);

dg_status launch_empty(int64_t workgroups, hipStream_t s);

// Measurement kernels (ubench.hip).  The stream kernel's grid: at most this
// many 256-thread work-groups, grid-stride beyond.
constexpr int64_t kUbStreamBlocks = 8192;
dg_status launch_ubench(const dg_ubench_desc* d, const void* const* in, void* out, hipStream_t s);
dg_status check_ubench(const dg_ubench_desc* d);

// work = false: the work-removed twin (global-memory accesses only)
dg_status launch_matmul(int64_t n, const void* a, const void* b, void* c, hipStream_t s, bool work = true);
bool matmul_vector_ok(int64_t n, const void* a, const void* b, const void* c);

// Program variants (variants.hip): grid gx x gy of `threads`-wide work-groups.
struct VariantShape {
    int64_t gx, gy;
    int threads;
};
VariantShape variant_shape(const dg_variant_desc* d);
dg_status check_variant(const dg_variant_desc* d);

}  // namespace dg
