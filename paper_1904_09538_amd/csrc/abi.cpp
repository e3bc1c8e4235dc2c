// extern "C" entry points of libdgdiff: argument validation and dispatch.
// Every device-side step runs in the library's own HIP kernels.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace dg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

dg_status fail(dg_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

dg_status hip_fail(hipError_t err, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(err));
    return DG_EHIP;
}

dg_status current_device(DeviceInfo* out) {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = -1;
    DG_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    for (const DeviceInfo& d : cache)
        if (d.device == dev) {
            *out = d;
            return DG_OK;
        }
    hipDeviceProp_t prop;
    DG_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    DeviceInfo d;
    d.device = dev;
    d.num_cu = prop.multiProcessorCount;
    d.warp_size = prop.warpSize;
    d.lds_per_block = prop.sharedMemPerBlock;
    std::strncpy(d.arch, prop.gcnArchName, sizeof(d.arch) - 1);
    if (d.warp_size != 64) return fail(DG_EUNSUPPORTED, "device is not wave64 (gfx950 expected)");
    cache.push_back(d);
    *out = d;
    return DG_OK;
}

}  // namespace dg

using namespace dg;

namespace dg {
// Sizes of a measurement-kernel descriptor (shared by the launch and the counts).
dg_status check_ubench(const dg_ubench_desc* d) {
    if (d->n < 0) return fail(DG_EINVAL, "measurement kernel: negative size");
    switch (d->kind) {
        case DG_UB_STREAM:
            if (d->a < 1 || d->a > 4) return fail(DG_EINVAL, "stream: 1..4 inputs");
            return DG_OK;
        case DG_UB_STRIDED:
            if (d->a < 1) return fail(DG_EINVAL, "strided: stride >= 1");
            return DG_OK;
        case DG_UB_FMA:
        case DG_UB_BARRIER:
            if (d->a < 0 || d->n > INT32_MAX) return fail(DG_EINVAL, "loop trips >= 0, work-groups < 2^31");
            return DG_OK;
        case DG_UB_MFMA:
            if (d->a < 0 || d->n > INT32_MAX) return fail(DG_EINVAL, "loop trips >= 0, work-groups < 2^31");
            if (d->dtype != DG_F32 && d->dtype != DG_BF16) return fail(DG_EUNSUPPORTED, "mfma: F32 or BF16");
            return DG_OK;
        case DG_UB_LDS:
            if (d->a < 0 || (d->b != 1 && d->b != 4) || d->n > INT32_MAX)
                return fail(DG_EINVAL, "lds: trips >= 0, width 1 or 4");
            return DG_OK;
        case DG_UB_OVERLAP:
            if (d->a < 0) return fail(DG_EINVAL, "overlap: m >= 0");
            return DG_OK;
        case DG_UB_TWIN_DG:
            if (d->a < 1 || d->a > 512 || d->b < 1 || d->b > 8) return fail(DG_EUNSUPPORTED, "DG twin: sizes");
            return DG_OK;
        case DG_UB_TILE_READ:
            if (d->n % 16 || d->n > 65536 || (d->a != 0 && d->a != 1))
                return fail(DG_EINVAL, "tile read: n a multiple of 16 up to 65536, pattern 0 or 1");
            return DG_OK;
        case DG_UB_TWIN_STENCIL:
            if (d->n % 4 || d->a < d->n + 2 || d->a % 4 || d->b < d->n || d->b % 4)
                return fail(DG_EUNSUPPORTED, "stencil twin: n and leading dimensions multiples of 4");
            return DG_OK;
        case DG_UB_TWIN_MATMUL:
            return DG_OK;
    }
    return fail(DG_EINVAL, "unknown measurement kernel");
}
}  // namespace dg

// Argument checks shared by both backward entry points; *done is set when
// there is nothing to compute.
static dg_status check_backward(const char* name, dg_dtype t, int32_t nmat, int64_t nelem,
                                int32_t nunit, const void* D, const void* u, const void* g,
                                void* grad_u, void* grad_D, void* ws, size_t ws_bytes, bool* done) {
    const std::string fn(name);
    if (t != DG_F32 && t != DG_F64) return fail(DG_EUNSUPPORTED, fn + ": FP32 or FP64 only");
    if (nelem < 0 || nmat < 1 || nunit < 1) return fail(DG_EINVAL, fn + ": sizes must be positive");
    if (nmat > 8 || nunit > 512) return fail(DG_EUNSUPPORTED, fn + ": nmat <= 8 and nunit <= 512");
    if (!grad_u && !grad_D) {
        *done = true;
        return DG_OK;
    }
    if (nelem > 0 && (!g || (grad_u && !D) || (grad_D && !u)))
        return fail(DG_EINVAL, fn + ": NULL input");
    const size_t es = dtype_size(t);
    const size_t nD = (size_t)nmat * nunit * nunit * es, nu = (size_t)nelem * nunit * es;
    const size_t ng = (size_t)nmat * nelem * nunit * es;
    if (grad_u && (overlaps(grad_u, nu, D, nD) || overlaps(grad_u, nu, u, nu) ||
                   overlaps(grad_u, nu, g, ng) || overlaps(grad_u, nu, grad_D, nD) ||
                   overlaps(grad_u, nu, ws, ws_bytes)))
        return fail(DG_EINVAL, fn + ": grad_u overlaps another array");
    if (grad_D && (overlaps(grad_D, nD, D, nD) || overlaps(grad_D, nD, u, nu) ||
                   overlaps(grad_D, nD, g, ng) || overlaps(grad_D, nD, ws, ws_bytes)))
        return fail(DG_EINVAL, fn + ": grad_D overlaps another array");
    if (ws && (overlaps(ws, ws_bytes, D, nD) || overlaps(ws, ws_bytes, u, nu) ||
               overlaps(ws, ws_bytes, g, ng)))
        return fail(DG_EINVAL, fn + ": workspace overlaps an input");
    return DG_OK;
}

extern "C" {

const char* dg_last_error(void) { return g_last_error.c_str(); }

dg_status dgdiff_apply(dg_dtype in_t, dg_dtype out_t, int32_t nmat, int64_t nelem, int32_t nunit,
                       const void* D, const void* u, void* out, const float* inv_sD,
                       const float* inv_su, const dg_tile* tile, dg_stream_t stream) {
    set_error("");
    if (in_t < DG_F64 || in_t > DG_FP8E4M3 || out_t < DG_F64 || out_t > DG_FP8E4M3)
        return fail(DG_EINVAL, "dgdiff_apply: unknown dtype");
    if (nelem < 0 || nmat < 1 || nunit < 1) return fail(DG_EINVAL, "dgdiff_apply: sizes must be positive");
    if (nmat > 8 || nunit > 512) return fail(DG_EUNSUPPORTED, "dgdiff_apply: nmat <= 8 and nunit <= 512");
    const bool fp = (in_t == DG_F32 && out_t == DG_F32) || (in_t == DG_F64 && out_t == DG_F64);
    const bool lowp = (in_t == DG_BF16 || in_t == DG_FP8E4M3) && out_t == DG_F32;
    if (!fp && !lowp) return fail(DG_EUNSUPPORTED, "dgdiff_apply: unsupported (in_t, out_t) pair");
    if (fp && (inv_sD || inv_su)) return fail(DG_EINVAL, "dgdiff_apply: scales are only for quantised input");
    if (in_t == DG_FP8E4M3 && (!inv_sD || !inv_su))
        return fail(DG_EINVAL, "dgdiff_apply: FP8 input needs both inverse scale arrays");
    const bool fused = tile && (tile->flags & DG_TILE_QUANT_U);
    if (fused && in_t != DG_BF16) return fail(DG_EINVAL, "dgdiff_apply: DG_TILE_QUANT_U is for BF16 input");
    if (nelem == 0) return DG_OK;
    if (!D || !u || !out) return fail(DG_EINVAL, "dgdiff_apply: NULL array");
    const size_t es = dtype_size(in_t), os = dtype_size(out_t);
    const size_t nD = (size_t)nmat * nunit * nunit * es;
    const size_t nu = (size_t)nelem * nunit * (fused ? 4 : es);   // fused: u is FP32
    const size_t no = (size_t)nmat * nelem * nunit * os;
    if (overlaps(out, no, D, nD) || overlaps(out, no, u, nu) ||
        overlaps(out, no, inv_sD, (size_t)nmat * 4) || overlaps(out, no, inv_su, (size_t)nelem * 4))
        return fail(DG_EINVAL, "dgdiff_apply: out overlaps an input");
    if (lowp)
        return launch_dg_forward_lowp(in_t, nmat, nelem, nunit, D, u, out, inv_sD, inv_su, tile,
                                      reinterpret_cast<hipStream_t>(stream));
    return launch_dg_forward_fp(in_t, nmat, nelem, nunit, D, u, out, tile,
                                reinterpret_cast<hipStream_t>(stream));
}

dg_status dgdiff_quantize(dg_dtype to, int64_t rows, int64_t cols, int32_t per_row_scale,
                          const float* x, void* q, float* inv_scale, dg_stream_t stream) {
    set_error("");
    if (to != DG_BF16 && to != DG_FP8E4M3)
        return fail(DG_EUNSUPPORTED, "dgdiff_quantize: target must be BF16 or FP8E4M3");
    if (rows < 0 || cols < 0) return fail(DG_EINVAL, "dgdiff_quantize: negative size");
    if (rows == 0 || cols == 0) return DG_OK;
    if (!x || !q) return fail(DG_EINVAL, "dgdiff_quantize: NULL array");
    if (to == DG_FP8E4M3 && !inv_scale) return fail(DG_EINVAL, "dgdiff_quantize: FP8 needs inv_scale");
    const size_t nx = (size_t)rows * cols * 4, nq = (size_t)rows * cols * dtype_size(to);
    const size_t ns = (size_t)(per_row_scale ? rows : 1) * 4;
    if (overlaps(q, nq, x, nx) || overlaps(inv_scale, ns, x, nx) || overlaps(inv_scale, ns, q, nq))
        return fail(DG_EINVAL, "dgdiff_quantize: outputs overlap");
    return launch_quantize(to, rows, cols, per_row_scale ? 1 : 0, x, q, inv_scale,
                           reinterpret_cast<hipStream_t>(stream));
}

size_t dgdiff_backward_workspace(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit) {
    if ((t != DG_F32 && t != DG_F64) || nmat < 1 || nmat > 8 || nunit < 1 || nunit > 512 ||
        nelem <= 0)
        return 0;
    return backward_workspace_bytes(t, nmat, nelem, nunit);
}

dg_status dgdiff_backward(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit, const void* D,
                          const void* u, const void* g, void* grad_u, void* grad_D, void* ws,
                          size_t ws_bytes, dg_stream_t stream) {
    set_error("");
    bool done = false;
    dg_status st = check_backward("dgdiff_backward", t, nmat, nelem, nunit, D, u, g, grad_u, grad_D,
                                  ws, ws_bytes, &done);
    if (st != DG_OK || done) return st;
    return launch_dg_backward(t, nmat, nelem, nunit, D, u, g, grad_u, grad_D, ws, ws_bytes,
                              reinterpret_cast<hipStream_t>(stream));
}

dg_status dgdiff_backward_noalloc(dg_dtype t, int32_t nmat, int64_t nelem, int32_t nunit,
                                  const void* D, const void* u, const void* g, void* grad_u,
                                  void* grad_D, dg_stream_t stream) {
    set_error("");
    bool done = false;
    dg_status st = check_backward("dgdiff_backward_noalloc", t, nmat, nelem, nunit, D, u, g, grad_u,
                                  grad_D, nullptr, 0, &done);
    if (st != DG_OK || done) return st;
    if (grad_D && 2 * (size_t)nmat * nunit * nunit * dtype_size(t) > kBackwardScratchBytes)
        return fail(DG_EUNSUPPORTED, "dgdiff_backward_noalloc: 2 * nmat * nunit^2 * sizeof(t) exceeds "
                                     "the fixed scratch of " +
                                         std::to_string(kBackwardScratchBytes) + " bytes");
    return launch_dg_backward_noalloc(t, nmat, nelem, nunit, D, u, g, grad_u, grad_D,
                                      reinterpret_cast<hipStream_t>(stream));
}

dg_status stencil5_apply(dg_dtype t, int64_t n, const void* u, int64_t ld_u, void* res,
                         int64_t ld_res, dg_stream_t stream) {
    set_error("");
    if (t != DG_F32 && t != DG_F64) return fail(DG_EUNSUPPORTED, "stencil5_apply: FP32 or FP64 only");
    if (n < 0) return fail(DG_EINVAL, "stencil5_apply: n must be >= 0");
    if (n == 0) return DG_OK;
    if (ld_u < n + 2 || ld_res < n) return fail(DG_EINVAL, "stencil5_apply: leading dimension too small");
    if (!u || !res) return fail(DG_EINVAL, "stencil5_apply: NULL array");
    const size_t es = dtype_size(t);
    if (overlaps(res, (size_t)n * ld_res * es, u, (size_t)(n + 2) * ld_u * es))
        return fail(DG_EINVAL, "stencil5_apply: res overlaps u");
    return launch_stencil5(t, n, u, ld_u, res, ld_res, reinterpret_cast<hipStream_t>(stream));
}

dg_status dg_ubench_run(const dg_ubench_desc* d, const void* const* in, void* out, dg_stream_t stream) {
    set_error("");
    if (!d) return fail(DG_EINVAL, "dg_ubench_run: NULL descriptor");
    dg_status st = check_ubench(d);
    if (st != DG_OK) return st;
    if (d->n == 0) return DG_OK;
    const int nin = d->kind == DG_UB_STREAM ? d->a
                  : (d->kind == DG_UB_TWIN_DG || d->kind == DG_UB_TWIN_MATMUL) ? 2
                  : (d->kind == DG_UB_STRIDED || d->kind == DG_UB_LDS || d->kind == DG_UB_OVERLAP ||
                     d->kind == DG_UB_TWIN_STENCIL || d->kind == DG_UB_TILE_READ) ? 1 : 0;
    if (!out || (nin && !in)) return fail(DG_EINVAL, "dg_ubench_run: NULL array");
    for (int k = 0; k < nin; ++k)
        if (!in[k]) return fail(DG_EINVAL, "dg_ubench_run: NULL input");
    return launch_ubench(d, in, out, reinterpret_cast<hipStream_t>(stream));
}

dg_status dg_empty_launch(int64_t workgroups, dg_stream_t stream) {
    set_error("");
    if (workgroups < 1 || workgroups > ((int64_t)1 << 31) - 1)
        return fail(DG_EINVAL, "dg_empty_launch: workgroups out of range");
    return launch_empty(workgroups, reinterpret_cast<hipStream_t>(stream));
}

dg_status matmul_apply(dg_dtype t, int64_t n, const void* a, const void* b, void* c,
                       dg_stream_t stream) {
    set_error("");
    if (t != DG_F32) return fail(DG_EUNSUPPORTED, "matmul_apply: FP32 only");
    if (n < 0) return fail(DG_EINVAL, "matmul_apply: n must be >= 0");
    if (n == 0) return DG_OK;
    if (n > (int64_t)1 << 20) return fail(DG_EUNSUPPORTED, "matmul_apply: n too large");
    if (!a || !b || !c) return fail(DG_EINVAL, "matmul_apply: NULL array");
    const size_t bytes = (size_t)n * n * 4;
    if (overlaps(c, bytes, a, bytes) || overlaps(c, bytes, b, bytes))
        return fail(DG_EINVAL, "matmul_apply: c overlaps an input");
    return launch_matmul(n, a, b, c, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
