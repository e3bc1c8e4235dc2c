// DG differentiation forward operator, FP32 and FP64 (kernel in dg_kernel.hpp):
//     out[m][e][i] = sum_j D[m][i][j] * u[e][j].
#include "dg_kernel.hpp"

namespace dg {
namespace {

using namespace kern;

template <typename T>
kern_fn forward_kernel(int kq, int cb, bool pair = false) {
    return cb == 4 ? pick_kernel<T, 4, 1>(kq, pair) : cb == 2 ? pick_kernel<T, 2, 1>(kq, pair)
                                                             : pick_kernel<T, 1, 1>(kq, pair);
}

template <typename T>
dg_status launch_fwd(int nmat, int64_t nelem, int nunit, const void* D, const void* u, void* out,
                     const dg_tile* tile, hipStream_t s) {
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    const bool rows_aligned =
        (nunit % Mma<T>::V == 0) && (reinterpret_cast<uintptr_t>(u) % 16 == 0);
    int cb;
    dg_status st = forward_cb(sizeof(T), kq, rows_aligned, tile ? tile->elems_per_wave : 0, &cb);
    if (st != DG_OK) return st;
    const int waves =
        (tile && tile->waves) ? tile->waves : forward_waves(sizeof(T), nunit, kq, cb, rows_aligned);
    if (waves < 1 || waves > 8) return fail(DG_EINVAL, "tile.waves must be in 1..8");
    KArgs a = {};
    a.D = D;
    a.src = u;
    a.out = out;
    a.nelem = nelem;
    a.seg_stride = 0;
    a.nunit = nunit;
    a.transpose = 0;
    return launch<T, 1>(a, nmat, kq, cb, tile, waves, forward_kernel<T>(kq, cb), s,
                        forward_kernel<T>(kq, cb, true), nullptr, true);
}

}  // namespace

dg_status launch_dg_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                               const void* u, void* out, const dg_tile* tile, hipStream_t s) {
    if (t == DG_F32) return launch_fwd<float>(nmat, nelem, nunit, D, u, out, tile, s);
    if (t == DG_F64) return launch_fwd<double>(nmat, nelem, nunit, D, u, out, tile, s);
    return fail(DG_EUNSUPPORTED, "launch_dg_forward_fp: dtype");
}

// Resolve a forward launch shape (0 fields -> defaults, occupancy queried on
// the current device) for the feature counter and the autotuner.
dg_status resolve_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit, dg_tile* tile) {
    const size_t ts = t == DG_F64 ? 8 : 4;
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    int cb;
    dg_status st = forward_cb(ts, kq, nunit % (int)(16 / ts) == 0, tile->elems_per_wave, &cb);
    if (st != DG_OK) return st;
    if (tile->waves == 0) tile->waves = forward_waves(ts, nunit, kq, cb, nunit % (int)(16 / ts) == 0);
    tile->elems_per_wave = 16 * cb;
    DeviceInfo dev;
    st = current_device(&dev);
    if (st != DG_OK) return st;
    Plan P;
    st = make_plan(ts, 1, nmat, nelem, nunit, kq, cb, tile->waves, tile->d_panels, 1, dev.num_cu,
                   nunit % (int)(16 / ts) == 0, &P);
    if (st != DG_OK) return st;
    tile->d_panels = P.ppg;
    {
        // the launch's own check: the work-group must fit the kernel's bound
        kern_fn f0 = t == DG_F64 ? forward_kernel<double>(kq, cb) : forward_kernel<float>(kq, cb);
        if (!f0) return fail(DG_EUNSUPPORTED, "no DG kernel instance");
        hipFuncAttributes fa;
        DG_HIP_CHECK(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(f0)));
        if (64 * tile->waves > fa.maxThreadsPerBlock)
            return fail(DG_EINVAL, "tile.waves above 4 needs a shape whose element data fit 64 registers");
    }
    if (tile->groups_per_cu == 0) {
        // the kernel a launch into 16-byte aligned output would take
        const bool pair = pair_eligible(ts, nunit, nunit % 4 == 0, P);
        kern_fn fn = t == DG_F64 ? forward_kernel<double>(kq, cb) : forward_kernel<float>(kq, cb, pair);
        if (!fn) return fail(DG_EUNSUPPORTED, "no DG kernel instance");
        DG_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.smem));
        int per_cu = 0;
        DG_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(fn), 64 * tile->waves, P.smem));
        tile->groups_per_cu = std::max(1, per_cu);
    }
    return DG_OK;
}

}  // namespace dg
