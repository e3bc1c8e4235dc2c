// DG differentiation forward operator, FP32 and FP64 (kernel in dg_kernel.hpp):
//     out[m][e][i] = sum_j D[m][i][j] * u[e][j].
#include "dg_kernel.hpp"

namespace dg {
namespace {

using namespace kern;

template <typename T>
dg_status launch_fwd(int nmat, int64_t nelem, int nunit, const void* D, const void* u, void* out,
                     const dg_tile* tile, hipStream_t s) {
    const int kq = kq_for(nunit);
    if (kq < 0) return fail(DG_EUNSUPPORTED, "nunit too large for the DG kernel");
    const int waves = (tile && tile->waves) ? tile->waves : 4;
    const int epw = (tile && tile->elems_per_wave) ? tile->elems_per_wave : 0;
    if (waves < 1 || waves > 4) return fail(DG_EINVAL, "tile.waves must be in 1..4");
    const bool rows_aligned =
        (nunit % Mma<T>::V == 0) && (reinterpret_cast<uintptr_t>(u) % 16 == 0);
    int cb;
    if (epw == 0) {
        // measured defaults (FP32, 2^21 elements): aligned short rows favour one
        // column block per wave (more waves in flight); otherwise more column
        // blocks per wave, as registers allow
        const int w = kq * (int)sizeof(T) / 4;  // KQ in 32-bit registers
        if (rows_aligned && w <= 16) cb = 1;
        else if (w <= 32) cb = 4;
        else if (w <= 64) cb = 2;
        else cb = 1;
    } else if (epw == 16) {
        cb = 1;
    } else if (epw == 32) {
        cb = 2;
    } else if (epw == 64 && kq * (int)sizeof(T) <= 32 * 4) {
        cb = 4;
    } else {
        return fail(DG_EINVAL,
                    "tile.elems_per_wave must be 16 or 32 (or 64 for nunit <= 128 in FP32)");
    }
    KArgs a = {};
    a.D = D;
    a.src = u;
    a.out = out;
    a.nelem = nelem;
    a.seg_stride = 0;
    a.nunit = nunit;
    a.transpose = 0;
    auto pick = [kq](int c) -> kern_fn {
        return c == 4 ? pick_kernel<T, 4, 1>(kq) : c == 2 ? pick_kernel<T, 2, 1>(kq)
                                                         : pick_kernel<T, 1, 1>(kq);
    };
    return launch<T, 1>(a, nmat, kq, cb, tile, waves, pick, s);
}

}  // namespace

dg_status launch_dg_forward_fp(dg_dtype t, int nmat, int64_t nelem, int nunit, const void* D,
                               const void* u, void* out, const dg_tile* tile, hipStream_t s) {
    if (t == DG_F32) return launch_fwd<float>(nmat, nelem, nunit, D, u, out, tile, s);
    if (t == DG_F64) return launch_fwd<double>(nmat, nelem, nunit, D, u, out, tile, s);
    return fail(DG_EUNSUPPORTED, "launch_dg_forward_fp: dtype");
}

}  // namespace dg
