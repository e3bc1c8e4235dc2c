// Closed-form operation counts of the program variants (variants.hip): the
// input features the variant-ranking model is fitted and evaluated on
// (Sections "Gathering Kernel Statistics" and "Kernel Features").
//
// Granularities (the paper's rules as read here): kernel launches and
// work-groups per launch; barriers per work-item times work-groups; vector-ALU
// and LDS work per wave instruction, counted as 64 lanes whatever the active
// lanes (sub-group granularity); global loads and stores in bytes of the lanes
// that issue them (work-item granularity).  Arithmetic is counted as written in
// the kernels: a fused multiply-add is 2 flops, an add 1.  Every global access
// pattern of the variants has its own feature; a twin's per-work-item
// destination store is the stride-1 pattern of the microbenchmark stores.
// A brute-force walk of the same schedules in the test oracle must give
// identical int64 counts.
#include "common.hpp"

namespace dg {
namespace {

const char* kVNames[VF_COUNT] = {
    "launch", "workgroups", "barrier_x_wg", "valu_f32_sg", "lds_sg", "gld_ub", "gst_ub",
    "gld_ub_strided", "gld_mm_pf_a", "gld_mm_pf_b", "gld_mm_nopf_a", "gld_mm_nopf_b", "gst_mm_c",
    "gld_dg_nopf_u", "gld_dg_dm", "gld_dg_upf_u", "gld_dg_dmpf_u", "gld_dg_dmpf_dm", "gld_dg_dmpft_u",
    "gst_dg_nopf_res", "gst_dg_upf_res", "gst_dg_dmpf_res", "gst_dg_dmpft_res", "gld_fd16_u",
    "gst_fd16_res", "gld_fd18_u", "gst_fd18_res"};

void count_variant(const dg_variant_desc* d, int64_t* c) {
    const VariantShape s = variant_shape(d);
    const int64_t W = s.gx * s.gy;
    if (W == 0) return;
    const bool twin = d->work_removed != 0;
    const int64_t k0 = (d->keep & DG_V_KEEP_IN0) ? 1 : 0, k1 = (d->keep & DG_V_KEEP_IN1) ? 1 : 0;
    const bool kout = !twin || (d->keep & DG_V_KEEP_OUT);
    const int64_t lanes = W * s.threads;        // work-items
    const int64_t n = d->n;
    c[VF_LAUNCH] = 1;
    c[VF_WORKGROUPS] = W;
    if (!kout) c[VF_GST_UB] = 4 * lanes;
    switch (d->kind) {
        case DG_V_MM_PF: {
            const int64_t K = n / 16;   // k steps
            if (!twin) {
                c[VF_BARRIER_X_WG] = 2 * K * W;
                c[VF_GLD_MM_PF_A] = c[VF_GLD_MM_PF_B] = 4 * K * lanes;
                c[VF_LDS_SG] = 4 * (2 + 2 * 16) * K * lanes;
                c[VF_VALU_F32_SG] = 2 * 16 * K * lanes;
            } else {
                c[VF_GLD_MM_PF_A] = 4 * K * lanes * k0;
                c[VF_GLD_MM_PF_B] = 4 * K * lanes * k1;
                c[VF_VALU_F32_SG] = K * lanes * (k0 + k1);
            }
            if (kout) c[VF_GST_MM_C] = 4 * n * n;
            return;
        }
        case DG_V_MM_NOPF:
            c[VF_GLD_MM_NOPF_A] = 4 * n * lanes * (twin ? k0 : 1);
            c[VF_GLD_MM_NOPF_B] = 4 * n * lanes * (twin ? k1 : 1);
            c[VF_VALU_F32_SG] = twin ? n * lanes * (k0 + k1) : 2 * n * lanes;
            if (kout) c[VF_GST_MM_C] = 4 * n * n;
            return;
        case DG_V_DG_NOPF:
        case DG_V_DG_PFU:
        case DG_V_DG_PFDM:
        case DG_V_DG_PFDMT: {
            const int64_t M = d->nmat, nu = d->nunit, J = nu / 16;
            const int64_t res = 4 * M * n * nu;   // one store per (m, element, node)
            if (d->kind == DG_V_DG_NOPF) {
                c[VF_GLD_DG_NOPF_U] = 4 * M * nu * lanes * (twin ? k0 : 1);
                c[VF_GLD_DG_DM] = 4 * M * nu * lanes * (twin ? k1 : 1);
                c[VF_VALU_F32_SG] = twin ? M * nu * lanes * (k0 + k1) : 2 * M * nu * lanes;
                if (kout) c[VF_GST_DG_NOPF_RES] = res;
            } else if (d->kind == DG_V_DG_PFU) {
                c[VF_GLD_DG_UPF_U] = 4 * J * lanes * (twin ? k0 : 1);
                c[VF_GLD_DG_DM] = 4 * M * nu * lanes * (twin ? k1 : 1);
                if (!twin) {
                    c[VF_BARRIER_X_WG] = 2 * J * W;
                    c[VF_LDS_SG] = 4 * (J + nu) * lanes;
                    c[VF_VALU_F32_SG] = 2 * M * nu * lanes;
                } else {
                    c[VF_VALU_F32_SG] = (J * k0 + M * nu * k1) * lanes;
                }
                if (kout) c[VF_GST_DG_UPF_RES] = res;
            } else {
                const bool tr = d->kind == DG_V_DG_PFDMT;
                c[VF_GLD_DG_DMPF_DM] = 4 * M * J * lanes * (twin ? k1 : 1);
                c[tr ? VF_GLD_DG_DMPFT_U : VF_GLD_DG_DMPF_U] = 4 * M * nu * lanes * (twin ? k0 : 1);
                if (!twin) {
                    c[VF_BARRIER_X_WG] = 2 * M * J * W;
                    c[VF_LDS_SG] = 4 * M * (J + nu) * lanes;
                    c[VF_VALU_F32_SG] = 2 * M * nu * lanes;
                } else {
                    c[VF_VALU_F32_SG] = (M * J * k1 + M * nu * k0) * lanes;
                }
                if (kout) c[tr ? VF_GST_DG_DMPFT_RES : VF_GST_DG_DMPF_RES] = res;
            }
            return;
        }
        case DG_V_FD16:
        case DG_V_FD18: {
            const bool big = d->kind == DG_V_FD18;
            // waves per work-group, and those holding a computing work-item
            // (l0, l1 < L - 2): 16 x 16 = 256 = 4 waves, all computing; 18 x 18
            // = 324 = 6 waves, the last (work-items 320..323, row 17) idle
            const int64_t wv = big ? 6 : 4, cw = big ? 5 : 4;
            c[big ? VF_GLD_FD18_U : VF_GLD_FD16_U] = 4 * lanes * (twin ? k0 : 1);
            if (!twin) {
                c[VF_BARRIER_X_WG] = W;
                c[VF_LDS_SG] = 256 * W * (wv + 5 * cw);
                c[VF_VALU_F32_SG] = 64 * 5 * cw * W;    // three adds and a fused multiply-add
            } else {
                c[VF_VALU_F32_SG] = 64 * wv * W * k0;
            }
            if (kout) c[big ? VF_GST_FD18_RES : VF_GST_FD16_RES] = 4 * n * n;
            return;
        }
    }
}

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" {

int32_t perf_variant_feature_count(void) { return VF_COUNT; }

const char* perf_variant_feature_name(int32_t k) { return (k >= 0 && k < VF_COUNT) ? kVNames[k] : ""; }

dg_status perf_variant_count(const dg_variant_desc* d, int64_t* counts) {
    set_error("");
    if (!d || !counts) return fail(DG_EINVAL, "perf_variant_count: NULL argument");
    for (int k = 0; k < VF_COUNT; ++k) counts[k] = 0;
    const dg_status st = check_variant(d);
    if (st != DG_OK) return st;
    count_variant(d, counts);
    return DG_OK;
}

}  // extern "C"
