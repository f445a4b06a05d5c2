// d = 3 micro boxes (FP64, second-order stencil): launch arguments shared by
// the host side (llhmm_host.cpp) and llhmm_micro3d.hip.  Not part of the
// public ABI.
#pragma once
#include "llhmm_internal.h"

namespace llhmm {

// One block per box, arrays in a per-box work area of work3d_size(n, order) doubles
// at plan.tab_offset.
struct Micro3dArgs {
    const BoxPlan *plans;
    const int32_t *box_ids;    // the batch's 3-D boxes
    int32_t nbox, mode;        // mode 0 solve, 1 evaluate H(m_init) only
    int32_t nmax, nq_max;      // largest n of the 3-D boxes; largest outputs per box (9: flux)
    int32_t orders, sampled;   // stencil orders present (bit 0 second, bit 1 fourth); a box's coefficient is sampled
    const double *coef_samples;   // sampled coefficients: face values [3][E6^3] per box at coef_offset, E6 = n + 6
    const CoefDev *coefs;
    const double *m_init;      // explicit initial data (extended grid, LLHMM_GHOST layers)
    const double *M_macro;     // macro field [3][n^3]
    MacroDev macro;
    double *work;              // 3-D work buffer (doubles)
    double *wts;               // space weights (written by the set-up)
    const double *wt;          // time-weight table
    double *partials;          // [slots][kMaxQ]
    int32_t *wave_status;      // [slots]
    double *box_const;         // [nboxes][kMaxQ] (zeroed for 3-D boxes)
    double *out_field;         // m_final or H (nullable)
    double kc[8];              // space kernel coefficients c_0..c_p
    int32_t kp, kq;
};
hipError_t launch_setup3d(const Micro3dArgs &a, hipStream_t s);
hipError_t launch_micro3d(const Micro3dArgs &a, hipStream_t s);
int64_t work3d_size(int n, int order);

}  // namespace llhmm
