// Slab-mode tile classes: 2-D boxes too large for one workgroup's registers
// and LDS (n = 80, 96, 112, 128), cut into row slabs that
// co-resident workgroups advance together, each in a window of R * NG rows
// with halo rows (k_slab).  Per class the first variant is the default;
// llhmm_batch_tune times the others.
#include "llhmm_micro_impl.h"

namespace llhmm {

template <typename T, int ORD, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW, int OPT>
hipError_t launch_slab(const SlabArgs &a, int nblocks, hipStream_t s) {
    if (a.mode == 1)
        hipLaunchKernelGGL((k_slab<T, ORD, QTY, BC, L, K, R, NG, NBUF, MINW, true, OPT>), dim3(nblocks), dim3(L * NG),
                           0, s, a);
    else
        hipLaunchKernelGGL((k_slab<T, ORD, QTY, BC, L, K, R, NG, NBUF, MINW, false, OPT>), dim3(nblocks),
                           dim3(L * NG), 0, s, a);
    return hipGetLastError();
}

template <typename T, int ORD, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW, int OPT>
hipError_t occupancy_slab(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, (const void *)k_slab<T, ORD, QTY, BC, L, K, R, NG, NBUF, MINW, false, OPT>, L * NG, 0);
}

#define LLHMM_SLAB_OPT(T, PREC, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, OPT)                                \
    SlabTileInfo{(K) * (L), ORD, BC, PREC, QTY, L, K, R, NG, NBUF, (L) * (NG),                             \
                 &launch_slab<T, ORD, QTY, BC, L, K, R, NG, NBUF, MINW, OPT>,                              \
                 &occupancy_slab<T, ORD, QTY, BC, L, K, R, NG, NBUF, MINW, OPT>,                           \
                 "slab " #T " o" #ORD " bc" #BC " q" #QTY " L" #L " K" #K " R" #R " NG" #NG " B" #NBUF " W" #MINW \
                 " opt" #OPT}
#define LLHMM_SLAB(T, PREC, ORD, BC, QTY, L, K, R, NG, NBUF, MINW) \
    LLHMM_SLAB_OPT(T, PREC, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, 0)
// second order, H(r) in registers
#define LLHMM_SLAB_QTY_HR(T, PREC, BC, L, K, R, NG, NBUF, MINW)                                            \
    LLHMM_SLAB_OPT(T, PREC, 2, BC, 0, L, K, R, NG, NBUF, MINW, kOptHReg),                                  \
        LLHMM_SLAB_OPT(T, PREC, 2, BC, 1, L, K, R, NG, NBUF, MINW, kOptHReg),                              \
        LLHMM_SLAB_OPT(T, PREC, 2, BC, 2, L, K, R, NG, NBUF, MINW, kOptHReg)

#define LLHMM_SLAB_QTY(T, PREC, BC, L, K, R, NG, NBUF, MINW)                                               \
    LLHMM_SLAB(T, PREC, 2, BC, 0, L, K, R, NG, NBUF, MINW), LLHMM_SLAB(T, PREC, 2, BC, 1, L, K, R, NG, NBUF, MINW), \
        LLHMM_SLAB(T, PREC, 2, BC, 2, L, K, R, NG, NBUF, MINW)
// fourth order: a halo of three rows per stage and step
#define LLHMM_SLAB_QTY4(T, PREC, BC, L, K, R, NG, NBUF, MINW)                                              \
    LLHMM_SLAB(T, PREC, 4, BC, 0, L, K, R, NG, NBUF, MINW), LLHMM_SLAB(T, PREC, 4, BC, 1, L, K, R, NG, NBUF, MINW), \
        LLHMM_SLAB(T, PREC, 4, BC, 2, L, K, R, NG, NBUF, MINW)

static const SlabTileInfo kSlab[] = {
    // FP32: windows of 32 rows.  First (the defaults, the tuner's choice on the
    // uneven batch): H(r) in registers, so the LDS left over by r and |r|^2 - 1
    // takes a double-buffered halo (one barrier per stage)
    LLHMM_SLAB_QTY_HR(float, 1, 0, 64, 2, 4, 8, 2, 1),
    LLHMM_SLAB_QTY_HR(float, 1, 1, 64, 2, 4, 8, 2, 1),
    LLHMM_SLAB_QTY_HR(float, 1, 0, 16, 6, 1, 32, 2, 1),
    LLHMM_SLAB_QTY_HR(float, 1, 1, 16, 6, 1, 32, 2, 1),
    // then the window's reference tables all in LDS, single-buffered halo
    LLHMM_SLAB_QTY(float, 1, 0, 64, 2, 4, 8, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 64, 2, 4, 8, 1, 1),
    // FP32 n = 96 with the tables in LDS: one row per lane (8 waves), then two
    // rows per lane (4 waves)
    LLHMM_SLAB_QTY(float, 1, 0, 16, 6, 1, 32, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 16, 6, 1, 32, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 0, 16, 6, 2, 16, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 16, 6, 2, 16, 1, 1),
    // FP32 n = 80 (5 points per lane, 32-row windows, H(r) in registers) and
    // n = 112 (7 points per lane, 16-row windows, one wave per SIMD)
    LLHMM_SLAB_QTY_HR(float, 1, 0, 16, 5, 1, 32, 2, 1),
    LLHMM_SLAB_QTY_HR(float, 1, 1, 16, 5, 1, 32, 2, 1),
    LLHMM_SLAB_QTY(float, 1, 0, 16, 7, 1, 16, 2, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 16, 7, 1, 16, 2, 1),
    // FP64: windows of 16 rows (reference tables read from global memory)
    LLHMM_SLAB_QTY(double, 0, 0, 64, 2, 2, 8, 2, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 64, 2, 2, 8, 2, 1),
    LLHMM_SLAB_QTY(double, 0, 0, 16, 6, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 16, 6, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 0, 16, 5, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 16, 5, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 0, 16, 7, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 16, 7, 1, 16, 1, 1),
    // fourth order (H(r) in registers for FP32): a halo of 3 rows per stage (12
    // for an RK4P step), which every slab must own at least once over: 40-row
    // windows for n = 128 (8 slabs of 16 rows), 36-row windows of three-row
    // groups for n = 96 (8 slabs of 12 rows)
    LLHMM_SLAB_QTY4(float, 1, 0, 64, 2, 4, 10, 1, 1),
    LLHMM_SLAB_QTY4(float, 1, 1, 64, 2, 4, 10, 1, 1),
    LLHMM_SLAB_QTY4(float, 1, 0, 16, 6, 3, 12, 1, 1),
    LLHMM_SLAB_QTY4(float, 1, 1, 16, 6, 3, 12, 1, 1),
    LLHMM_SLAB_QTY4(double, 0, 0, 64, 2, 4, 10, 1, 1),
    LLHMM_SLAB_QTY4(double, 0, 1, 64, 2, 4, 10, 1, 1),
    LLHMM_SLAB_QTY4(double, 0, 0, 16, 6, 3, 12, 1, 1),
    LLHMM_SLAB_QTY4(double, 0, 1, 16, 6, 3, 12, 1, 1),
};

const SlabTileInfo *tiles_slab(int *count) {
    *count = (int)(sizeof(kSlab) / sizeof(kSlab[0]));
    return kSlab;
}

}  // namespace llhmm
