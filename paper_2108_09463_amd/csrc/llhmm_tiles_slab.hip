// Slab-mode tile classes: 2-D second-order boxes too large for one
// workgroup's registers and LDS (n = 96, 128), cut into row slabs that
// co-resident workgroups advance together, each in a window of R * NG rows
// with halo rows (k_slab).  Per class the first variant is the default;
// llhmm_batch_tune times the others.
#include "llhmm_micro_impl.h"

namespace llhmm {

template <typename T, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW>
hipError_t launch_slab(const SlabArgs &a, int nblocks, hipStream_t s) {
    if (a.mode == 1)
        hipLaunchKernelGGL((k_slab<T, QTY, BC, L, K, R, NG, NBUF, MINW, true>), dim3(nblocks), dim3(L * NG), 0, s, a);
    else
        hipLaunchKernelGGL((k_slab<T, QTY, BC, L, K, R, NG, NBUF, MINW, false>), dim3(nblocks), dim3(L * NG), 0, s, a);
    return hipGetLastError();
}

template <typename T, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW>
hipError_t occupancy_slab(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, (const void *)k_slab<T, QTY, BC, L, K, R, NG, NBUF, MINW, false>, L * NG, 0);
}

#define LLHMM_SLAB(T, PREC, BC, QTY, L, K, R, NG, NBUF, MINW)                                              \
    SlabTileInfo{(K) * (L), BC, PREC, QTY, L, K, R, NG, NBUF, (L) * (NG),                                  \
                 &launch_slab<T, QTY, BC, L, K, R, NG, NBUF, MINW>,                                        \
                 &occupancy_slab<T, QTY, BC, L, K, R, NG, NBUF, MINW>,                                     \
                 "slab " #T " bc" #BC " q" #QTY " L" #L " K" #K " R" #R " NG" #NG " B" #NBUF " W" #MINW}

#define LLHMM_SLAB_QTY(T, PREC, BC, L, K, R, NG, NBUF, MINW)                                               \
    LLHMM_SLAB(T, PREC, BC, 0, L, K, R, NG, NBUF, MINW), LLHMM_SLAB(T, PREC, BC, 1, L, K, R, NG, NBUF, MINW), \
        LLHMM_SLAB(T, PREC, BC, 2, L, K, R, NG, NBUF, MINW)

static const SlabTileInfo kSlab[] = {
    // FP32: windows of 32 rows (LDS holds the window's reference tables)
    LLHMM_SLAB_QTY(float, 1, 0, 64, 2, 4, 8, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 64, 2, 4, 8, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 0, 16, 6, 2, 16, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 16, 6, 2, 16, 1, 1),
    // FP32 n = 96, second variant: one row per lane, 8 waves (two per SIMD)
    LLHMM_SLAB_QTY(float, 1, 0, 16, 6, 1, 32, 1, 1),
    LLHMM_SLAB_QTY(float, 1, 1, 16, 6, 1, 32, 1, 1),
    // FP64: windows of 16 rows (reference tables read from global memory)
    LLHMM_SLAB_QTY(double, 0, 0, 64, 2, 2, 8, 2, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 64, 2, 2, 8, 2, 1),
    LLHMM_SLAB_QTY(double, 0, 0, 16, 6, 1, 16, 1, 1),
    LLHMM_SLAB_QTY(double, 0, 1, 16, 6, 1, 16, 1, 1),
};

const SlabTileInfo *tiles_slab(int *count) {
    *count = (int)(sizeof(kSlab) / sizeof(kSlab[0]));
    return kSlab;
}

}  // namespace llhmm
