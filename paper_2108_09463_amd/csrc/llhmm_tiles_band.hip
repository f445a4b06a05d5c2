// Band-mode tile classes: 2-D, second-order boxes too large for one block's
// registers and LDS (n = 96, 128), advanced in full-width row strips.
#include "llhmm_micro_impl.h"

namespace llhmm {

template <typename T, int QTY, int BC, int L, int K, int R, int NG, int NBUF, int MINW>
hipError_t launch_band(const BandArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_band<T, QTY, BC, L, K, R, NG, NBUF, MINW>), dim3(nblocks), dim3(L * NG), 0, s, a);
    return hipGetLastError();
}

#define LLHMM_BAND(T, PREC, BC, QTY, L, K, R, NG, NBUF, MINW)                                        \
    BandTileInfo{(K) * (L), BC, PREC, QTY, L, K, R, NG, NBUF, (L) * (NG),                            \
                 &launch_band<T, QTY, BC, L, K, R, NG, NBUF, MINW>,                                  \
                 "band " #T " bc" #BC " q" #QTY " L" #L " K" #K " R" #R " NG" #NG " B" #NBUF " W" #MINW}

#define LLHMM_BAND_QTY(T, PREC, BC, L, K, R, NG, NBUF, MINW)                                         \
    LLHMM_BAND(T, PREC, BC, 0, L, K, R, NG, NBUF, MINW), LLHMM_BAND(T, PREC, BC, 1, L, K, R, NG, NBUF, MINW), \
        LLHMM_BAND(T, PREC, BC, 2, L, K, R, NG, NBUF, MINW)

static const BandTileInfo kBand[] = {
    // FP32: windows of 32 rows (LDS holds the window's reference tables)
    LLHMM_BAND_QTY(float, 1, 0, 64, 2, 4, 8, 1, 1),
    LLHMM_BAND_QTY(float, 1, 1, 64, 2, 4, 8, 1, 1),
    LLHMM_BAND_QTY(float, 1, 0, 16, 6, 2, 16, 1, 1),
    LLHMM_BAND_QTY(float, 1, 1, 16, 6, 2, 16, 1, 1),
    // FP32 n = 96, second variant: 24-row windows, one row per lane, 6 waves per block
    LLHMM_BAND_QTY(float, 1, 0, 16, 6, 1, 24, 1, 1),
    LLHMM_BAND_QTY(float, 1, 1, 16, 6, 1, 24, 1, 1),
    // FP64: windows of 16 rows (reference tables read from global memory)
    LLHMM_BAND_QTY(double, 0, 0, 64, 2, 2, 8, 2, 1),
    LLHMM_BAND_QTY(double, 0, 1, 64, 2, 2, 8, 2, 1),
    LLHMM_BAND_QTY(double, 0, 0, 16, 6, 1, 16, 1, 1),
    LLHMM_BAND_QTY(double, 0, 1, 16, 6, 1, 16, 1, 1),
};

const BandTileInfo *tiles_band(int *count) {
    *count = (int)(sizeof(kBand) / sizeof(kBand[0]));
    return kBand;
}

}  // namespace llhmm
