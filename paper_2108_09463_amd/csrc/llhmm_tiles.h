// Tile-class registration helpers: one explicit instantiation of k_micro per
// (precision, dim, order, boundary, layout) with its launcher.
#pragma once
#include "llhmm_micro_impl.h"

namespace llhmm {

template <typename T, int D, int ORD, int BC, int QTY, int L, int K, int R, int NG, int NBUF, int MINW, int OPT>
hipError_t launch_tile(const MicroArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_micro<T, D, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, OPT>), dim3(nblocks),
                       dim3(L * NG), 0, s, a);
    return hipGetLastError();
}

#define LLHMM_TILE_OPT(T, PREC, D, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, OPT)                       \
    TileInfo{D, (K) * (L), ORD, BC, PREC, QTY, L, K, R, NG, NBUF, (L) * (NG),                  \
             (D) == 1 ? (NG) : 1, &launch_tile<T, D, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, OPT>,    \
             #T " d" #D " o" #ORD " bc" #BC " q" #QTY " L" #L " K" #K " R" #R " NG" #NG " B" #NBUF " W" #MINW \
             " opt" #OPT, OPT}
#define LLHMM_TILE(T, PREC, D, ORD, BC, QTY, L, K, R, NG, NBUF, MINW) \
    LLHMM_TILE_OPT(T, PREC, D, ORD, BC, QTY, L, K, R, NG, NBUF, MINW, 0)

}  // namespace llhmm
