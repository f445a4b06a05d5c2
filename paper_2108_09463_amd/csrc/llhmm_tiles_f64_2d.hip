// FP64 2-D tile classes (the plain FP64 GPU path).
#include "llhmm_tiles.h"

namespace llhmm {
static const TileInfo kTiles[] = {
    LLHMM_TILE(double, 0, 2, 2, 0, 0, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 1, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 2, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 0, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 0, 64, 1, 8, 8, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 0, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 1, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 2, 16, 2, 2, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 0, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 0, 64, 1, 8, 8, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 1, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 2, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 1, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 2, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 1, 64, 1, 8, 8, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 0, 2, 64, 1, 8, 8, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 1, 64, 1, 8, 8, 2, 2),
    LLHMM_TILE(double, 0, 2, 2, 1, 2, 64, 1, 8, 8, 2, 2),
};
const TileInfo *tiles_f64_2d(int *count) {
    *count = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    return kTiles;
}
}  // namespace llhmm
