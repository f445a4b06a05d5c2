// F64 1-D tile classes.
#include "llhmm_tiles.h"

namespace llhmm {
static const TileInfo kTiles[] = {
    LLHMM_TILE(double, 0, 1, 2, 0, 0, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 0, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 0, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 1, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 1, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 1, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 2, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 2, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 0, 2, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 0, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 0, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 0, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 1, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 1, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 1, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 2, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 2, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 0, 2, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 0, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 0, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 0, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 1, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 1, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 1, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 2, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 2, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 2, 1, 2, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 0, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 0, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 0, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 1, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 1, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 1, 64, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 2, 16, 4, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 2, 16, 8, 1, 4, 1, 2),
    LLHMM_TILE(double, 0, 1, 4, 1, 2, 64, 4, 1, 4, 1, 2),
};
const TileInfo *tiles_f64_1d(int *count) {
    *count = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    return kTiles;
}
}  // namespace llhmm
