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
    // n = 16: 4 row groups of 4 rows, one point per lane (one wavefront per box)
#define LLHMM_N16_F64(BC, QTY) LLHMM_TILE(double, 0, 2, 2, BC, QTY, 16, 1, 4, 4, 2, 16)
    LLHMM_N16_F64(0, 0), LLHMM_N16_F64(0, 1), LLHMM_N16_F64(0, 2),
    LLHMM_N16_F64(1, 0), LLHMM_N16_F64(1, 1), LLHMM_N16_F64(1, 2),
#undef LLHMM_N16_F64
    // fourth order in the reference + perturbation form (no boundary offsets, so
    // lanes narrower than the stencil's reach are allowed): n = 32 with the
    // reference tables in LDS, n = 64 with them read from global memory
#define LLHMM_O4_F64(BC, QTY)                                                        \
    LLHMM_TILE_OPT(double, 0, 2, 4, BC, QTY, 16, 2, 4, 8, 1, 1, kOptForm1),          \
        LLHMM_TILE_OPT(double, 0, 2, 4, BC, QTY, 16, 3, 3, 16, 1, 1, kOptForm1 | kOptRefG), \
        LLHMM_TILE_OPT(double, 0, 2, 4, BC, QTY, 64, 1, 8, 8, 1, 1, kOptForm1 | kOptRefG)
    LLHMM_O4_F64(0, 0), LLHMM_O4_F64(0, 1), LLHMM_O4_F64(0, 2),
    LLHMM_O4_F64(1, 0), LLHMM_O4_F64(1, 1), LLHMM_O4_F64(1, 2),
#undef LLHMM_O4_F64
};
const TileInfo *tiles_f64_2d(int *count) {
    *count = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    return kTiles;
}
}  // namespace llhmm
