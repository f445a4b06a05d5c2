// FP32 2-D tile classes (state and stencil in FP32, averages in FP64).
#include "llhmm_tiles.h"

namespace llhmm {
static const TileInfo kTiles[] = {
    LLHMM_TILE(float, 1, 2, 2, 0, 0, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 0, 0, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 0, 0, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE(float, 1, 2, 2, 0, 1, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 0, 1, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 0, 1, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE(float, 1, 2, 2, 0, 2, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 0, 2, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 0, 2, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE_OPT(float, 1, 2, 2, 0, 0, 64, 1, 4, 16, 2, 1, kOptHReg),
    LLHMM_TILE(float, 1, 2, 2, 1, 0, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 1, 0, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 1, 0, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE(float, 1, 2, 2, 1, 1, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 1, 1, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 1, 1, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE(float, 1, 2, 2, 1, 2, 16, 2, 4, 8, 2, 2),
    LLHMM_TILE(float, 1, 2, 2, 1, 2, 16, 3, 3, 16, 2, 2),
    LLHMM_TILE(float, 1, 2, 4, 1, 2, 16, 3, 3, 16, 1, 1),
    LLHMM_TILE_OPT(float, 1, 2, 2, 1, 0, 64, 1, 4, 16, 2, 1, kOptHReg),
    LLHMM_TILE_OPT(float, 1, 2, 2, 0, 1, 64, 1, 4, 16, 2, 1, kOptHReg),
    LLHMM_TILE_OPT(float, 1, 2, 2, 0, 2, 64, 1, 4, 16, 2, 1, kOptHReg),
    LLHMM_TILE_OPT(float, 1, 2, 2, 1, 1, 64, 1, 4, 16, 2, 1, kOptHReg),
    LLHMM_TILE_OPT(float, 1, 2, 2, 1, 2, 64, 1, 4, 16, 2, 1, kOptHReg),
    // n = 16: 4 row groups of 4 rows, one point per lane (one wavefront per box)
#define LLHMM_N16_F32(BC, QTY) LLHMM_TILE(float, 1, 2, 2, BC, QTY, 16, 1, 4, 4, 2, 16)
    LLHMM_N16_F32(0, 0), LLHMM_N16_F32(0, 1), LLHMM_N16_F32(0, 2),
    LLHMM_N16_F32(1, 0), LLHMM_N16_F32(1, 1), LLHMM_N16_F32(1, 2),
#undef LLHMM_N16_F32
    // fourth order at n = 32 (two points per lane: x1 neighbours up to two lanes
    // away) and n = 64 (one point per lane, three lanes away)
#define LLHMM_O4_F32(BC, QTY)                                      \
    LLHMM_TILE(float, 1, 2, 4, BC, QTY, 16, 2, 4, 8, 1, 1),       \
        LLHMM_TILE(float, 1, 2, 4, BC, QTY, 64, 1, 8, 8, 1, 1)
    LLHMM_O4_F32(0, 0), LLHMM_O4_F32(0, 1), LLHMM_O4_F32(0, 2),
    LLHMM_O4_F32(1, 0), LLHMM_O4_F32(1, 1), LLHMM_O4_F32(1, 2),
#undef LLHMM_O4_F32
};
const TileInfo *tiles_f32_2d(int *count) {
    *count = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    return kTiles;
}
}  // namespace llhmm
