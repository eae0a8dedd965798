// rbc_dispatch.cpp -- routes a tile launch to the object compiled for its
// 16-feature slab count.
#include "rbc_common.h"

namespace rbc {

hipError_t launch_tile_mfma(int ks, int c, int mode, dim3 grid, const TileArgs& a,
                            hipStream_t st) {
    switch (ks) {
        case 1: return launch_tile_mfma_ks1(c, mode, grid, a, st);
        case 2: return launch_tile_mfma_ks2(c, mode, grid, a, st);
        case 3: return launch_tile_mfma_ks3(c, mode, grid, a, st);
        case 4: return launch_tile_mfma_ks4(c, mode, grid, a, st);
        case 5: return launch_tile_mfma_ks5(c, mode, grid, a, st);
        case 6: return launch_tile_mfma_ks6(c, mode, grid, a, st);
        case 7: return launch_tile_mfma_ks7(c, mode, grid, a, st);
        case 8: return launch_tile_mfma_ks8(c, mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tile_valu(int metric, int ks, int c, int mode, dim3 grid,
                            const TileArgs& a, hipStream_t st) {
    switch (ks) {
        case 1: return launch_tile_valu_ks1(metric, c, mode, grid, a, st);
        case 2: return launch_tile_valu_ks2(metric, c, mode, grid, a, st);
        case 3: return launch_tile_valu_ks3(metric, c, mode, grid, a, st);
        case 4: return launch_tile_valu_ks4(metric, c, mode, grid, a, st);
        case 5: return launch_tile_valu_ks5(metric, c, mode, grid, a, st);
        case 6: return launch_tile_valu_ks6(metric, c, mode, grid, a, st);
        case 7: return launch_tile_valu_ks7(metric, c, mode, grid, a, st);
        case 8: return launch_tile_valu_ks8(metric, c, mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tile_lowp(int fmt, int kb, int c, int mode, dim3 grid, const TileArgs& a,
                            hipStream_t st) {
    if (fmt == 1) return launch_tile_lowp_kb1(fmt, c, mode, grid, a, st);
    switch (kb) {
        case 1: return launch_tile_lowp_kb1(fmt, c, mode, grid, a, st);
        case 2: return launch_tile_lowp_kb2(fmt, c, mode, grid, a, st);
        case 3: return launch_tile_lowp_kb3(fmt, c, mode, grid, a, st);
        case 4: return launch_tile_lowp_kb4(fmt, c, mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace rbc
