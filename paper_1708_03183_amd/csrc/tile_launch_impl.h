#pragma once
// Instantiations of the tile kernels for degree DGT_TILE_K (included once by
// each tile_k*.hip unit).
#include "common.h"
#include "tile_exec.h"
#include "tile_kernel.h"

namespace dgt {

template <typename Kern>
static void tile_go(Kern kern, int nt, int grid, size_t lds, hipStream_t st, const TileArgs &A, bool attr) {
    if (attr) {
        DGT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return;
    }
    kern<<<grid, nt, lds, st>>>(A);
}

template <int K, typename T, int NT>
static void tile_launch_nt(TileKernel kind, bool vel, bool upw, bool pen, int grid, size_t lds, hipStream_t st,
                           const TileArgs &A, bool attr) {
    if (kind == TK_OP) {
        auto kern = vel ? (upw ? k_tile_op<K, T, true, true, NT> : k_tile_op<K, T, true, false, NT>)
                        : (upw ? k_tile_op<K, T, false, true, NT> : k_tile_op<K, T, false, false, NT>);
        tile_go(kern, NT, grid, lds, st, A, attr);
    } else {
        auto kern = upw ? (pen ? k_tile<K, T, true, true, NT> : k_tile<K, T, true, false, NT>)
                        : (pen ? k_tile<K, T, false, true, NT> : k_tile<K, T, false, false, NT>);
        tile_go(kern, NT, grid, lds, st, A, attr);
    }
}

template <>
void tile_launch<DGT_TILE_K, double>(TileKernel kind, int nt, bool vel, bool upw, bool pen, int grid, size_t lds,
                                     hipStream_t st, const TileArgs &A, bool attr);
template <>
void tile_launch<DGT_TILE_K, float>(TileKernel kind, int nt, bool vel, bool upw, bool pen, int grid, size_t lds,
                                    hipStream_t st, const TileArgs &A, bool attr);

template <int K, typename T>
static void tile_launch_any(TileKernel kind, int nt, bool vel, bool upw, bool pen, int grid, size_t lds,
                            hipStream_t st, const TileArgs &A, bool attr) {
    DGT_REQUIRE(nt == 128 || nt == 256 || nt == 512, DGT_EINVAL, "tile workgroup size must be 128, 256 or 512");
    if (nt == 512) tile_launch_nt<K, T, 512>(kind, vel, upw, pen, grid, lds, st, A, attr);
    else if (nt == 256) tile_launch_nt<K, T, 256>(kind, vel, upw, pen, grid, lds, st, A, attr);
    else tile_launch_nt<K, T, 128>(kind, vel, upw, pen, grid, lds, st, A, attr);
}

template <>
void tile_launch<DGT_TILE_K, double>(TileKernel kind, int nt, bool vel, bool upw, bool pen, int grid, size_t lds,
                                     hipStream_t st, const TileArgs &A, bool attr) {
    tile_launch_any<DGT_TILE_K, double>(kind, nt, vel, upw, pen, grid, lds, st, A, attr);
}

template <>
void tile_launch<DGT_TILE_K, float>(TileKernel kind, int nt, bool vel, bool upw, bool pen, int grid, size_t lds,
                                    hipStream_t st, const TileArgs &A, bool attr) {
    tile_launch_any<DGT_TILE_K, float>(kind, nt, vel, upw, pen, grid, lds, st, A, attr);
}

template <>
void tile_upload_ref<DGT_TILE_K, double>(const RefElem &E, hipStream_t st) {
    upload_ref<DGT_TILE_K, double>(E, st);
}

template <>
void tile_upload_ref<DGT_TILE_K, float>(const RefElem &E, hipStream_t st) {
    upload_ref<DGT_TILE_K, float>(E, st);
}

}  // namespace dgt
