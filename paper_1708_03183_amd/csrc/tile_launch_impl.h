#pragma once
// Instantiations of the tile kernels for degree DGT_TILE_K (included once by
// each tile_k*.hip unit).
#include "common.h"
#include "tile_exec.h"
#include "tile_chain.h"
#include "tile_kernel.h"
#include "tile_mfma.h"
#include "tile_batch.h"

namespace dgt {

template <typename Kern>
static void tile_go(Kern kern, int nt, int grid, size_t lds, hipStream_t st, const TileArgs &A, TileAction act,
                    int *occ) {
    if (act == TA_ATTR) {
        DGT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return;
    }
    if (act == TA_OCCUPANCY) {
        DGT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, nt, lds));
        return;
    }
    kern<<<grid, nt, lds, st>>>(A);
}

template <int K, typename T, int NT>
static void tile_launch_chain(bool upw, int order, int o0, int nops, int grid, size_t lds, hipStream_t st,
                              const TileArgs &A, TileAction act, int *occ) {
    auto pick = [&]<int ORD, int O0, int N>() {
        auto kern = upw ? k_tile_chain<K, T, true, ORD, O0, N, NT> : k_tile_chain<K, T, false, ORD, O0, N, NT>;
        tile_go(kern, NT, grid, lds, st, A, act, occ);
    };
    DGT_REQUIRE(chain_built(K, nops), DGT_EINVAL, "no chain kernel for this operator sequence at this degree");
    if constexpr (chain_built(K, 3)) {
        if (order == 4 && o0 == 0 && nops == 3) return pick.template operator()<4, 0, 3>();
        if (order == 4 && o0 == 3 && nops == 3) return pick.template operator()<4, 3, 3>();
        if (order == 4 && o0 == 0 && nops == 6) return pick.template operator()<4, 0, 6>();
        if (order == 2 && o0 == 0 && nops == 2) return pick.template operator()<2, 0, 2>();
        if (order == 2 && o0 == 0 && nops == 4) return pick.template operator()<2, 0, 4>();
        if (order == 4 && o0 == 3 && nops == 6) return pick.template operator()<4, 3, 6>();
    }
    if (order == 4 && nops == 1 && o0 == 0) pick.template operator()<4, 0, 1>();
    else if (order == 4 && nops == 1 && o0 == 1) pick.template operator()<4, 1, 1>();
    else if (order == 4 && nops == 1 && o0 == 2) pick.template operator()<4, 2, 1>();
    else if (order == 4 && nops == 1 && o0 == 3) pick.template operator()<4, 3, 1>();
    else if (order == 4 && nops == 1 && o0 == 4) pick.template operator()<4, 4, 1>();
    else if (order == 4 && nops == 1 && o0 == 5) pick.template operator()<4, 5, 1>();
    else if (order == 2 && nops == 1 && o0 == 0) pick.template operator()<2, 0, 1>();
    else if (order == 2 && nops == 1 && o0 == 1) pick.template operator()<2, 1, 1>();
    else DGT_REQUIRE(false, DGT_EINVAL, "no chain kernel for this operator sequence");
}

template <typename Kern>
static void batch_go(Kern kern, int nt, int grid, size_t lds, hipStream_t st, const BatchArgs &B, TileAction act,
                     int *occ) {
    if (act == TA_ATTR) {
        DGT_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        return;
    }
    if (act == TA_OCCUPANCY) {
        DGT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, nt, lds));
        return;
    }
    kern<<<grid, nt, lds, st>>>(B, B.args);
}

template <int K, typename T, int NT>
static void batch_launch_nt(bool upw, int order, int o0, int nops, int grid, size_t lds, hipStream_t st,
                            const BatchArgs &B, TileAction act, int *occ) {
    auto pick = [&]<int ORD, int O0, int N>() {
        auto kern = upw ? k_tile_chain_batch<K, T, true, ORD, O0, N, NT> : k_tile_chain_batch<K, T, false, ORD, O0, N, NT>;
        batch_go(kern, NT, grid, lds, st, B, act, occ);
    };
    if (order == 4 && o0 == 0 && nops == 3) pick.template operator()<4, 0, 3>();
    else if (order == 4 && o0 == 3 && nops == 3) pick.template operator()<4, 3, 3>();
    else if (order == 2 && o0 == 0 && nops == 2) pick.template operator()<2, 0, 2>();
    else DGT_REQUIRE(false, DGT_EINVAL, "batched launches are built for half steps and the order-2 step");
}

template <int K, typename T>
static void tile_launch_batch_any(bool upw, int order, int o0, int nops, int nt, int grid, size_t lds, hipStream_t st,
                                  const BatchArgs &B, TileAction act, int *occ) {
    if constexpr (K <= 2) {
        if (nt == 512) batch_launch_nt<K, T, 512>(upw, order, o0, nops, grid, lds, st, B, act, occ);
        else if (nt == 256) batch_launch_nt<K, T, 256>(upw, order, o0, nops, grid, lds, st, B, act, occ);
        else DGT_REQUIRE(false, DGT_EINVAL, "batched launches use workgroups of 256 or 512 threads");
    } else {
        DGT_REQUIRE(false, DGT_EINVAL, "batched launches are built for degrees 1 and 2");
    }
}

template <int K, typename T>
static void tile_launch_mfma(bool upw, int order, int o0, int nops, int grid, size_t lds, hipStream_t st,
                             const TileArgs &A, TileAction act, int *occ) {
    if constexpr (K >= 3) {
        auto pick = [&]<int ORD, int O0, int N>() {
            auto kern = upw ? k_tile_mfma<K, T, true, ORD, O0, N, MFMA_NT> : k_tile_mfma<K, T, false, ORD, O0, N, MFMA_NT>;
            tile_go(kern, MFMA_NT, grid, lds, st, A, act, occ);
        };
        if (order == 4 && o0 == 0 && nops == 3) pick.template operator()<4, 0, 3>();
        else if (order == 4 && o0 == 3 && nops == 3) pick.template operator()<4, 3, 3>();
        else if (order == 4 && nops == 1 && o0 == 0) pick.template operator()<4, 0, 1>();
        else if (order == 4 && nops == 1 && o0 == 1) pick.template operator()<4, 1, 1>();
        else if (order == 4 && nops == 1 && o0 == 2) pick.template operator()<4, 2, 1>();
        else if (order == 4 && nops == 1 && o0 == 3) pick.template operator()<4, 3, 1>();
        else if (order == 4 && nops == 1 && o0 == 4) pick.template operator()<4, 4, 1>();
        else if (order == 4 && nops == 1 && o0 == 5) pick.template operator()<4, 5, 1>();
        else if (order == 2 && nops == 1 && o0 == 0) pick.template operator()<2, 0, 1>();
        else if (order == 2 && nops == 1 && o0 == 1) pick.template operator()<2, 1, 1>();
        else DGT_REQUIRE(false, DGT_EINVAL, "no matrix-core kernel for this operator sequence");
    } else {
        DGT_REQUIRE(false, DGT_EINVAL, "the matrix-core tile kernel is built for degrees 3 and 4");
    }
}

template <int K, typename T, int NT>
static void tile_launch_nt(bool upw, bool pen, int grid, size_t lds, hipStream_t st, const TileArgs &A, TileAction act,
                           int *occ) {
    if constexpr (NT == 512) {
        if (A.scratch) {  // working sets in global scratch (no dynamic LDS)
            auto kern = upw ? (pen ? k_tile<K, T, true, true, NT, true> : k_tile<K, T, true, false, NT, true>)
                            : (pen ? k_tile<K, T, false, true, NT, true> : k_tile<K, T, false, false, NT, true>);
            tile_go(kern, NT, grid, 0, st, A, act, occ);
            return;
        }
    }
    DGT_REQUIRE(!A.scratch, DGT_EINVAL, "global working sets run with workgroups of 512");
    auto kern = upw ? (pen ? k_tile<K, T, true, true, NT> : k_tile<K, T, true, false, NT>)
                    : (pen ? k_tile<K, T, false, true, NT> : k_tile<K, T, false, false, NT>);
    tile_go(kern, NT, grid, lds, st, A, act, occ);
}

template <int K, typename T>
static void tile_launch_any(TileKernel kind, int nt, bool upw, bool pen, int order, int o0, int nops,
                            int grid, size_t lds, hipStream_t st, const TileArgs &A, TileAction act, int *occ) {
    DGT_REQUIRE(nt == 128 || nt == 256 || nt == 512, DGT_EINVAL, "tile workgroup size must be 128, 256 or 512");
    if (kind == TK_MFMA) {
        DGT_REQUIRE(nt == MFMA_NT, DGT_EINVAL, "matrix-core tile kernel workgroup size mismatch");
        tile_launch_mfma<K, T>(upw, order, o0, nops, grid, lds, st, A, act, occ);
        return;
    }
    if (kind == TK_CHAIN) {
        if (nt == 512) tile_launch_chain<K, T, 512>(upw, order, o0, nops, grid, lds, st, A, act, occ);
        else if (nt == 256) tile_launch_chain<K, T, 256>(upw, order, o0, nops, grid, lds, st, A, act, occ);
        else tile_launch_chain<K, T, 128>(upw, order, o0, nops, grid, lds, st, A, act, occ);
        return;
    }
    if (nt == 512) tile_launch_nt<K, T, 512>(upw, pen, grid, lds, st, A, act, occ);
    else if (nt == 256) tile_launch_nt<K, T, 256>(upw, pen, grid, lds, st, A, act, occ);
    else tile_launch_nt<K, T, 128>(upw, pen, grid, lds, st, A, act, occ);
}

template <>
void tile_launch<DGT_TILE_K, double>(TileKernel kind, int nt, bool upw, bool pen, int order, int o0, int nops,
                                     int grid, size_t lds, hipStream_t st, const TileArgs &A, TileAction act, int *occ) {
    tile_launch_any<DGT_TILE_K, double>(kind, nt, upw, pen, order, o0, nops, grid, lds, st, A, act, occ);
}

template <>
void tile_launch<DGT_TILE_K, float>(TileKernel kind, int nt, bool upw, bool pen, int order, int o0, int nops,
                                    int grid, size_t lds, hipStream_t st, const TileArgs &A, TileAction act, int *occ) {
    tile_launch_any<DGT_TILE_K, float>(kind, nt, upw, pen, order, o0, nops, grid, lds, st, A, act, occ);
}

template <>
void tile_launch_batch<DGT_TILE_K, double>(bool upw, int order, int o0, int nops, int nt, int grid, size_t lds,
                                           hipStream_t st, const BatchArgs &B, TileAction act, int *occ) {
    tile_launch_batch_any<DGT_TILE_K, double>(upw, order, o0, nops, nt, grid, lds, st, B, act, occ);
}

template <>
void tile_launch_batch<DGT_TILE_K, float>(bool upw, int order, int o0, int nops, int nt, int grid, size_t lds,
                                          hipStream_t st, const BatchArgs &B, TileAction act, int *occ) {
    tile_launch_batch_any<DGT_TILE_K, float>(upw, order, o0, nops, nt, grid, lds, st, B, act, occ);
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
