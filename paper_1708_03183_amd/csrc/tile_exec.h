#pragma once
// Host entry points of the tiled executor's kernels, one translation unit per
// polynomial degree (tile_k1.hip .. tile_k4.hip).
#include <hip/hip_runtime.h>

#include "refelem.h"
#include "tile_args.h"

namespace dgt {

enum TileKernel { TK_GENERIC = 0, TK_CHAIN = 1, TK_MFMA = 2 };

// operator sequences the chain kernel is built for: (time order, first operator, operators);
// operators past the step's last belong to the next step of a chain fused over steps: two
// whole second-order steps, and the stress half of a fourth-order step with the velocity
// half of the next
constexpr int TILE_CHAINS[14][3] = {{4, 0, 3}, {4, 3, 3}, {4, 0, 6}, {2, 0, 2}, {4, 0, 1}, {4, 1, 1}, {4, 2, 1},
                                    {4, 3, 1}, {4, 4, 1}, {4, 5, 1}, {2, 0, 1}, {2, 1, 1}, {2, 0, 4}, {4, 3, 6}};

// Multi-operator chains hold every field of a cell in registers; from P3 on they
// no longer fit (spills, one wave per SIMD), so only single operators are built.
constexpr bool chain_built(int k, int nops) { return nops == 1 || k <= 2; }

// The matrix-core kernel (P3/P4) keeps the fields neighbours read in LDS, so it
// runs half steps of the fourth-order scheme too (a whole step's footprint would
// not fit; in the two-operator second-order step the first update's field is the
// second operator's operand, which the kernel does not keep in LDS).
constexpr bool mfma_built(int k, int order, int nops) { return k >= 3 && (nops == 1 || (order == 4 && nops == 3)); }
constexpr int MFMA_NT = 512;  // its workgroup size (eight waves)

// Copies the reference element into the constant memory of the degree-K unit.
template <int K, typename T>
void tile_upload_ref(const RefElem &E, hipStream_t st);

enum TileAction { TA_LAUNCH = 0, TA_ATTR = 1, TA_OCCUPANCY = 2 };

// Launches one colour of a sub-chain (TA_LAUNCH), raises the kernel's dynamic
// LDS limit (TA_ATTR), or stores in *occ how many of its workgroups one CU holds
// (TA_OCCUPANCY).  Generic kernel: any sub-chain, nt work
// items per tile.  Operator kernel: one operator application (vel selects the
// velocity operator) with an optional trailing update; needs nt >= the
// largest footprint.  Chain kernel: operators [o0, o0 + nops) of the order-`order`
// step (one of TILE_CHAINS), nt >= the largest footprint.  Matrix-core kernel
// (k >= 3): the same operator sequences, nt = MFMA_NT, any footprint that fits
// the LDS plan.
template <int K, typename T>
void tile_launch(TileKernel kind, int nt, bool upw, bool pen, int order, int o0, int nops, int grid,
                 size_t lds, hipStream_t st, const TileArgs &A, TileAction act, int *occ = nullptr);

// Launches one sub-chain of several meshes (the chain kernel's operator sequence
// [o0, o0 + nops), P1/P2, dependence-driven), or queries it like tile_launch.
template <int K, typename T>
void tile_launch_batch(bool upw, int order, int o0, int nops, int nt, int grid, size_t lds, hipStream_t st,
                       const BatchArgs &B, TileAction act, int *occ = nullptr);

// workgroup sizes the tile kernels are built for
constexpr int TILE_NT[3] = {128, 256, 512};

}  // namespace dgt
