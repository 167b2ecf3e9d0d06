#pragma once
// Launch arguments of the tiled executor's kernels (host and device).
#include <cstdint>

#include "dg_kernels.h"

namespace dgt {

struct TLoop {
    int8_t kind, in, out, pen;
    int8_t partner;  // exterior loop fused into this interior loop, or -1
    int8_t grp;      // neighbour table of a facet loop, or -1
    int8_t step;     // time step of the loop counted from the sub-chain's first (fused chains)
    float scale_f, pscale_f;
    double scale_d, pscale_d;
};

// neighbour-table codes
constexpr uint32_t NB_VALID = 1u << 31, NB_BND = 1u << 30, NB_FREE = 1u << 29;

struct TileArgs {
    int32_t nloops;
    TLoop loops[31];
    const int32_t *foot_off;  // [ntiles+1]
    const int32_t *foot;      // exec cell ids, ascending per tile
    const uint32_t *facc;     // loop bits + single-tile flag per footprint entry
    const uint32_t *tnb;      // per tile: [nfl][3][nfoot] neighbour codes
    const int32_t *tnb_off;   // [ntiles+1]
    const int32_t *tiles;     // tiles of this sub-chain in execution order
    // per position of `tiles`: the tile, its first footprint slot, its footprint length
    // and its neighbour-table offset, read by the chain kernel in one load
    const int32_t *tmeta;     // [ntiles][4]
    int32_t tile_base;        // first tile of the colour in `tiles`
    void *F[F_COUNT];
    const void *geo;
    int64_t nc;
    uint32_t loops_mask[F_COUNT], rfirst_mask[F_COUNT], writes_mask[F_COUNT];
    int32_t persistent_mask;   // fields always written back when written
    int32_t lds_row[F_COUNT];  // offset of each field in a slot's LDS row (-1: unused)
    int32_t nrow;              // LDS elements per slot (odd), geometry in the last G_NROWS
    int32_t stride;            // slot capacity (largest footprint of the sub-chain)
    int32_t nfl;               // facet loops with a neighbour table
    void *scratch;             // generic kernel with tiles beyond the LDS: per-workgroup working sets
    int64_t scratch_bytes;     // bytes of one working set (a multiple of 256)
    // shots: independent states on the same mesh; a work item is a (tile, shot) pair,
    // item i taking tile i / nshots and shot i % nshots, so consecutive workgroups share
    // a tile's metadata and geometry
    int32_t nshots;
    int64_t fshot[F_COUNT];     // elements between two shots' copies of a field
    const int32_t *src_cells;   // [nshots] exec id of each shot's source cell, or -1
    double dt, src_amp;         // src_amp = dt * r(t^{n+1/2}), the same wavelet for every shot
    double src_amps[4];         // the same for the sub-chain's steps n, n+1, ... (chains fused over steps)
    const void *src_vec;        // [nshots][Np] inverse mass times the basis at each source
    // dependence-driven schedule (chain kernel): one launch per sub-chain; workgroups take
    // tiles in colour order from a ticket counter, and a tile starts once every
    // lower-colour tile whose footprint meets its own has finished
    int32_t persist;            // 0: one launch per colour (tiles[tile_base + blockIdx.x])
    int32_t ntiles;             // tiles of the sub-chain
    int32_t nexec;              // tiles that run (all but a region-aware schedule's T_ne)
    const int32_t *need;        // [ntiles] predecessors per tile
    const int32_t *succ_off;    // [ntiles+1] successors (CSR)
    const int32_t *succ;
    uint32_t *cnt;              // [nshots][ntiles] finished predecessors, counted across launches
    uint32_t *head;             // ticket counter, counted across launches
    int32_t *err;               // set when a wait times out
    uint32_t epoch;             // launches of this plan so far (this one included)
    uint32_t head_base;         // tickets taken by earlier launches
    uint32_t spin_limit;        // polls before a wait gives up
};

// Several meshes in one launch per sub-chain (dependence-driven schedule): a work
// queue over (mesh, tile, shot) items, segments of one mesh's tiles of one colour
// ordered by colour, then mesh.
struct BatchArgs {
    const TileArgs *args;      // [nmesh] per-mesh launch arguments (device)
    int32_t persist;           // 1: dependence-driven (tickets); 0: one colour, one item per workgroup
    int32_t seg_first;         // colour launches: the colour's first segment, its first ticket
    uint32_t ticket_base;
    int32_t nseg;              // segments searched (from seg_first)
    const int32_t *seg_start;  // [nseg + 1] first ticket of each segment
    const int32_t *seg_mesh;   // [nseg] mesh of the segment
    const int32_t *seg_local;  // [nseg] the segment's first item in its mesh's own order
    uint32_t *head;            // ticket counter, counted across launches
    uint32_t head_base;        // tickets taken by earlier launches
    uint32_t total;            // items of this launch
    uint32_t epoch;            // launches of this sub-chain since the counters were cleared
    // source amplitude of the step: amp_tab[mesh * amp_stride + (*amp_base) + amp_idx]
    // (amp_base NULL: 0; graph replays move *amp_base between replays)
    const double *amp_tab;
    const int32_t *amp_base;
    int32_t amp_idx, amp_stride;
};

}  // namespace dgt
