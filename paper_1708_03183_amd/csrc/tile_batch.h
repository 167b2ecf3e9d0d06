#pragma once
// Several solvers (meshes, each with its shots) advanced together on the
// register-resident chain kernel: one queue over the (mesh, tile, shot) items of
// all of them, ordered by colour, then mesh (segment g holds the items of one
// mesh's tiles of one colour, in that mesh's own execution order).  Colour
// launches: one launch per colour of a sub-chain for all meshes, one item per
// workgroup.  Dependence-driven: one launch per sub-chain, workgroups take
// tickets; a tile's predecessors are tiles of the same mesh with lower colours,
// so they sit in earlier segments and were taken by workgroups already running,
// and the wait argument of the single-mesh schedule holds unchanged.  Each mesh keeps its own
// fields, schedule, dependence counters and source; an item runs exactly the
// arithmetic of the single-mesh kernel on its mesh's data.
#include <hip/hip_runtime.h>

#include "tile_chain.h"

namespace dgt {


template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
__device__ __forceinline__ void batch_body(const RefC<K, T> &Rf, const BatchArgs &b,
                                           const TileArgs *__restrict__ args, unsigned char *smem) {
    __shared__ int s_tile, s_shot, s_mesh, s_f0, s_nfoot, s_b0;
    __shared__ double s_amp;
    T *lds = reinterpret_cast<T *>(smem);
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t t = b.persist ? atomicAdd(b.head, 1u) - b.head_base
                                         : b.ticket_base + (uint32_t)xcd_item((int)blockIdx.x, (int)gridDim.x);
            if (b.persist && t >= b.total) {
                s_tile = -1;
            } else {
                int lo = b.seg_first, hi = b.seg_first + b.nseg - 1;  // last segment starting at or before t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((uint32_t)b.seg_start[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                const int m = b.seg_mesh[lo];
                const TileArgs &a = args[m];
                const uint32_t local = (uint32_t)b.seg_local[lo] + (t - (uint32_t)b.seg_start[lo]);
                s_mesh = m;
                s_shot = (int)(local % (uint32_t)a.nshots);
                const TileMeta mt = tile_meta(a, (int)(local / (uint32_t)a.nshots));
                s_tile = mt.x;
                s_f0 = mt.y;
                s_nfoot = mt.z;
                s_b0 = mt.w;
                s_amp = b.amp_tab[(int64_t)m * b.amp_stride + (b.amp_base ? *b.amp_base : 0) + b.amp_idx];
            }
        }
        __syncthreads();
        // the item is the same for the whole workgroup: scalar registers
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);
        if (tile < 0) return;
        const int mesh = __builtin_amdgcn_readfirstlane(s_mesh);
        const int shot = __builtin_amdgcn_readfirstlane(s_shot);
        const TileArgs &a = args[mesh];
        chain_tile<K, T, UPW, ORDER, O0, NOPS>(Rf, a, lds, tile, s_f0, s_nfoot, s_b0, shot, (T)s_amp, b.epoch);
        if (!b.persist) return;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = a.succ_off[tile]; k < a.succ_off[tile + 1]; ++k)
                __hip_atomic_fetch_add(a.cnt + (int64_t)shot * a.ntiles + a.succ[k], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
// args: the members' launch arguments (b.args), a separate read-only, non-aliased
// kernel argument so that the compiler loads their fields into scalar registers
__global__ __launch_bounds__(NT) void k_tile_chain_batch(const BatchArgs b, const TileArgs *__restrict__ args) {
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (K <= 2 && UPW) {  // reference matrices in LDS, as in the single-mesh kernel
        __shared__ __align__(16) RefC<K, T> sref;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&R<K, T>());
        uint32_t *dst = reinterpret_cast<uint32_t *>(&sref);
        for (int i = threadIdx.x; i < (int)(sizeof(RefC<K, T>) / 4); i += NT) dst[i] = src[i];
        __syncthreads();
        batch_body<K, T, UPW, ORDER, O0, NOPS, NT>(sref, b, args, smem);
    } else {
        batch_body<K, T, UPW, ORDER, O0, NOPS, NT>(R<K, T>(), b, args, smem);
    }
}

}  // namespace dgt
