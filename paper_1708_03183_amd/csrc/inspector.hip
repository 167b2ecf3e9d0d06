// GPU sparse-tiling inspector (Sec. 5.1; Alg. 1, Alg. 3, Alg. 4) for gfx950.
//
// Every step is a deterministic function of the chain: sorts use unique keys,
// maxima use the packed key (colour+1)<<32 | tile, and colouring is a
// Jones-Plassmann sweep whose result depends only on the tile graph.  The
// schedule is therefore bit-identical to any other implementation of the same
// definition (the tests compare it with an independent CPU inspector).
//
// Readings where the paper leaves room:
//  * a projection starts from the previous projection of its set and is only
//    raised (never reset), for every descriptor whatever its mode;
//  * sigma_j starts at bottom once and is the MAX over all descriptors/slots;
//    an iteration left at bottom goes to the first tile of colour 0;
//  * projections are emptied at the start of each conflict round;
//  * two different tiles of one colour touching a common element of any set,
//    in any loops of the (sub-)chain, conflict: each pair becomes a fake edge;
//  * tiles are adjacent when a map into the seed set joins their iterations,
//    or a map from the seed set sends two of their iterations to one element;
//  * colouring priority is (fmix32(t), t), fmix32 the MurmurHash3 finaliser;
//  * seed order 1 = Hilbert index of coordinates quantised to 2^16 per axis.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce_by_key.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <sstream>

#include "common.h"
#include "inspector.h"

namespace dgt {

// ----------------------------------------------------------------- kernels

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint64_t tile_key(const int32_t *color, int32_t t) {
    return ((uint64_t)(uint32_t)(color[t] + 1) << 32) | (uint32_t)t;
}

// Hilbert curve index on a 2^16 grid: quadrant digit per level, then the
// sub-square is reflected/transposed so the curve stays continuous.
__device__ uint64_t hilbert16(uint32_t x, uint32_t y) {
    uint64_t d = 0;
#pragma unroll 1
    for (int lvl = 15; lvl >= 0; --lvl) {
        const uint32_t half = 1u << lvl;
        const uint32_t qx = (x >> lvl) & 1u, qy = (y >> lvl) & 1u;
        d += ((uint64_t)half * half) * ((3u * qx) ^ qy);
        const uint32_t mask = half - 1u;
        x &= mask;
        y &= mask;
        if (!qy) {
            if (qx) {
                x = mask - x;
                y = mask - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

// bounding box of n points: each block reduces a grid-stride share of the points to
// (min x, max x, min y, max y) in part[4 * block]; k_minmax_final reduces the parts
// (min and max are exact, so the result does not depend on the grid)
__device__ __forceinline__ void minmax_block(double (&v)[4]) {
    __shared__ double s[4][256];
    for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    for (int q = 0; q < 4; ++q) v[q] = s[q][0];
}

__global__ __launch_bounds__(256) void k_minmax_part(const double *__restrict__ xy, int64_t n,
                                                     double *__restrict__ part) {
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = xy[2 * i], b = xy[2 * i + 1];
        v[0] = fmin(v[0], a);
        v[1] = fmax(v[1], a);
        v[2] = fmin(v[2], b);
        v[3] = fmax(v[3], b);
    }
    minmax_block(v);
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = v[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_minmax_final(const double *__restrict__ part, int nparts,
                                                      double *__restrict__ out4) {
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        v[0] = fmin(v[0], part[4 * b]);
        v[1] = fmax(v[1], part[4 * b + 1]);
        v[2] = fmin(v[2], part[4 * b + 2]);
        v[3] = fmax(v[3], part[4 * b + 3]);
    }
    minmax_block(v);
    if (threadIdx.x < 4) out4[threadIdx.x] = v[threadIdx.x];
}

__device__ uint32_t quantise16(double v, double lo, double hi) {
    const double ext = __dsub_rn(hi, lo);
    if (!(ext > 0.0)) return 0u;
    const double q = floor(__dmul_rn(__ddiv_rn(__dsub_rn(v, lo), ext), 65536.0));
    return q >= 65535.0 ? 65535u : (uint32_t)q;
}

__global__ void k_hilbert_keys(const double *__restrict__ xy, int64_t n, const double *__restrict__ box,
                               uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t qx = quantise16(xy[2 * i], box[0], box[1]);
    const uint32_t qy = quantise16(xy[2 * i + 1], box[2], box[3]);
    keys[i] = (hilbert16(qx, qy) << 32) | (uint64_t)i;
}

__global__ void k_tile0_from_sorted(const uint64_t *__restrict__ sorted, int64_t n, int64_t ts,
                                    int32_t *__restrict__ tile0, int32_t *__restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = (int64_t)(sorted[p] & 0xffffffffull);
    tile0[i] = (int32_t)(p / ts);
    if (rank) rank[i] = (int32_t)p;
}

__global__ void k_tile0_identity(int64_t n, int64_t ts, int32_t *__restrict__ tile0, int32_t *__restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tile0[i] = (int32_t)(i / ts);
    if (rank) rank[i] = (int32_t)i;
}

// regions (Sec. 3.3, 5.1.2): keys (region << 32 | seed rank), sorted to give the
// seeds of each region in seed order
__global__ void k_region_keys(const uint8_t *__restrict__ region, const int32_t *__restrict__ rank, int64_t n,
                              uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = ((uint64_t)region[i] << 32) | (uint32_t)rank[i];
}

__global__ void k_rank_order(const int32_t *__restrict__ rank, int64_t n, int32_t *__restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) order[rank[i]] = (int32_t)i;
}

// blocks of ts seeds per region: core tiles from 0, boundary tiles from ncore, and
// every non-exec seed in tile tne
__global__ void k_tile0_regions(const uint64_t *__restrict__ sorted, int64_t n, const int32_t *__restrict__ order,
                                int64_t start1, int32_t ncore, int32_t tne, int64_t ts, int32_t *__restrict__ tile0) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t r = (uint32_t)(sorted[p] >> 32);
    const int32_t i = order[sorted[p] & 0xffffffffull];
    tile0[i] = r == 2 ? tne : (r == 1 ? ncore + (int32_t)((p - start1) / ts) : (int32_t)(p / ts));
}

// one halo exchange per chain: seeds written by an iteration of T_ne become stale
__global__ void k_stale(const int32_t *__restrict__ sigma, int64_t n, int32_t tne, const int32_t *__restrict__ map,
                        int arity, uint8_t *__restrict__ region) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= n || sigma[it] != tne) return;
    if (!map) region[it] = 2;
    else
        for (int k = 0; k < arity; ++k) region[map[it * arity + k]] = 2;
}

// inverse map (Fig. 8): keys (target<<32 | source)
__global__ void k_inv_keys(const int32_t *__restrict__ vals, int64_t nsrc, int arity, uint64_t *__restrict__ keys,
                           int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsrc * arity) return;
    const int32_t tgt = vals[i];
    keys[i] = ((uint64_t)(uint32_t)tgt << 32) | (uint64_t)(i / arity);
    atomicAdd(&count[tgt], 1);
}

__global__ void k_low32(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)(keys[i] & 0xffffffffull);
}

// CSR offsets of keys sorted by their high word (each < ngroups): off[g] is the first
// position whose high word is >= g.  Thread i (0..n) writes the offsets of the groups
// that start at i, so every offset is written once, without atomics.
__global__ void k_sorted_offsets(const uint64_t *__restrict__ keys, int64_t n, int64_t ngroups,
                                 int32_t *__restrict__ off) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t lo = i == 0 ? 0 : (int64_t)(keys[i - 1] >> 32) + 1;
    const int64_t hi = i == n ? ngroups : min((int64_t)(keys[i] >> 32), ngroups);  // stays in bounds
    for (int64_t g = lo; g <= hi; ++g) off[g] = (int32_t)i;
}

// tile pairs through a map into the seed set: all pairs of slots of one source
__global__ void k_adj_into(const int32_t *__restrict__ vals, int64_t nsrc, int arity,
                           const int32_t *__restrict__ tile0, uint64_t *__restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    int64_t w = s * (int64_t)(arity * (arity - 1) / 2);
    for (int a = 0; a < arity; ++a)
        for (int b = a + 1; b < arity; ++b) {
            int32_t t1 = tile0[vals[s * arity + a]], t2 = tile0[vals[s * arity + b]];
            if (t1 > t2) { const int32_t t = t1; t1 = t2; t2 = t; }
            out[w++] = (t1 == t2) ? ~0ull : (((uint64_t)(uint32_t)t1 << 32) | (uint32_t)t2);
        }
}

// pair counts per target of a map from the seed set
__global__ void k_adj_from_count(const int32_t *__restrict__ off, int64_t ntgt, int64_t *__restrict__ cnt) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ntgt) return;
    const int64_t d = off[x + 1] - off[x];
    cnt[x] = d * (d - 1) / 2;
}

__global__ void k_adj_from(const int32_t *__restrict__ off, const int32_t *__restrict__ val, int64_t ntgt,
                           const int64_t *__restrict__ pos, const int32_t *__restrict__ tile0,
                           uint64_t *__restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= ntgt) return;
    int64_t w = pos[x];
    for (int32_t a = off[x]; a < off[x + 1]; ++a)
        for (int32_t b = a + 1; b < off[x + 1]; ++b) {
            int32_t t1 = tile0[val[a]], t2 = tile0[val[b]];
            if (t1 > t2) { const int32_t t = t1; t1 = t2; t2 = t; }
            out[w++] = (t1 == t2) ? ~0ull : (((uint64_t)(uint32_t)t1 << 32) | (uint32_t)t2);
        }
}

__global__ void k_sym_edges(const uint64_t *__restrict__ e, int64_t n, uint64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t a = e[i] >> 32, b = e[i] & 0xffffffffull;
    out[2 * i] = (a << 32) | b;
    out[2 * i + 1] = (b << 32) | a;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Jones-Plassmann round, part 1: uncoloured local maxima of the priority
// (with tile regions treg, only neighbours in the tile's own region count)
__global__ void k_jp_mark(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                          const int32_t *__restrict__ color, int32_t n, int8_t *__restrict__ mark,
                          const uint8_t *__restrict__ treg) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int8_t m = 0;
    if (color[t] < 0) {
        const uint64_t pt = ((uint64_t)fmix32((uint32_t)t) << 32) | (uint32_t)t;
        m = 1;
        for (int32_t k = off[t]; k < off[t + 1]; ++k) {
            const int32_t u = adj[k];
            if (color[u] >= 0 || (treg && treg[u] != treg[t])) continue;
            const uint64_t pu = ((uint64_t)fmix32((uint32_t)u) << 32) | (uint32_t)u;
            if (pu > pt) { m = 0; break; }
        }
    }
    mark[t] = m;
}

// part 2: each marked tile takes the smallest colour unused by coloured neighbours
__global__ void k_jp_assign(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                            int32_t *__restrict__ color, int32_t n, const int8_t *__restrict__ mark,
                            int32_t *__restrict__ stats /* [0] coloured this round, [1] max colour, [2] overflow */,
                            const uint8_t *__restrict__ treg) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || !mark[t]) return;
    uint64_t used = 0;
    for (int32_t k = off[t]; k < off[t + 1]; ++k) {
        if (treg && treg[adj[k]] != treg[t]) continue;
        const int32_t c = color[adj[k]];
        if (c >= 64) atomicExch(&stats[2], 1);
        else if (c >= 0) used |= 1ull << c;
    }
    const int col = (~used == 0ull) ? 64 : __ffsll((unsigned long long)~used) - 1;
    if (col >= 64) { atomicExch(&stats[2], 1); return; }
    color[t] = col;
    atomicAdd(&stats[0], 1);
    atomicMax(&stats[1], col);
}

__global__ void k_first_color0(const int32_t *__restrict__ color, int32_t n, int32_t *__restrict__ out) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && color[t] == 0) atomicMin(out, t);
}

// Alg. 3, direct descriptor: phi = max(phi_prev, key(sigma))
__global__ void k_proj_direct(uint64_t *__restrict__ phi, int has_prev, const int32_t *__restrict__ sigma,
                              const int32_t *__restrict__ color, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t k = tile_key(color, sigma[e]);
    const uint64_t p = has_prev ? phi[e] : 0ull;
    phi[e] = k > p ? k : p;
}

// Alg. 3, indirect descriptor: gather-max through the inverse map
__global__ void k_proj_indirect(uint64_t *__restrict__ phi, int has_prev, const int32_t *__restrict__ inv_off,
                                const int32_t *__restrict__ inv_val, const int32_t *__restrict__ sigma,
                                const int32_t *__restrict__ color, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint64_t best = has_prev ? phi[e] : 0ull;
    for (int32_t a = inv_off[e]; a < inv_off[e + 1]; ++a) {
        const uint64_t k = tile_key(color, sigma[inv_val[a]]);
        best = k > best ? k : best;
    }
    phi[e] = best;
}

struct TileDesc {
    const uint64_t *phi;   // projection of the target set (nullptr: none yet)
    const int32_t *map;    // nullptr: direct
    int32_t arity;
};

struct LoopTilingArgs {
    int32_t nd;
    TileDesc d[8];
};

// Alg. 4: sigma_j[e] = MAX over descriptors and slots of the projections
__global__ void k_tile_loop(LoopTilingArgs a, int64_t n, const int32_t *__restrict__ deft, int32_t *__restrict__ sigma) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint64_t best = 0;
    for (int i = 0; i < a.nd; ++i) {
        const TileDesc &D = a.d[i];
        if (!D.phi) continue;
        if (!D.map) {
            const uint64_t v = D.phi[e];
            best = v > best ? v : best;
        } else {
            for (int k = 0; k < D.arity; ++k) {
                const uint64_t v = D.phi[D.map[e * D.arity + k]];
                best = v > best ? v : best;
            }
        }
    }
    sigma[e] = best ? (int32_t)(best & 0xffffffffull) : *deft;
}

// touches of one set: (element<<32 | tile) with loop bit
__global__ void k_touch(const int32_t *__restrict__ sigma, const int32_t *__restrict__ map, int arity, int64_t n,
                        uint32_t bit, uint64_t *__restrict__ keys, uint32_t *__restrict__ bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * arity) return;
    const int64_t it = i / arity;
    const uint32_t x = map ? (uint32_t)map[i] : (uint32_t)it;
    keys[i] = ((uint64_t)x << 32) | (uint32_t)sigma[it];
    bits[i] = bit;
}

// conflicts among the unique (element, tile) touches of one set
__global__ void k_conflicts(const uint64_t *__restrict__ keys, int64_t n, const int32_t *__restrict__ color,
                            uint64_t *__restrict__ out, int64_t cap, unsigned long long *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = keys[i] >> 32;
    const int32_t ti = (int32_t)(keys[i] & 0xffffffffull);
    for (int64_t j = i + 1; j < n && (keys[j] >> 32) == x; ++j) {
        const int32_t tj = (int32_t)(keys[j] & 0xffffffffull);
        if (color[ti] == color[tj]) {
            const unsigned long long w = atomicAdd(count, 1ull);
            const int32_t a = ti < tj ? ti : tj, b = ti < tj ? tj : ti;
            if ((int64_t)w < cap) out[w] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
        }
    }
}

// dependence edges among the tiles that share one element: every pair of entries of
// one group of the sorted unique (element<<32 | tile) touches; count pass, then emit
// pass oriented from the lower colour to the higher (equal colours flag an error)
__global__ void k_dep_count(const uint64_t *__restrict__ keys, int64_t n, int64_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = keys[i] >> 32;
    int64_t c = 0;
    for (int64_t j = i + 1; j < n && (keys[j] >> 32) == x; ++j) ++c;
    cnt[i] = c;
}

__global__ void k_dep_emit(const uint64_t *__restrict__ keys, int64_t n, const int64_t *__restrict__ pos,
                           const int32_t *__restrict__ color, uint64_t *__restrict__ out, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = keys[i] >> 32;
    const uint32_t ti = (uint32_t)(keys[i] & 0xffffffffull);
    int64_t w = pos[i];
    for (int64_t j = i + 1; j < n && (keys[j] >> 32) == x; ++j) {
        const uint32_t tj = (uint32_t)(keys[j] & 0xffffffffull);
        if (color[ti] == color[tj]) *bad = 1;
        const bool lo = color[ti] < color[tj];
        out[w++] = ((uint64_t)(lo ? ti : tj) << 32) | (lo ? tj : ti);
    }
}

__global__ void k_low32_hist(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&count[(int32_t)(keys[i] & 0xffffffffull)], 1);
}

// footprint entries: re-key to (tile<<32 | element) and flag single-tile elements
__global__ void k_foot_rekey(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ bits, int64_t n,
                             uint64_t *__restrict__ okeys, uint32_t *__restrict__ obits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = keys[i] >> 32;
    const bool single = (i == 0 || (keys[i - 1] >> 32) != x) && (i + 1 == n || (keys[i + 1] >> 32) != x);
    okeys[i] = ((keys[i] & 0xffffffffull) << 32) | x;
    obits[i] = bits[i] | (single ? 0x80000000u : 0u);
}

__global__ void k_sigma_keys(const int32_t *__restrict__ sigma, int64_t n, uint64_t *__restrict__ keys) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) keys[e] = ((uint64_t)(uint32_t)sigma[e] << 32) | (uint64_t)e;
}

__global__ void k_color_keys(const int32_t *__restrict__ color, int32_t n, uint64_t *__restrict__ keys) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) keys[t] = ((uint64_t)(uint32_t)color[t] << 32) | (uint32_t)t;
}

// ----------------------------------------------------------------- primitives

struct BitOr {
    __device__ __forceinline__ uint32_t operator()(uint32_t a, uint32_t b) const { return a | b; }
};

void sort_keys(DBuf<uint64_t> &keys, int64_t n, hipStream_t st, int end_bit) {
    if (n <= 1) return;
    DBuf<uint64_t> out(n);
    size_t tmp = 0;
    DGT_HIP(rocprim::radix_sort_keys(nullptr, tmp, keys.p, out.p, (size_t)n, 0u, (unsigned)end_bit, st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::radix_sort_keys(t.p, tmp, keys.p, out.p, (size_t)n, 0u, (unsigned)end_bit, st));
    keys = std::move(out);
}

void sort_pairs(DBuf<uint64_t> &keys, DBuf<uint32_t> &vals, int64_t n, hipStream_t st) {
    if (n <= 1) return;
    DBuf<uint64_t> ko(n);
    DBuf<uint32_t> vo(n);
    size_t tmp = 0;
    DGT_HIP(rocprim::radix_sort_pairs(nullptr, tmp, keys.p, ko.p, vals.p, vo.p, (size_t)n, 0u, 64u, st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::radix_sort_pairs(t.p, tmp, keys.p, ko.p, vals.p, vo.p, (size_t)n, 0u, 64u, st));
    keys = std::move(ko);
    vals = std::move(vo);
}

// unique keys; returns count (sentinel ~0 entries dropped)
static int64_t unique_keys(DBuf<uint64_t> &keys, int64_t n, hipStream_t st) {
    if (n == 0) return 0;
    DBuf<uint64_t> out(n);
    DBuf<int64_t> cnt(1);
    size_t tmp = 0;
    DGT_HIP(rocprim::unique(nullptr, tmp, keys.p, out.p, cnt.p, (size_t)n, rocprim::equal_to<uint64_t>(), st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::unique(t.p, tmp, keys.p, out.p, cnt.p, (size_t)n, rocprim::equal_to<uint64_t>(), st));
    int64_t m = cnt.download(st)[0];
    if (m > 0) {
        uint64_t last;
        DGT_HIP(hipMemcpyAsync(&last, out.p + m - 1, 8, hipMemcpyDeviceToHost, st));
        DGT_HIP(hipStreamSynchronize(st));
        if (last == ~0ull) m--;
    }
    keys = std::move(out);
    return m;
}

static void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t st) {
    size_t tmp = 0;
    DGT_HIP(rocprim::exclusive_scan(nullptr, tmp, in, out, int32_t(0), (size_t)n, rocprim::plus<int32_t>(), st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::exclusive_scan(t.p, tmp, in, out, int32_t(0), (size_t)n, rocprim::plus<int32_t>(), st));
}

static void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st) {
    size_t tmp = 0;
    DGT_HIP(rocprim::exclusive_scan(nullptr, tmp, in, out, int64_t(0), (size_t)n, rocprim::plus<int64_t>(), st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::exclusive_scan(t.p, tmp, in, out, int64_t(0), (size_t)n, rocprim::plus<int64_t>(), st));
}

// counts [n] -> offsets [n+1] (exclusive scan with total at the end)
static void counts_to_offsets(DBuf<int32_t> &cnt, int64_t n, DBuf<int32_t> &off, hipStream_t st) {
    off.alloc(n + 1);
    if (n == 0) {
        DGT_HIP(hipMemsetAsync(off.p, 0, sizeof(int32_t), st));
        return;
    }
    DBuf<int32_t> tmp(n + 1);
    DGT_HIP(hipMemsetAsync(tmp.p + n, 0, sizeof(int32_t), st));
    DGT_HIP(hipMemcpyAsync(tmp.p, cnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    exclusive_scan_i32(tmp.p, off.p, n + 1, st);
}

// CSR offsets of sorted (high32 << 32 | low32) keys grouped by the high word
static void offsets_by_high(const DBuf<uint64_t> &keys, int64_t n, int64_t ngroups, DBuf<int32_t> &off,
                            hipStream_t st) {
    off.alloc(ngroups + 1);
    k_sorted_offsets<<<blocks_for(n + 1, 256), 256, 0, st>>>(keys.p, n, ngroups, off.p);
}

// ----------------------------------------------------------------- host driver

void Inspector::build_inverse(const ChainDesc &c, int mi, hipStream_t st) {
    const ChainMap &m = c.maps[mi];
    const int64_t ns = c.size[m.from], nt = c.size[m.to];
    const int64_t n = ns * m.arity;
    DBuf<uint64_t> keys(n > 0 ? n : 1);
    DBuf<int32_t> cnt(nt + 1);
    DGT_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (nt + 1), st));
    if (n) k_inv_keys<<<blocks_for(n, 256), 256, 0, st>>>(dmap[mi].p, ns, m.arity, keys.p, cnt.p);
    sort_keys(keys, n, st);
    inv_val[mi].alloc(n > 0 ? n : 1);
    if (n) k_low32<<<blocks_for(n, 256), 256, 0, st>>>(keys.p, n, inv_val[mi].p);
    counts_to_offsets(cnt, nt, inv_off[mi], st);
}

Inspector::Inspector(const ChainDesc &c, hipStream_t st) : chain(c), stream(st) {
    for (int mi = 0; mi < c.nmaps; ++mi) {
        dmap[mi].upload(c.maps[mi].values, st);
        build_inverse(c, mi, st);
    }
}

namespace {

struct SubRun {
    int first, n;
    int64_t n0;
    int32_t ntiles;
};

}  // namespace

void Inspector::seed_partition(int seedset, int64_t ts, int partition, const double *seed_xy_host,
                               const double *seed_xy_dev, DBuf<int32_t> &tile0, DBuf<int32_t> &rank) {
    hipStream_t st = stream;
    const int64_t n0 = chain.size[seedset];
    tile0.alloc(n0 > 0 ? n0 : 1);
    rank.alloc(n0 > 0 ? n0 : 1);
    if (n0 == 0) return;
    if (partition == 0) {
        k_tile0_identity<<<blocks_for(n0, 256), 256, 0, st>>>(n0, ts, tile0.p, rank.p);
        return;
    }
    DBuf<double> xy_owned;
    const double *xy = seed_xy_dev;
    if (!xy) {
        DGT_REQUIRE(seed_xy_host, DGT_EINVAL, "partition 1 needs seed_xy");
        xy_owned.upload(seed_xy_host, 2 * n0, st);
        xy = xy_owned.p;
    }
    DBuf<double> box(4);
    {
        const int nparts = (int)std::min<int64_t>(1024, blocks_for(n0, 256));
        DBuf<double> part(4 * nparts);
        k_minmax_part<<<nparts, 256, 0, st>>>(xy, n0, part.p);
        k_minmax_final<<<1, 256, 0, st>>>(part.p, nparts, box.p);
    }
    DBuf<uint64_t> keys(n0);
    k_hilbert_keys<<<blocks_for(n0, 256), 256, 0, st>>>(xy, n0, box.p, keys.p);
    sort_keys(keys, n0, st);
    k_tile0_from_sorted<<<blocks_for(n0, 256), 256, 0, st>>>(keys.p, n0, ts, tile0.p, rank.p);
}

// Seed partition with regions (Sec. 5.1.2): the seeds of each region in seed
// order, cut into blocks of ts; core tiles first, then boundary tiles, then T_ne.
void Inspector::region_partition(int64_t n0, int64_t ts, const DBuf<int32_t> &rank, SubSched &sb,
                                 DBuf<int32_t> &tile0) {
    hipStream_t st = stream;
    int64_t cnt[3] = {0, 0, 0};
    for (int64_t i = 0; i < n0; ++i) cnt[sb.region[i]]++;
    sb.ncore = (int32_t)((cnt[0] + ts - 1) / ts);
    sb.nbnd = (int32_t)((cnt[1] + ts - 1) / ts);
    sb.tne = sb.ncore + sb.nbnd;
    if (n0 == 0) return;
    DBuf<uint8_t> reg;
    reg.upload(sb.region, st);
    DBuf<uint64_t> keys(n0);
    DBuf<int32_t> order(n0);
    k_region_keys<<<blocks_for(n0, 256), 256, 0, st>>>(reg.p, rank.p, n0, keys.p);
    k_rank_order<<<blocks_for(n0, 256), 256, 0, st>>>(rank.p, n0, order.p);
    sort_keys(keys, n0, st);
    k_tile0_regions<<<blocks_for(n0, 256), 256, 0, st>>>(keys.p, n0, order.p, cnt[0], sb.ncore, sb.tne, ts,
                                                          tile0.p);
}

int64_t Inspector::seed_edges(int first, int nl, const DBuf<int32_t> &tile0, DBuf<uint64_t> &edges) {
    hipStream_t st = stream;
    const int seed = chain.loops[first].set;
    bool used[8] = {false};
    for (int j = first; j < first + nl; ++j)
        for (int i = 0; i < chain.loops[j].ndesc; ++i)
            if (chain.loops[j].d[i].map >= 0) used[chain.loops[j].d[i].map] = true;
    std::vector<DBuf<uint64_t>> parts;
    std::vector<int64_t> lens;
    for (int mi = 0; mi < chain.nmaps; ++mi) {
        if (!used[mi]) continue;
        const ChainMap &m = chain.maps[mi];
        if (m.to == seed && m.arity >= 2) {
            const int64_t ns = chain.size[m.from];
            const int64_t np = ns * (m.arity * (m.arity - 1) / 2);
            DBuf<uint64_t> out(np > 0 ? np : 1);
            if (ns) k_adj_into<<<blocks_for(ns, 256), 256, 0, st>>>(dmap[mi].p, ns, m.arity, tile0.p, out.p);
            parts.push_back(std::move(out));
            lens.push_back(np);
        }
        if (m.from == seed) {
            const int64_t nt = chain.size[m.to];
            DBuf<int64_t> cnt(nt + 1), pos(nt + 1);
            DGT_HIP(hipMemsetAsync(cnt.p + nt, 0, sizeof(int64_t), st));
            if (nt) k_adj_from_count<<<blocks_for(nt, 256), 256, 0, st>>>(inv_off[mi].p, nt, cnt.p);
            exclusive_scan_i64(cnt.p, pos.p, nt + 1, st);
            const int64_t np = pos.download(st)[nt];
            DBuf<uint64_t> out(np > 0 ? np : 1);
            if (nt && np)
                k_adj_from<<<blocks_for(nt, 256), 256, 0, st>>>(inv_off[mi].p, inv_val[mi].p, nt, pos.p, tile0.p,
                                                                out.p);
            parts.push_back(std::move(out));
            lens.push_back(np);
        }
    }
    int64_t total = 0;
    for (auto l : lens) total += l;
    edges.alloc(total > 0 ? total : 1);
    int64_t w = 0;
    for (size_t i = 0; i < parts.size(); ++i) {
        if (lens[i])
            DGT_HIP(hipMemcpyAsync(edges.p + w, parts[i].p, sizeof(uint64_t) * lens[i], hipMemcpyDeviceToDevice, st));
        w += lens[i];
    }
    sort_keys(edges, total, st);
    return unique_keys(edges, total, st);
}

// Colour-class cap: one pass over the tiles in ascending id; a tile whose class
// holds more than cap tiles moves to the smallest colour holding fewer than cap
// tiles that none of its neighbours has, or to a new colour.  Every class then
// holds at most cap tiles and the colouring stays proper.  Sequential by nature
// (each move depends on the previous ones), so it runs on the host between the
// GPU colouring and the GPU tiling; returns the new number of colours.
static int cap_colour_classes(int32_t ntiles, const std::vector<int32_t> &off, const std::vector<int32_t> &adj,
                              std::vector<int32_t> &color, int ncol, int cap) {
    std::vector<int32_t> size(64, 0);
    for (int32_t t = 0; t < ntiles; ++t) size[color[t]]++;
    for (int32_t t = 0; t < ntiles; ++t) {
        const int c = color[t];
        if (size[c] <= cap) continue;
        uint64_t used = 0;
        for (int32_t k = off[t]; k < off[t + 1]; ++k) used |= 1ull << color[adj[k]];
        int c2 = 0;
        while (c2 < ncol && (c2 == c || size[c2] >= cap || ((used >> c2) & 1))) ++c2;
        if (c2 == ncol) {
            DGT_REQUIRE(ncol < 64, DGT_EUNSUPPORTED, "the colour-class cap needs more than 64 colours");
            ++ncol;
        }
        color[t] = c2;
        size[c]--;
        size[c2]++;
    }
    return ncol;
}

// Jones-Plassmann colouring of the tile graph given by unique edges (a<b),
// then the colour-class cap when cap > 0
int Inspector::colour(int32_t ntiles, const DBuf<uint64_t> &edges, int64_t ne, DBuf<int32_t> &color, int cap,
                      const SubSched *regions) {
    hipStream_t st = stream;
    // regions: each region's tiles are coloured on the edges inside it
    DBuf<uint8_t> treg;
    std::vector<uint8_t> treg_h;  // kept until the colouring has synchronised
    if (regions) {
        treg_h.resize(ntiles);
        for (int32_t t = 0; t < ntiles; ++t) treg_h[t] = t < regions->ncore ? 0 : (t < regions->tne ? 1 : 2);
        treg.upload(treg_h, st);
    }
    DBuf<uint64_t> sym(2 * ne > 0 ? 2 * ne : 1);
    if (ne) k_sym_edges<<<blocks_for(ne, 256), 256, 0, st>>>(edges.p, ne, sym.p);
    sort_keys(sym, 2 * ne, st);
    DBuf<int32_t> off, adj(2 * ne > 0 ? 2 * ne : 1);
    offsets_by_high(sym, 2 * ne, ntiles, off, st);
    if (ne) k_low32<<<blocks_for(2 * ne, 256), 256, 0, st>>>(sym.p, 2 * ne, adj.p);
    color.alloc(ntiles);
    k_fill_i32<<<blocks_for(ntiles, 256), 256, 0, st>>>(color.p, ntiles, -1);
    DBuf<int8_t> mark(ntiles);
    DBuf<int32_t> stats(3);
    DGT_HIP(hipMemsetAsync(stats.p, 0, sizeof(int32_t) * 3, st));
    int32_t done = 0;
    int guard_rounds = 0;
    while (done < ntiles) {
        // several rounds between host checks
        for (int r = 0; r < 8; ++r) {
            k_jp_mark<<<blocks_for(ntiles, 256), 256, 0, st>>>(off.p, adj.p, color.p, ntiles, mark.p, treg.p);
            k_jp_assign<<<blocks_for(ntiles, 256), 256, 0, st>>>(off.p, adj.p, color.p, ntiles, mark.p, stats.p,
                                                                 treg.p);
        }
        auto h = stats.download(st);
        DGT_REQUIRE(h[2] == 0, DGT_EUNSUPPORTED, "tile colouring needs more than 64 colours");
        done = h[0];
        DGT_REQUIRE(++guard_rounds < 1000000, DGT_ESTATE, "colouring did not terminate");
        if (done >= ntiles) {
            int ncol = h[1] + 1;
            if (regions) {  // boundary colours after the core ones, T_ne alone on top
                auto hc = color.download(st, ntiles);
                int ccore = 0, cbnd = 0;
                for (int32_t t = 0; t < ntiles; ++t) {
                    if (t < regions->ncore) ccore = std::max(ccore, hc[t] + 1);
                    else if (t < regions->tne) cbnd = std::max(cbnd, hc[t] + 1);
                }
                for (int32_t t = regions->ncore; t < ntiles; ++t) hc[t] = t < regions->tne ? hc[t] + ccore : ccore + cbnd;
                ncol = ccore + cbnd + 1;
                DGT_REQUIRE(ncol <= 64, DGT_EUNSUPPORTED, "tile colouring needs more than 64 colours");
                color.upload(hc, st);
                return ncol;
            }
            if (cap > 0) {
                auto hc = color.download(st, ntiles);
                auto ho = off.download(st, ntiles + 1);
                auto ha = adj.download(st, 2 * ne > 0 ? 2 * ne : 1);
                ncol = cap_colour_classes(ntiles, ho, ha, hc, ncol, cap);
                color.upload(hc, st);
            }
            return ncol;
        }
    }
    return 0;
}

void Inspector::run_sub(Schedule &S, SubSched &sb, int64_t ts, int partition, const double *xy_host,
                        const double *xy_dev, int max_rounds, int cap) {
    hipStream_t st = stream;
    const int first = sb.first, nl = sb.n;
    const int seedset = chain.loops[first].set;
    const int64_t n0 = chain.size[seedset];
    int32_t ntiles = (int32_t)((n0 + ts - 1) / ts);
    if (ntiles == 0) ntiles = 1;
    DBuf<int32_t> tile0, rank;
    seed_partition(seedset, ts, partition, xy_host, xy_dev, tile0, rank);
    const bool regions = sb.tne >= 0;
    if (regions) {
        region_partition(n0, ts, rank, sb, tile0);
        ntiles = sb.tne + 1;
    }
    if (first == 0 || !S.seed_rank.p) {
        S.seed_rank = std::move(rank);
        S.seed_set = seedset;
    }
    DBuf<uint64_t> edges;
    int64_t ne = seed_edges(first, nl, tile0, edges);
    DBuf<int32_t> deft(1);
    // per-set projection buffers
    DBuf<uint64_t> phi[8];
    for (int s = 0; s < chain.nsets; ++s) phi[s].alloc(chain.size[s] > 0 ? chain.size[s] : 1);
    int round = 0, ncol = 0;
    for (; round < max_rounds; ++round) {
        ncol = colour(ntiles, edges, ne, sb.color, cap, regions ? &sb : nullptr);
        // default tile: first tile of colour 0
        int32_t big = INT32_MAX;
        DGT_HIP(hipMemcpyAsync(deft.p, &big, 4, hipMemcpyHostToDevice, st));
        k_first_color0<<<blocks_for(ntiles, 256), 256, 0, st>>>(sb.color.p, ntiles, deft.p);
        // sigma_seed = partition
        if (n0)
            DGT_HIP(hipMemcpyAsync(S.sigma[first].p, tile0.p, sizeof(int32_t) * n0, hipMemcpyDeviceToDevice, st));
        bool has[8] = {false};
        for (int j = first + 1; j < first + nl; ++j) {
            // project L_{j-1} (Alg. 3) for every distinct (target set, map) descriptor
            const ChainLoop &Lp = chain.loops[j - 1];
            const int64_t np_ = chain.size[Lp.set];
            int seen[16][2];
            int nseen = 0;
            for (int i = 0; i < Lp.ndesc; ++i) {
                const int mp = Lp.d[i].map;
                const int S_ = mp < 0 ? Lp.set : chain.maps[mp].to;
                bool dup = false;
                for (int q = 0; q < nseen; ++q) dup |= (seen[q][0] == S_ && seen[q][1] == mp);
                if (dup) continue;
                seen[nseen][0] = S_;
                seen[nseen][1] = mp;
                nseen++;
                const int64_t nS = chain.size[S_];
                if (nS == 0) { has[S_] = true; continue; }
                if (mp < 0) {
                    k_proj_direct<<<blocks_for(nS, 256), 256, 0, st>>>(phi[S_].p, has[S_] ? 1 : 0,
                                                                       S.sigma[j - 1].p, sb.color.p, nS);
                } else {
                    k_proj_indirect<<<blocks_for(nS, 256), 256, 0, st>>>(phi[S_].p, has[S_] ? 1 : 0,
                                                                         inv_off[mp].p, inv_val[mp].p,
                                                                         S.sigma[j - 1].p, sb.color.p, nS);
                }
                (void)np_;
                has[S_] = true;
            }
            // tile L_j (Alg. 4)
            const ChainLoop &L = chain.loops[j];
            LoopTilingArgs ta{};
            ta.nd = 0;
            for (int i = 0; i < L.ndesc; ++i) {
                const int mp = L.d[i].map;
                const int S_ = mp < 0 ? L.set : chain.maps[mp].to;
                TileDesc d;
                d.phi = has[S_] ? phi[S_].p : nullptr;
                d.map = mp < 0 ? nullptr : dmap[mp].p;
                d.arity = mp < 0 ? 1 : chain.maps[mp].arity;
                ta.d[ta.nd++] = d;
            }
            const int64_t nj = chain.size[L.set];
            if (nj) k_tile_loop<<<blocks_for(nj, 256), 256, 0, st>>>(ta, nj, deft.p, S.sigma[j].p);
        }
        // conflicts (all sets, all loops of the sub-chain)
        int64_t nconf = conflicts(first, nl, sb.color, edges, ne);
        if (nconf == 0) break;
    }
    DGT_REQUIRE(round < max_rounds, DGT_ESTATE, "inspector exceeded max_conflict_rounds");
    sb.ntiles = ntiles;
    sb.ncolors = ncol;
    sb.rounds = round + 1;
    footprints(first, nl, sb);
    // tiles in execution order
    {
        DBuf<uint64_t> keys(ntiles);
        k_color_keys<<<blocks_for(ntiles, 256), 256, 0, st>>>(sb.color.p, ntiles, keys.p);
        sort_keys(keys, ntiles, st);
        sb.tiles_by_color.alloc(ntiles);
        k_low32<<<blocks_for(ntiles, 256), 256, 0, st>>>(keys.p, ntiles, sb.tiles_by_color.p);
        offsets_by_high(keys, ntiles, ncol, sb.color_off, st);
    }
    // iteration lists (assign)
    for (int j = first; j < first + nl; ++j) {
        const int64_t nj = chain.size[chain.loops[j].set];
        DBuf<uint64_t> keys(nj > 0 ? nj : 1);
        if (nj) k_sigma_keys<<<blocks_for(nj, 256), 256, 0, st>>>(S.sigma[j].p, nj, keys.p);
        sort_keys(keys, nj, st);
        S.iters[j].alloc(nj > 0 ? nj : 1);
        if (nj) k_low32<<<blocks_for(nj, 256), 256, 0, st>>>(keys.p, nj, S.iters[j].p);
        offsets_by_high(keys, nj, ntiles, S.it_off[j], st);
    }
}

// unique (element<<32|tile) touches of set s with OR-ed loop bits
int64_t Inspector::touches(int first, int nl, int s, DBuf<uint64_t> &keys, DBuf<uint32_t> &bits,
                           const Schedule &S) {
    hipStream_t st = stream;
    int64_t total = 0;
    struct Item { int j, map; int arity; int64_t n; };
    std::vector<Item> items;
    for (int j = first; j < first + nl; ++j) {
        const ChainLoop &L = chain.loops[j];
        int seen[8], nseen = 0;
        for (int i = 0; i < L.ndesc; ++i) {
            const int mp = L.d[i].map;
            const int S_ = mp < 0 ? L.set : chain.maps[mp].to;
            if (S_ != s) continue;
            bool dup = false;
            for (int q = 0; q < nseen; ++q) dup |= seen[q] == mp;
            if (dup) continue;
            seen[nseen++] = mp;
            const int ar = mp < 0 ? 1 : chain.maps[mp].arity;
            items.push_back({j, mp, ar, chain.size[L.set]});
            total += chain.size[L.set] * ar;
        }
    }
    keys.alloc(total > 0 ? total : 1);
    bits.alloc(total > 0 ? total : 1);
    int64_t w = 0;
    for (auto &it : items) {
        const int64_t m = it.n * it.arity;
        if (m)
            k_touch<<<blocks_for(m, 256), 256, 0, st>>>(S.sigma[it.j].p, it.map < 0 ? nullptr : dmap[it.map].p,
                                                        it.arity, it.n, 1u << (it.j - first), keys.p + w, bits.p + w);
        w += m;
    }
    if (total == 0) return 0;
    sort_pairs(keys, bits, total, st);
    // reduce by key (OR of bits)
    DBuf<uint64_t> uk(total);
    DBuf<uint32_t> ub(total);
    DBuf<int64_t> cnt(1);
    size_t tmp = 0;
    DGT_HIP(rocprim::reduce_by_key(nullptr, tmp, keys.p, bits.p, (size_t)total, uk.p, ub.p, cnt.p, BitOr(),
                                   rocprim::equal_to<uint64_t>(), st));
    DBuf<char> t(tmp);
    DGT_HIP(rocprim::reduce_by_key(t.p, tmp, keys.p, bits.p, (size_t)total, uk.p, ub.p, cnt.p, BitOr(),
                                   rocprim::equal_to<uint64_t>(), st));
    const int64_t m = cnt.download(st)[0];
    keys = std::move(uk);
    bits = std::move(ub);
    return m;
}

int64_t Inspector::conflicts(int first, int nl, const DBuf<int32_t> &color, DBuf<uint64_t> &edges, int64_t &ne) {
    hipStream_t st = stream;
    std::vector<DBuf<uint64_t>> found;
    std::vector<int64_t> nfound;
    int64_t total = 0;
    tk_valid = false;
    for (int s = 0; s < chain.nsets; ++s) {
        DBuf<uint64_t> &keys = tk_keys[s];
        DBuf<uint32_t> &bits = tk_bits[s];
        const int64_t m = touches(first, nl, s, keys, bits, *cur);
        tk_len[s] = m;
        if (m == 0) continue;
        int64_t cap = std::max<int64_t>(1024, m);
        for (;;) {
            DBuf<uint64_t> out(cap);
            DBuf<unsigned long long> cnt(1);
            DGT_HIP(hipMemsetAsync(cnt.p, 0, 8, st));
            k_conflicts<<<blocks_for(m, 256), 256, 0, st>>>(keys.p, m, color.p, out.p, cap, cnt.p);
            const int64_t c = (int64_t)cnt.download(st)[0];
            if (c <= cap) {
                if (c) {
                    found.push_back(std::move(out));
                    nfound.push_back(c);
                    total += c;
                }
                break;
            }
            cap = c;
        }
    }
    tk_valid = true;
    if (total == 0) return 0;
    // fake connections: edges <- unique(edges U conflicts)
    DBuf<uint64_t> all(ne + total);
    if (ne) DGT_HIP(hipMemcpyAsync(all.p, edges.p, sizeof(uint64_t) * ne, hipMemcpyDeviceToDevice, st));
    int64_t w = ne;
    for (size_t i = 0; i < found.size(); ++i) {
        DGT_HIP(hipMemcpyAsync(all.p + w, found[i].p, sizeof(uint64_t) * nfound[i], hipMemcpyDeviceToDevice, st));
        w += nfound[i];
    }
    sort_keys(all, w, st);
    ne = unique_keys(all, w, st);
    edges = std::move(all);
    return total;
}

void Inspector::footprints(int first, int nl, SubSched &sb) {
    hipStream_t st = stream;
    // the last conflict pass found none, so its touches are those of the final tiling
    if (!tk_valid)
        for (int s = 0; s < chain.nsets; ++s) tk_len[s] = touches(first, nl, s, tk_keys[s], tk_bits[s], *cur);
    tk_valid = false;
    dependences(sb, tk_keys, tk_len);
    for (int s = 0; s < chain.nsets; ++s) {
        DBuf<uint64_t> keys = std::move(tk_keys[s]);
        DBuf<uint32_t> bits = std::move(tk_bits[s]);
        const int64_t m = tk_len[s];
        sb.foot_len[s] = m;
        if (m == 0) {
            sb.foot_off[s].alloc(sb.ntiles + 1);
            DGT_HIP(hipMemsetAsync(sb.foot_off[s].p, 0, sizeof(int32_t) * (sb.ntiles + 1), st));
            sb.foot[s].alloc(1);
            sb.acc[s].alloc(1);
            continue;
        }
        DBuf<uint64_t> k2(m);
        DBuf<uint32_t> b2(m);
        k_foot_rekey<<<blocks_for(m, 256), 256, 0, st>>>(keys.p, bits.p, m, k2.p, b2.p);
        sort_pairs(k2, b2, m, st);
        sb.foot[s].alloc(m);
        k_low32<<<blocks_for(m, 256), 256, 0, st>>>(k2.p, m, sb.foot[s].p);
        sb.acc[s] = std::move(b2);
        offsets_by_high(k2, m, sb.ntiles, sb.foot_off[s], st);
    }
}

void Inspector::dependences(SubSched &sb, const DBuf<uint64_t> *keys, const int64_t *len) {
    hipStream_t st = stream;
    const int32_t nt = sb.ntiles;
    std::vector<DBuf<uint64_t>> parts;
    std::vector<int64_t> lens;
    DBuf<int32_t> bad(1);
    DGT_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), st));
    int64_t total = 0;
    for (int s = 0; s < chain.nsets; ++s) {
        const int64_t m = len[s];
        if (m < 2) continue;
        DBuf<int64_t> cnt(m + 1), pos(m + 1);
        DGT_HIP(hipMemsetAsync(cnt.p + m, 0, sizeof(int64_t), st));
        k_dep_count<<<blocks_for(m, 256), 256, 0, st>>>(keys[s].p, m, cnt.p);
        exclusive_scan_i64(cnt.p, pos.p, m + 1, st);
        int64_t np = 0;
        DGT_HIP(hipMemcpyAsync(&np, pos.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        DGT_HIP(hipStreamSynchronize(st));
        if (np == 0) continue;
        DBuf<uint64_t> out(np);
        k_dep_emit<<<blocks_for(m, 256), 256, 0, st>>>(keys[s].p, m, pos.p, sb.color.p, out.p, bad.p);
        parts.push_back(std::move(out));
        lens.push_back(np);
        total += np;
    }
    DBuf<uint64_t> edges(total > 0 ? total : 1);
    int64_t w = 0;
    for (size_t i = 0; i < parts.size(); ++i) {
        DGT_HIP(hipMemcpyAsync(edges.p + w, parts[i].p, sizeof(uint64_t) * lens[i], hipMemcpyDeviceToDevice, st));
        w += lens[i];
    }
    parts.clear();
    sort_keys(edges, total, st);
    const int64_t ne = unique_keys(edges, total, st);
    DGT_REQUIRE(bad.download(st)[0] == 0, DGT_ESTATE, "two tiles of one colour share an element");
    sb.dep_edges = ne;
    sb.dep_need.alloc(nt);
    DGT_HIP(hipMemsetAsync(sb.dep_need.p, 0, sizeof(int32_t) * nt, st));
    if (ne) k_low32_hist<<<blocks_for(ne, 256), 256, 0, st>>>(edges.p, ne, sb.dep_need.p);
    offsets_by_high(edges, ne, nt, sb.dep_off, st);
    sb.dep_succ.alloc(ne > 0 ? ne : 1);
    if (ne) k_low32<<<blocks_for(ne, 256), 256, 0, st>>>(edges.p, ne, sb.dep_succ.p);
}

// One halo exchange per chain: seeds written by T_ne of sub-chain sb turn non-exec.
void Inspector::carry_stale(const Schedule &S, const SubSched &sb, std::vector<uint8_t> &region) {
    hipStream_t st = stream;
    const int64_t n0 = (int64_t)region.size();
    if (n0 == 0) return;
    DBuf<uint8_t> reg;
    reg.upload(region, st);
    for (int j = sb.first; j < sb.first + sb.n; ++j) {
        const ChainLoop &L = chain.loops[j];
        const int64_t n = chain.size[L.set];
        if (n == 0) continue;
        for (int i = 0; i < L.ndesc; ++i) {
            if (L.d[i].mode == DGT_R) continue;
            const int mp = L.d[i].map;
            k_stale<<<blocks_for(n, 256), 256, 0, st>>>(S.sigma[j].p, n, sb.tne, mp < 0 ? nullptr : dmap[mp].p,
                                                        mp < 0 ? 1 : chain.maps[mp].arity, reg.p);
        }
    }
    region = reg.download(st, n0);
}

std::unique_ptr<Schedule> Inspector::run(int64_t ts, int partition, const double *xy_host, const double *xy_dev,
                                         int max_rounds, int cap, const std::vector<int32_t> &splits,
                                         const std::vector<int32_t> &sub_ts, const uint8_t *region_host,
                                         int carry) {
    hipStream_t st = stream;
    DGT_REQUIRE(ts >= 1, DGT_EINVAL, "tile_size must be >= 1");
    DGT_REQUIRE(sub_ts.empty() || sub_ts.size() == splits.size() + 1, DGT_EINVAL,
                "sub_tile_sizes needs one tile size per sub-chain");
    for (int32_t t : sub_ts) DGT_REQUIRE(t >= 1, DGT_EINVAL, "sub-chain tile sizes must be >= 1");
    DGT_REQUIRE(cap >= 0, DGT_EINVAL, "max_colour_tiles must be >= 0");
    DGT_REQUIRE(max_rounds >= 1, DGT_EINVAL, "max_conflict_rounds must be >= 1");
    DGT_REQUIRE(chain.nloops >= 1, DGT_EINVAL, "empty loop chain");
    std::vector<uint8_t> region;
    if (region_host) {
        const int rset = chain.loops[0].set;
        DGT_REQUIRE(cap == 0, DGT_EINVAL, "seed regions do not combine with max_colour_tiles");
        DGT_REQUIRE(carry == 0 || carry == 1, DGT_EINVAL, "region_carry must be 0 or 1");
        for (int32_t sp : splits)
            DGT_REQUIRE(sp >= 0 && sp < chain.nloops && chain.loops[sp].set == rset, DGT_EINVAL,
                        "with seed regions every sub-chain starts on the seed set of loop 0");
        region.assign(region_host, region_host + chain.size[rset]);
        for (uint8_t r : region) DGT_REQUIRE(r <= 2, DGT_EINVAL, "seed regions are 0, 1 or 2");
        if (carry)
            for (int j = 0; j < chain.nloops; ++j)
                for (int i = 0; i < chain.loops[j].ndesc; ++i) {
                    const dgt_desc &d = chain.loops[j].d[i];
                    const int tset = d.map < 0 ? chain.loops[j].set : chain.maps[d.map].to;
                    DGT_REQUIRE(d.mode == DGT_R || tset == rset, DGT_EINVAL,
                                "region_carry needs every write of the chain to land in the seed set");
                }
    }
    auto S = std::make_unique<Schedule>();
    cur = S.get();
    S->nloops = chain.nloops;
    for (int j = 0; j < chain.nloops; ++j) {
        S->loop_size[j] = chain.size[chain.loops[j].set];
        S->sigma[j].alloc(S->loop_size[j] > 0 ? S->loop_size[j] : 1);
    }
    hipEvent_t e0, e1;
    DGT_HIP(hipEventCreate(&e0));
    DGT_HIP(hipEventCreate(&e1));
    DGT_HIP(hipEventRecord(e0, st));
    auto t0 = std::chrono::steady_clock::now();
    int start = 0;
    for (size_t i = 0; i <= splits.size(); ++i) {
        const int end = i < splits.size() ? splits[i] : chain.nloops;
        DGT_REQUIRE(end > start && end <= chain.nloops && end - start <= 31, DGT_EINVAL,
                    "splits must be ascending with sub-chains of 1..31 loops");
        if (partition == 1)
            DGT_REQUIRE(chain.loops[start].set == chain.loops[0].set, DGT_EINVAL,
                        "partition 1 needs every sub-chain to start on the seed set");
        S->sub.emplace_back();
        SubSched &sb = S->sub.back();
        sb.first = start;
        sb.n = end - start;
        for (int j = start; j < end; ++j) S->sub_of[j] = (int)S->sub.size() - 1;
        if (region_host) {
            sb.region = region;
            sb.tne = 0;  // regions requested; run_sub sets the tile ranges
        }
        // a fusion scheme gives each sub-chain its own seed tile size (Sec. 7.2)
        run_sub(*S, sb, sub_ts.empty() ? ts : sub_ts[i], partition, xy_host, xy_dev, max_rounds, cap);
        if (region_host && carry) carry_stale(*S, sb, region);
        start = end;
    }
    DGT_HIP(hipEventRecord(e1, st));
    DGT_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DGT_HIP(hipEventElapsedTime(&ms, e0, e1));
    S->gpu_ms = ms;
    S->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    S->stream = st;
    cur = nullptr;
    return S;
}

}  // namespace dgt
