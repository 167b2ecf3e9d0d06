#pragma once
// Tile executor for sub-chains made of several consecutive operator
// applications of the DG time step (half a step or a whole step of the
// leapfrog scheme).  One thread per footprint cell holds every field of its
// cell in registers; before each operator the cells publish the traces their
// neighbours read (the operator's input and penalty fields) to LDS.  The
// gather at the start and the write-back at the end follow the same rule as
// the other tile kernels (first access reads, written and needed elsewhere),
// so the result is that of the chain executed in order.
#include <hip/hip_runtime.h>

#include <utility>

#include "dg_kernels.h"
#include "refconst.h"
#include "tile_args.h"

namespace dgt {

// The operator applications of one time step, in chain order (the chain the
// solver builds: Taylor order 4 has six, leapfrog order 2 has two).
struct OpDesc {
    bool vel;     // velocity operator (stress-like input), else stress operator
    int in, out;  // fields
    int pen;      // penalty field (used when the flux is upwind), or -1
    int upd;      // update after the operator: 0 none, 1 fourth order, 2 second order
    int part;     // field added with weight dt by the fourth-order update, or -1
};

// operators and loops of one step; a chain fused over several steps numbers its
// operators on across the steps (operator o is operator o mod ops_per_step of step
// o / ops_per_step)
__host__ __device__ constexpr int ops_per_step(int order) { return order == 4 ? 6 : 2; }
__host__ __device__ constexpr int loops_per_step(int order) { return order == 4 ? 26 : 8; }

__host__ __device__ constexpr OpDesc op_desc(int order, int o) {
    o %= ops_per_step(order);
    if (order == 2)
        return o == 0 ? OpDesc{true, F_S, F_Z, F_V, 2, -1} : OpDesc{false, F_V, F_Z, F_S, 2, -1};
    switch (o) {
    case 0: return OpDesc{true, F_S, F_U, -1, 0, -1};
    case 1: return OpDesc{false, F_U, F_X, -1, 0, -1};
    case 2: return OpDesc{true, F_X, F_Z, F_V, 1, F_U};
    case 3: return OpDesc{false, F_V, F_X, -1, 0, -1};
    case 4: return OpDesc{true, F_X, F_U, -1, 0, -1};
    default: return OpDesc{false, F_U, F_Z, F_S, 1, F_X};
    }
}

// index of operator o's volume loop in the chain (each operator: volume,
// interior facets, exterior facets, then a solve at order 4; updates after
// operators 2 and 5 at order 4, after both at order 2)
__host__ __device__ constexpr int op_first_loop(int order, int o) {
    const int st = o / ops_per_step(order), q = o % ops_per_step(order);
    return st * loops_per_step(order) + (order == 2 ? 4 * q : 4 * q + (q >= 3 ? 1 : 0));
}

__host__ __device__ constexpr int op_upd_loop(int order, int o) { return op_first_loop(order, o) + (order == 2 ? 3 : 4); }

// fields operator o touches, its update included (bit per field)
__host__ __device__ constexpr uint32_t op_fields(int order, int o) {
    const OpDesc D = op_desc(order, o);
    uint32_t m = (1u << D.in) | (1u << D.out);
    if (D.pen >= 0) m |= 1u << D.pen;
    if (D.upd) m |= 1u << (D.vel ? F_V : F_S);
    if (D.part >= 0) m |= 1u << D.part;
    return m;
}

// fields operator o writes (its output, and the updated field)
__host__ __device__ constexpr uint32_t op_writes(int order, int o) {
    const OpDesc D = op_desc(order, o);
    return (1u << D.out) | (D.upd ? 1u << (D.vel ? F_V : F_S) : 0u);
}

// first operator of [o0, o0 + n) touching field f, and the last one writing it (-1: none)
__host__ __device__ constexpr int field_first_op(int order, int o0, int n, int f) {
    for (int o = o0; o < o0 + n; ++o)
        if ((op_fields(order, o) >> f) & 1u) return o;
    return -1;
}
__host__ __device__ constexpr int field_last_write(int order, int o0, int n, int f) {
    int last = -1;
    for (int o = o0; o < o0 + n; ++o)
        if ((op_writes(order, o) >> f) & 1u) last = o;
    return last;
}

// Workgroups of a launch go to the GPU's eight XCDs in turn (workgroup b to XCD b mod 8),
// each XCD with its own L2.  A colour launch's workgroup b takes item xcd_item(b, n) of
// its n items, so that every XCD runs one contiguous run of the items -- neighbouring
// tiles in the seed order, which share halo cells, and the shots of a tile -- instead
// of every eighth item.  (A bijection of [0, n); only locality depends on the dispatch.)
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Device-memory pointers held in launch arguments that live in memory (the batched
// kernels) reach the kernel as generic pointers; these say they point to global
// memory, so accesses stay global_load / global_store instead of flat ones.
template <typename T>
using gptr_t = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr_t<T> gp(T *p) {
    return (gptr_t<T>)p;
}

// Field accesses that can meet another tile's data within one launch of the
// dependence-driven schedule (every write-back, and the gathers of fields the
// sub-chain writes) are coherent at device scope: they neither hit a stale line of
// another XCD's L2 nor stay dirty in one, so no cache write-back or invalidation is
// needed between dependent tiles.
template <typename P>
__device__ __forceinline__ auto load_field(P p, bool coherent) {
    return coherent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
template <typename P, typename T>
__device__ __forceinline__ void store_field(P p, T v, bool coherent) {
    if (coherent) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <int K, typename T>
struct CellRegs {
    static constexpr int NP = np_of(K);
    T f[F_COUNT][3][NP];  // fields of the cell (velocity-like ones use two components)
    T g[G_NROWS];
    T nrm[3][3];  // per local facet: unit outward normal (x, y) and |facet| / |J|
};

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int O>
__device__ __forceinline__ void chain_op(const RefC<K, T> &Rf, CellRegs<K, T> &r, const TileArgs &a,
                                         T *__restrict__ lds, int NR, bool act,
                                         int s, uint32_t acc, uint16_t fl, const uint32_t (&nb)[3], int64_t x,
                                         int shot, T amp) {
    constexpr int NP = np_of(K), NFP = K + 1;
    constexpr OpDesc D = op_desc(ORDER, O);
    constexpr int NI = D.vel ? 3 : 2, NO = D.vel ? 2 : 3;
    constexpr int j0 = op_first_loop(ORDER, O) - op_first_loop(ORDER, O0);
    constexpr int ju = op_upd_loop(ORDER, O) - op_first_loop(ORDER, O0);
    constexpr int PO = 2 + NP * NI;  // penalty traces in a row; impedances at 0 and 1
    const bool pen = D.pen >= 0 && a.loops[j0 + 1].pen >= 0;
    T(&vin)[3][NP] = r.f[D.in];
    T(&o)[3][NP] = r.f[D.out];

    // gather the fields whose first use in the sub-chain is this operator (those this
    // cell reads before writing); their loads overlap the previous operator's barrier
    if (act) {
#pragma unroll
        for (int f = 0; f < F_COUNT; ++f) {
            if (field_first_op(ORDER, O0, NOPS, f) != O || !((fl >> f) & 1)) continue;
            // (the dependence-driven schedule gathers the first operator's read-only fields
            // before its dependence wait)
            if (O == O0 && a.persist && field_last_write(ORDER, O0, NOPS, f) < 0) continue;
            const auto F = gp(reinterpret_cast<const T *>(a.F[f])) + shot * a.fshot[f];
            // only fields the sub-chain writes can change during the launch; the others
            // were written by earlier launches and need no device-scope coherence
            const bool coh = a.persist && field_last_write(ORDER, O0, NOPS, f) >= 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= field_ncomp(f)) break;
#pragma unroll
                for (int i = 0; i < NP; ++i)
                    r.f[f][c][i] = load_field(F + (int64_t)(c * NP + i) * a.nc + x, coh);
            }
        }
    }
    if (O > O0) __syncthreads();  // the neighbours have read the previous operator's traces
    if (act) {
        T *row = lds + (size_t)s * NR;
        if (O == O0) {
            row[0] = r.g[G_ZP];
            row[1] = r.g[G_ZS];
        }
#pragma unroll
        for (int c = 0; c < NI; ++c)
#pragma unroll
            for (int i = 0; i < NP; ++i) row[2 + c * NP + i] = vin[c][i];
        if (D.pen >= 0 && pen) {
#pragma unroll
            for (int c = 0; c < NO; ++c)
#pragma unroll
                for (int i = 0; i < NP; ++i) row[PO + c * NP + i] = r.f[D.pen < 0 ? 0 : D.pen][c][i];
        }
    }
    __syncthreads();
    if (!act) return;

    const T rx = r.g[G_RX], ry = r.g[G_RY], sx = r.g[G_SX], sy = r.g[G_SY];
    if ((acc >> j0) & 1u) {  // volume term
        const T scale = sizeof(T) == 8 ? (T)a.loops[j0].scale_d : (T)a.loops[j0].scale_f;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            T ar[NI], as[NI];
#pragma unroll
            for (int c = 0; c < NI; ++c) ar[c] = as[c] = 0;
#pragma unroll
            for (int jj = 0; jj < NP; ++jj) {
                const T dr = Rf.Dr[i * NP + jj], ds = Rf.Ds[i * NP + jj];
#pragma unroll
                for (int c = 0; c < NI; ++c) {
                    ar[c] += dr * vin[c][jj];
                    as[c] += ds * vin[c][jj];
                }
            }
            if constexpr (D.vel) {
                const T irho = r.g[G_IRHO];
                o[0][i] = scale * irho * ((rx * ar[0] + sx * as[0]) + (ry * ar[2] + sy * as[2]));
                o[1][i] = scale * irho * ((rx * ar[2] + sx * as[2]) + (ry * ar[1] + sy * as[1]));
            } else {
                const T lam = r.g[G_LAM], mu = r.g[G_MU];
                const T exx = rx * ar[0] + sx * as[0], eyy = ry * ar[1] + sy * as[1];
                const T exy = T(0.5) * ((ry * ar[0] + sy * as[0]) + (rx * ar[1] + sx * as[1]));
                o[0][i] = scale * ((lam + 2 * mu) * exx + lam * eyy);
                o[1][i] = scale * (lam * exx + (lam + 2 * mu) * eyy);
                o[2][i] = scale * (2 * mu * exy);
            }
        }
    }
    if ((nb[0] | nb[1] | nb[2]) & NB_VALID) {  // this cell's side of the operator's facets in the tile
        const T scale = sizeof(T) == 8 ? (T)a.loops[j0 + 1].scale_d : (T)a.loops[j0 + 1].scale_f;
        const T psc = pen ? (sizeof(T) == 8 ? (T)a.loops[j0 + 1].pscale_d : (T)a.loops[j0 + 1].pscale_f) : T(0);
        const T(&vp)[3][NP] = r.f[D.pen < 0 ? D.out : D.pen];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const uint32_t code = nb[p];
            if (!(code & NB_VALID)) continue;
            const T nx = r.nrm[p][0], ny = r.nrm[p][1], fs = r.nrm[p][2];
            const bool bnd = code & NB_BND;
            const int l1 = (code >> 14) & 3;
            const T *row1 = lds + (size_t)(code & 0x3fff) * NR;
            T gq[NFP][3];
            if (bnd) {
                const bool fr = code & NB_FREE;
#pragma unroll
                for (int m = 0; m < NFP; ++m) {
                    const int n0 = fnode(K, p, m);
                    T a0[NI], p0[NO];
#pragma unroll
                    for (int c = 0; c < NI; ++c) a0[c] = vin[c][n0];
#pragma unroll
                    for (int c = 0; c < NO; ++c) p0[c] = pen ? vp[c][n0] : T(0);
                    gq[m][0] = gq[m][1] = gq[m][2] = 0;
                    if constexpr (D.vel)
                        flux_v_ext<T, UPW, true>(a0, p0, fr, nx, ny, r.g[G_ZP], r.g[G_ZS], fs * r.g[G_IRHO], scale,
                                                 psc, gq[m]);
                    else
                        flux_s_ext<T, UPW, true>(a0, p0, fr, nx, ny, r.g[G_ZP], r.g[G_ZS], r.g[G_LAM], r.g[G_MU], fs,
                                                 scale, psc, gq[m]);
                }
            } else {
                // This cell's side of the interior flux written through the jumps across
                // the facet: with T = sigma n and t = (-ny, nx), the upwind traction state
                // minus this side's traction is zp0/(zp0+zp1) [T.n] n + zs0/(zs0+zs1) [T.t] t,
                // and the velocity state minus this side's velocity is zp1/(zp0+zp1) [v.n] n
                // + zs1/(zs0+zs1) [v.t] t (the same flux as the facet loop's, one side of it);
                // the central flux halves the jump.  Facet constants first, then per node.
                const T zp0 = r.g[G_ZP], zs0 = r.g[G_ZS], zp1 = row1[0], zs1 = row1[1];
                const T nn = nx * nx, mm = ny * ny, nm = nx * ny, nd = nn - mm;
                const T ip = T(1) / (zp0 + zp1), is = T(1) / (zs0 + zs1);
                T kn, kt, qn, qt, C1[3], C2[3];
                if constexpr (D.vel) {
                    const T w0 = fs * r.g[G_IRHO];
                    kn = UPW ? w0 * scale * zp0 * ip : T(0.5) * w0 * scale;
                    kt = UPW ? w0 * scale * zs0 * is : T(0);
                    qn = w0 * psc * zp0 * zp1 * ip;
                    qt = w0 * psc * zs0 * zs1 * is;
                    (void)C1;
                    (void)C2;
                } else {
                    const T lam = r.g[G_LAM], mu = r.g[G_MU];
                    const T w = fs, l2m = w * (lam + 2 * mu), lw = w * lam, mw = w * mu;
                    if (UPW) {
                        kn = scale * zp1 * ip;
                        kt = scale * zs1 * is;
                        qn = psc * ip;
                        qt = psc * is;
                        C1[0] = l2m * nn + lw * mm;
                        C1[1] = lw * nn + l2m * mm;
                        C1[2] = 2 * mw * nm;
                        C2[0] = -2 * mw * nm;
                        C2[1] = 2 * mw * nm;
                        C2[2] = mw * nd;
                    } else {
                        const T kc = T(0.5) * scale;
                        kn = kt = qn = qt = T(0);
                        C1[0] = kc * l2m * nx;  // out = C1 * dvx + C2 * dvy
                        C2[0] = kc * lw * ny;
                        C1[1] = kc * lw * nx;
                        C2[1] = kc * l2m * ny;
                        C1[2] = kc * mw * ny;
                        C2[2] = kc * mw * nx;
                    }
                }
#pragma unroll
                for (int m = 0; m < NFP; ++m) {
                    const int n0 = fnode(K, p, m);
                    const int n1 = l1 == 0 ? fnode(K, 0, K - m) : (l1 == 1 ? fnode(K, 1, K - m) : fnode(K, 2, K - m));
                    T d[NI];  // jump of the operated field (neighbour minus this cell)
#pragma unroll
                    for (int c = 0; c < NI; ++c) d[c] = row1[2 + c * NP + n1] - vin[c][n0];
                    if constexpr (D.vel) {
                        if (UPW) {
                            T An = kn * ((d[0] * nn + d[1] * mm) + d[2] * (2 * nm));
                            T At = kt * (d[2] * nd + nm * (d[1] - d[0]));
                            if constexpr (D.pen >= 0) {  // upwind flux: penalties are on whenever the operator has one
                                const T ex = row1[PO + n1] - vp[0][n0], ey = row1[PO + NP + n1] - vp[1][n0];
                                An += qn * (ex * nx + ey * ny);
                                At += qt * (ey * nx - ex * ny);
                            }
                            gq[m][0] = An * nx - At * ny;
                            gq[m][1] = An * ny + At * nx;
                        } else {
                            gq[m][0] = kn * (d[0] * nx + d[2] * ny);
                            gq[m][1] = kn * (d[2] * nx + d[1] * ny);
                        }
                        gq[m][2] = 0;
                    } else {
                        if (UPW) {
                            T En = kn * (d[0] * nx + d[1] * ny);
                            T Et = kt * (d[1] * nx - d[0] * ny);
                            if constexpr (D.pen >= 0) {
                                const T sxx = row1[PO + n1] - vp[0][n0], syy = row1[PO + NP + n1] - vp[1][n0],
                                        sxy = row1[PO + 2 * NP + n1] - vp[2][n0];
                                En += qn * ((sxx * nn + syy * mm) + sxy * (2 * nm));
                                Et += qt * (sxy * nd + nm * (syy - sxx));
                            }
#pragma unroll
                            for (int c = 0; c < 3; ++c) gq[m][c] = En * C1[c] + Et * C2[c];
                        } else {
#pragma unroll
                            for (int c = 0; c < 3; ++c) gq[m][c] = C1[c] * d[0] + C2[c] * d[1];
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NP; ++i)
#pragma unroll
                for (int m = 0; m < NFP; ++m) {
                    const T lv = Rf.lift[(p * NP + i) * NFP + m];
#pragma unroll
                    for (int c = 0; c < NO; ++c) o[c][i] += lv * gq[m][c];
                }
        }
    }
    if constexpr (D.upd != 0) {  // the update consuming this operator's output
        if (ju < a.nloops && ((acc >> ju) & 1u)) {
            T(&q)[3][NP] = r.f[D.vel ? F_V : F_S];
            const T dt = (T)a.dt;
            const bool src = !D.vel && x == a.src_cells[shot];
            const auto sv = gp(reinterpret_cast<const T *>(a.src_vec)) + shot * NP;
#pragma unroll
            for (int c = 0; c < NO; ++c)
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    T add = o[c][i];
                    if constexpr (D.upd == 1) add = dt * r.f[D.part < 0 ? 0 : D.part][c][i] + add;
                    // amp is the source amplitude of the sub-chain's first step; an operator of
                    // a later step of a fused chain takes its own step's
                    if constexpr (O / ops_per_step(ORDER) == 0) {
                        if (src && c < 2) add += amp * sv[i];
                    } else {
                        if (src && c < 2) add += (T)a.src_amps[O / ops_per_step(ORDER)] * sv[i];
                    }
                    q[c][i] += add;
                }
        }
    }
    // write back the fields this operator writes for the last time in the sub-chain
#pragma unroll
    for (int f = 0; f < F_COUNT; ++f) {
        if (field_last_write(ORDER, O0, NOPS, f) != O || !((fl >> (8 + f)) & 1)) continue;
        const auto F = gp(reinterpret_cast<T *>(a.F[f])) + shot * a.fshot[f];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (c >= field_ncomp(f)) break;
#pragma unroll
            for (int i = 0; i < NP; ++i) store_field(F + (int64_t)(c * NP + i) * a.nc + x, r.f[f][c][i], a.persist);
        }
    }
}

// Dependence-driven schedule, thread 0 of a workgroup: the next (tile, shot) item is
// ticket t of the launch (tiles in colour order, tile_meta of position t / nshots);
// wait_preds waits until every predecessor of the tile has finished for the same
// shot.  Predecessors have lower colours, hence lower tickets, so they were taken by
// workgroups already running: the wait ends unless a counter is wrong, and the poll
// limit ends it then too (the error flag tells the host, and the tile's results are
// invalid).
__device__ __forceinline__ bool wait_preds(const TileArgs &a, int tile, int shot, uint32_t epoch) {
    const uint32_t need = (uint32_t)a.need[tile], base = (epoch - 1u) * need;
    const uint32_t *cnt = a.cnt + (int64_t)shot * a.ntiles + tile;
    uint32_t polls = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base < need) {
        if (++polls > a.spin_limit) {
            atomicExch(a.err, 1);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Tile metadata at position pos of the sub-chain's colour order: the tile, its first
// footprint slot, its footprint length and its neighbour-table offset.
struct TileMeta {
    int x, y, z, w;  // tile, first footprint slot, footprint length, neighbour-table offset
};
__device__ __forceinline__ TileMeta tile_meta(const TileArgs &a, int pos) {
    const auto p = gp(a.tmeta) + 4 * (int64_t)pos;
    return TileMeta{p[0], p[1], p[2], p[3]};
}

// f0, nfoot, b0: the tile's first footprint slot, footprint length and neighbour-table
// offset (from tile_meta)
template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS>
__device__ __forceinline__ void chain_tile(const RefC<K, T> &Rf, const TileArgs &a, T *__restrict__ lds, int tile,
                                           int f0, int nfoot, int b0, int shot, T amp, uint32_t epoch) {
    constexpr int NP = np_of(K);
    const int s = threadIdx.x;
    const bool act = s < nfoot;

    CellRegs<K, T> r;
    uint32_t acc = 0, nb[NOPS][3];
    int64_t x = 0;
    uint16_t fl = 0;
#pragma unroll
    for (int q = 0; q < NOPS; ++q) nb[q][0] = nb[q][1] = nb[q][2] = 0;
#pragma unroll
    for (int f = 0; f < F_COUNT; ++f)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < NP; ++i) r.f[f][c][i] = 0;
    if (act) {
        acc = gp(a.facc)[f0 + s];
        x = gp(a.foot)[f0 + s];
        const bool single = acc >> 31;
#pragma unroll
        for (int f = 0; f < F_COUNT; ++f) {
            const uint32_t m = acc & a.loops_mask[f];
            if (m && ((m & (~m + 1u)) & a.rfirst_mask[f])) fl |= 1u << f;
            if ((acc & a.writes_mask[f]) && (((a.persistent_mask >> f) & 1) || !single)) fl |= 1u << (8 + f);
        }
#pragma unroll
        for (int q = 0; q < NOPS; ++q)
#pragma unroll
            for (int p = 0; p < 3; ++p) nb[q][p] = gp(a.tnb)[b0 + (q * 3 + p) * nfoot + s];
        const auto geo = gp(reinterpret_cast<const T *>(a.geo));
#pragma unroll
        for (int q = 0; q < G_NROWS; ++q) r.g[q] = geo[(int64_t)q * a.nc + x];
        // the facet normals serve every operator of the sub-chain
#pragma unroll
        for (int p = 0; p < 3; ++p)
            facet_normal<T>(p, r.g[G_RX], r.g[G_RY], r.g[G_SX], r.g[G_SY], r.nrm[p][0], r.nrm[p][1], r.nrm[p][2]);
    }
    if (a.persist) {
        // dependence-driven schedule: the tile's metadata, geometry and the fields its first
        // operator reads but no operator of the sub-chain writes (finished by earlier
        // launches) do not depend on other tiles of this launch, so they are loaded before
        // waiting for the tile's predecessors; only what follows is on the dependence path
        if (act) {
#pragma unroll
            for (int f = 0; f < F_COUNT; ++f) {
                if (field_first_op(ORDER, O0, NOPS, f) != O0 || field_last_write(ORDER, O0, NOPS, f) >= 0 ||
                    !((fl >> f) & 1))
                    continue;
                const auto F = gp(reinterpret_cast<const T *>(a.F[f])) + shot * a.fshot[f];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (c >= field_ncomp(f)) break;
#pragma unroll
                    for (int i = 0; i < NP; ++i) r.f[f][c][i] = F[(int64_t)(c * NP + i) * a.nc + x];
                }
            }
        }
        if (threadIdx.x == 0) wait_preds(a, tile, shot, epoch);
        __syncthreads();
    }
    // fields are gathered at their first use and written back after their last write
    [&]<int... Q>(std::integer_sequence<int, Q...>) {
        (chain_op<K, T, UPW, ORDER, O0, NOPS, O0 + Q>(Rf, r, a, lds, a.nrow, act, s, acc, fl, nb[Q], x, shot, amp),
         ...);
    }(std::make_integer_sequence<int, NOPS>{});
}

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
__device__ __forceinline__ void chain_kernel_body(const RefC<K, T> &Rf, const TileArgs &a, unsigned char *smem) {
    __shared__ int s_next, s_shot, s_f0, s_nfoot, s_b0;
    T *lds = reinterpret_cast<T *>(smem);
    if (!a.persist) {  // one launch per colour
        const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
        const TileMeta m = tile_meta(a, a.tile_base + item / a.nshots);
        chain_tile<K, T, UPW, ORDER, O0, NOPS>(Rf, a, lds, m.x, m.y, m.z, m.w, item % a.nshots, (T)a.src_amp,
                                               a.epoch);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) {  // the next (tile, shot) ticket; chain_tile waits for the predecessors
            const uint32_t ticket = atomicAdd(a.head, 1u) - a.head_base;
            if (ticket >= (uint32_t)a.nexec * (uint32_t)a.nshots) {
                s_next = -1;
            } else {
                const TileMeta m = tile_meta(a, (int)(ticket / (uint32_t)a.nshots));
                s_shot = (int)(ticket % (uint32_t)a.nshots);
                s_next = m.x;
                s_f0 = m.y;
                s_nfoot = m.z;
                s_b0 = m.w;
            }
        }
        __syncthreads();
        const int tile = s_next, shot = s_shot;
        if (tile < 0) return;
        chain_tile<K, T, UPW, ORDER, O0, NOPS>(Rf, a, lds, tile, s_f0, s_nfoot, s_b0, shot, (T)a.src_amp, a.epoch);
        // every wave waits for its coherent field stores to complete, so once the barrier
        // is passed the whole tile is visible at device scope and its successors may start
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = a.succ_off[tile]; k < a.succ_off[tile + 1]; ++k)
                __hip_atomic_fetch_add(a.cnt + (int64_t)shot * a.ntiles + a.succ[k], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
__global__ __launch_bounds__(NT) void k_tile_chain(const TileArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (K <= 2 && UPW) {
        // P1/P2 upwind: the reference matrices in LDS; every lane reads the same word
        // (a broadcast), so the operators no longer hold them in scalar registers,
        // which the compiler spilled to vector lanes.  P3/P4 keep constant memory
        // (their small tiles lose more to the extra LDS than they gain), and so does
        // the central flux (its lighter operators lose more to the LDS reads)
        __shared__ __align__(16) RefC<K, T> sref;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&R<K, T>());
        uint32_t *dst = reinterpret_cast<uint32_t *>(&sref);
        for (int i = threadIdx.x; i < (int)(sizeof(RefC<K, T>) / 4); i += NT) dst[i] = src[i];
        __syncthreads();
        chain_kernel_body<K, T, UPW, ORDER, O0, NOPS, NT>(sref, a, smem);
    } else {
        chain_kernel_body<K, T, UPW, ORDER, O0, NOPS, NT>(R<K, T>(), a, smem);
    }
}

}  // namespace dgt
