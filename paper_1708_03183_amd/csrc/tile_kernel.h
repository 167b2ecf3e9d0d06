#pragma once
// Fused tiled executor of the DG chain (Alg. 2 of the paper on one GPU): for a
// colour, one workgroup per tile; the tile's footprint cells are staged in LDS,
// every loop of the (sub-)chain runs on them in chain order with a barrier
// between loops, and what the tile wrote (and other tiles or sub-chains need)
// goes back to HBM.
//
// Work inside a tile is cell-centric: one work item per footprint slot (and
// node group for P3/P4).  Cell loops run on the slots whose loop bit is set in
// the footprint; a facet loop runs through a per-slot neighbour table (the
// local map of the loop: for each local facet of the cell, the neighbour's slot
// and local facet, or the boundary kind) and each cell computes and lifts its
// own side of the facet flux, so no two work items ever write the same slot.
#include <hip/hip_runtime.h>

#include "dg_kernels.h"
#include "refconst.h"
#include "tile_args.h"
#include "tile_chain.h"

namespace dgt {

template <int K, typename T, int F>
__device__ __forceinline__ void stage_field(T *__restrict__ row, const TileArgs &a, int64_t x, uint16_t fl, bool in,
                                            int shot) {
    constexpr int NV = field_ncomp(F) * np_of(K);
    if (a.lds_row[F] < 0) return;
    T *f = reinterpret_cast<T *>(a.F[F]) + shot * a.fshot[F];
    if (in) {
        if (!((fl >> F) & 1)) return;
        T v[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r) v[r] = f[(int64_t)r * a.nc + x];
#pragma unroll
        for (int r = 0; r < NV; ++r) row[a.lds_row[F] + r] = v[r];
    } else {
        if (!((fl >> (8 + F)) & 1)) return;
#pragma unroll
        for (int r = 0; r < NV; ++r) f[(int64_t)r * a.nc + x] = row[a.lds_row[F] + r];
    }
}

// GMEM: the tile's working set (the same layout) lives in a global scratch region of
// the workgroup instead of LDS, for tiles whose footprint exceeds the LDS (it stays in
// L2 and the MALL while the tile runs); the barriers order it as they order LDS, since a
// workgroup's waves share one compute unit and its vector L1.
template <int K, typename T, bool UPW, bool PEN, int NT, bool GMEM = false>
__global__ __launch_bounds__(NT) void k_tile(const TileArgs a) {
    constexpr int NP = np_of(K), NFP = K + 1;
    constexpr int NG = K <= 2 ? 1 : (K == 3 ? 2 : 3);  // node groups per cell
    constexpr int NPG = (NP + NG - 1) / NG;             // nodes per group
    extern __shared__ __align__(16) unsigned char smem_lds[];
    unsigned char *smem = GMEM ? reinterpret_cast<unsigned char *>(a.scratch) + (size_t)blockIdx.x * a.scratch_bytes
                               : smem_lds;
    const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);  // contiguous items per XCD
    const int tile = a.tiles[a.tile_base + item / a.nshots];
    const int shot = item % a.nshots;
    const int f0 = a.foot_off[tile];
    const int nfoot = a.foot_off[tile + 1] - f0;
    const int S = a.stride, NR = a.nrow;
    T *lds = reinterpret_cast<T *>(smem);  // [slot][NR]
    uint32_t *sacc = reinterpret_cast<uint32_t *>(lds + (size_t)S * NR);
    int32_t *sfoot = reinterpret_cast<int32_t *>(sacc + S);
    uint32_t *snb = reinterpret_cast<uint32_t *>(sfoot + S);  // [nfl][3][nfoot]
    uint16_t *flags = reinterpret_cast<uint16_t *>(snb + (size_t)a.nfl * 3 * S);
    const int tid = threadIdx.x;
    const auto &Rf = R<K, T>();
    const int64_t nc = a.nc;
    const int GR = NR - G_NROWS;  // geometry offset in a row

    // the tile's cell ids, loop bits and gather/scatter flags per slot
    for (int s = tid; s < nfoot; s += NT) {
        const uint32_t acc = a.facc[f0 + s];
        sacc[s] = acc;
        sfoot[s] = a.foot[f0 + s];
        const bool single = acc >> 31;
        uint16_t g = 0, w = 0;
#pragma unroll
        for (int f = 0; f < F_COUNT; ++f) {
            if (a.lds_row[f] < 0) continue;
            const uint32_t m = acc & a.loops_mask[f];
            if (m && ((m & (~m + 1u)) & a.rfirst_mask[f])) g |= 1u << f;
            if ((acc & a.writes_mask[f]) && (((a.persistent_mask >> f) & 1) || !single)) w |= 1u << f;
        }
        flags[s] = (uint16_t)(g | (w << 8));
    }
    {
        const int b0 = a.tnb_off[tile], n = a.tnb_off[tile + 1] - b0;
        for (int i = tid; i < n; i += NT) snb[i] = a.tnb[b0 + i];
    }
    __syncthreads();
    // gather the footprint: one slot per work item, all its rows in flight at once
    {
        const T *geo = reinterpret_cast<const T *>(a.geo);
        for (int s = tid; s < nfoot; s += NT) {
            const int64_t x = sfoot[s];
            const uint16_t fl = flags[s];
            T *row = lds + (size_t)s * NR;
            T gv[G_NROWS];
#pragma unroll
            for (int r = 0; r < G_NROWS; ++r) gv[r] = geo[(int64_t)r * nc + x];
            stage_field<K, T, 0>(row, a, x, fl, true, shot);
            stage_field<K, T, 1>(row, a, x, fl, true, shot);
            stage_field<K, T, 2>(row, a, x, fl, true, shot);
            stage_field<K, T, 3>(row, a, x, fl, true, shot);
            stage_field<K, T, 4>(row, a, x, fl, true, shot);
#pragma unroll
            for (int r = 0; r < G_NROWS; ++r) row[GR + r] = gv[r];
        }
    }
    __syncthreads();

    const T dt = (T)a.dt;
    for (int j = 0; j < a.nloops; ++j) {
        const TLoop L = a.loops[j];
        if (L.kind == KV_SOLVE) continue;  // folded into the operators: no data moves
        const T scale = sizeof(T) == 8 ? (T)L.scale_d : (T)L.scale_f;
        const T pscale = sizeof(T) == 8 ? (T)L.pscale_d : (T)L.pscale_f;
        const int oin = a.lds_row[L.in < 0 ? 0 : L.in], oout = a.lds_row[L.out < 0 ? 0 : L.out];
        const int open = L.pen >= 0 ? a.lds_row[L.pen] : 0;
        for (int item = tid; item < nfoot * NG; item += NT) {
            const int s = NG == 1 ? item : item / NG;
            const int g = NG == 1 ? 0 : item - s * NG;
            T *row = lds + (size_t)s * NR;
            const T *geo = row + GR;
            switch (L.kind) {
            case KV_VOL_V:
            case KV_VOL_S: {
                if (!((sacc[s] >> j) & 1)) break;
                const T rx = geo[G_RX], ry = geo[G_RY], sx = geo[G_SX], sy = geo[G_SY];
                const T *u = row + oin;
                T *o = row + oout;
#pragma unroll
                for (int ii = 0; ii < NPG; ++ii) {
                    const int i = g * NPG + ii;
                    if (NG > 1 && i >= NP) break;
                    if (L.kind == KV_VOL_V) {
                        T ar[3] = {0, 0, 0}, as[3] = {0, 0, 0};
#pragma unroll
                        for (int jj = 0; jj < NP; ++jj) {
                            const T dr = Rf.Dr[i * NP + jj], ds = Rf.Ds[i * NP + jj];
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                ar[c] += dr * u[c * NP + jj];
                                as[c] += ds * u[c * NP + jj];
                            }
                        }
                        const T irho = geo[G_IRHO];
                        o[0 * NP + i] = scale * irho * ((rx * ar[0] + sx * as[0]) + (ry * ar[2] + sy * as[2]));
                        o[1 * NP + i] = scale * irho * ((rx * ar[2] + sx * as[2]) + (ry * ar[1] + sy * as[1]));
                    } else {
                        T ar[2] = {0, 0}, as[2] = {0, 0};
#pragma unroll
                        for (int jj = 0; jj < NP; ++jj) {
                            const T dr = Rf.Dr[i * NP + jj], ds = Rf.Ds[i * NP + jj];
#pragma unroll
                            for (int c = 0; c < 2; ++c) {
                                ar[c] += dr * u[c * NP + jj];
                                as[c] += ds * u[c * NP + jj];
                            }
                        }
                        const T lam = geo[G_LAM], mu = geo[G_MU];
                        const T exx = rx * ar[0] + sx * as[0], eyy = ry * ar[1] + sy * as[1];
                        const T exy = T(0.5) * ((ry * ar[0] + sy * as[0]) + (rx * ar[1] + sx * as[1]));
                        o[0 * NP + i] = scale * ((lam + 2 * mu) * exx + lam * eyy);
                        o[1 * NP + i] = scale * (lam * exx + (lam + 2 * mu) * eyy);
                        o[2 * NP + i] = scale * (2 * mu * exy);
                    }
                }
                break;
            }
            case KV_INT_V:
            case KV_INT_S:
            case KV_EXT_V:
            case KV_EXT_S: {
                const bool vel = L.kind == KV_INT_V || L.kind == KV_EXT_V;
                const uint32_t *nb = snb + (size_t)L.grp * 3 * nfoot + s;
                const uint32_t cd[3] = {nb[0], nb[nfoot], nb[2 * nfoot]};
                if (!((cd[0] | cd[1] | cd[2]) & NB_VALID)) break;
                const bool pen = PEN && L.pen >= 0;
                const T psc = pen ? pscale : T(0);
                T acc[NPG][3];
#pragma unroll
                for (int ii = 0; ii < NPG; ++ii) acc[ii][0] = acc[ii][1] = acc[ii][2] = 0;
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const uint32_t code = cd[p];
                    if (!(code & NB_VALID)) continue;
                    T nx, ny, fs;
                    facet_normal<T>(p, geo[G_RX], geo[G_RY], geo[G_SX], geo[G_SY], nx, ny, fs);
                    const bool bnd = code & NB_BND;
                    const int s1 = code & 0x3fff, l1 = (code >> 14) & 3;
                    const T *row1 = lds + (size_t)(bnd ? s : s1) * NR;
                    const T *geo1 = row1 + GR;
#pragma unroll
                    for (int m = 0; m < NFP; ++m) {
                        const int n0 = Rf.fn[p * NFP + m];
                        const int n1 = Rf.fn[l1 * NFP + (K - m)];
                        T gq[3] = {0, 0, 0};
                        if (vel) {
                            T sa[3], va[2] = {0, 0};
#pragma unroll
                            for (int c = 0; c < 3; ++c) sa[c] = row[oin + c * NP + n0];
                            if (pen) {
#pragma unroll
                                for (int c = 0; c < 2; ++c) va[c] = row[open + c * NP + n0];
                            }
                            if (bnd) {
                                flux_v_ext<T, UPW, PEN>(sa, va, code & NB_FREE, nx, ny, geo[G_ZP], geo[G_ZS],
                                                        fs * geo[G_IRHO], scale, psc, gq);
                            } else {
                                T sb[3], vb[2] = {0, 0}, g1[3];
#pragma unroll
                                for (int c = 0; c < 3; ++c) sb[c] = row1[oin + c * NP + n1];
                                if (pen) {
#pragma unroll
                                    for (int c = 0; c < 2; ++c) vb[c] = row1[open + c * NP + n1];
                                }
                                flux_v_int<T, UPW, PEN>(sa, sb, va, vb, nx, ny, geo[G_ZP], geo[G_ZS], geo1[G_ZP],
                                                        geo1[G_ZS], fs * geo[G_IRHO], T(0), scale, psc, gq, g1);
                            }
                        } else {
                            T va[2], sa[3] = {0, 0, 0};
#pragma unroll
                            for (int c = 0; c < 2; ++c) va[c] = row[oin + c * NP + n0];
                            if (pen) {
#pragma unroll
                                for (int c = 0; c < 3; ++c) sa[c] = row[open + c * NP + n0];
                            }
                            if (bnd) {
                                flux_s_ext<T, UPW, PEN>(va, sa, code & NB_FREE, nx, ny, geo[G_ZP], geo[G_ZS],
                                                        geo[G_LAM], geo[G_MU], fs, scale, psc, gq);
                            } else {
                                T vb[2], sb[3] = {0, 0, 0}, g1[3];
#pragma unroll
                                for (int c = 0; c < 2; ++c) vb[c] = row1[oin + c * NP + n1];
                                if (pen) {
#pragma unroll
                                    for (int c = 0; c < 3; ++c) sb[c] = row1[open + c * NP + n1];
                                }
                                flux_s_int<T, UPW, PEN>(va, vb, sa, sb, nx, ny, geo[G_ZP], geo[G_ZS], geo1[G_ZP],
                                                        geo1[G_ZS], geo[G_LAM], geo[G_MU], geo1[G_LAM],
                                                        geo1[G_MU], fs, T(0), scale, psc, gq, g1);
                            }
                        }
#pragma unroll
                        for (int ii = 0; ii < NPG; ++ii) {
                            const int i = g * NPG + ii;
                            if (NG > 1 && i >= NP) break;
                            const T lv = Rf.lift[(p * NP + i) * NFP + m];
                            acc[ii][0] += lv * gq[0];
                            acc[ii][1] += lv * gq[1];
                            acc[ii][2] += lv * gq[2];
                        }
                    }
                }
                T *o = row + oout;
#pragma unroll
                for (int ii = 0; ii < NPG; ++ii) {
                    const int i = g * NPG + ii;
                    if (NG > 1 && i >= NP) break;
                    o[0 * NP + i] += acc[ii][0];
                    o[1 * NP + i] += acc[ii][1];
                    if (!vel) o[2 * NP + i] += acc[ii][2];
                }
                break;
            }
            case KV_UPD_V:
            case KV_UPD2_V: {
                if (!((sacc[s] >> j) & 1)) break;
                const bool o4 = L.kind == KV_UPD_V;
                T *V = row + a.lds_row[F_V];
                const T *Z = row + a.lds_row[F_Z];
                const T *U = row + (o4 ? a.lds_row[F_U] : 0);
#pragma unroll
                for (int ii = 0; ii < NPG; ++ii) {
                    const int i = g * NPG + ii;
                    if (NG > 1 && i >= NP) break;
#pragma unroll
                    for (int c = 0; c < 2; ++c) V[c * NP + i] += (o4 ? dt * U[c * NP + i] : T(0)) + Z[c * NP + i];
                }
                break;
            }
            case KV_UPD_S:
            case KV_UPD2_S: {
                if (!((sacc[s] >> j) & 1)) break;
                const bool o4 = L.kind == KV_UPD_S;
                T *Sg = row + a.lds_row[F_S];
                const T *Z = row + a.lds_row[F_Z];
                const T *X = row + (o4 ? a.lds_row[F_X] : 0);
                const bool src = sfoot[s] == a.src_cells[shot];
                const T *sv = reinterpret_cast<const T *>(a.src_vec) + shot * NP;
#pragma unroll
                for (int ii = 0; ii < NPG; ++ii) {
                    const int i = g * NPG + ii;
                    if (NG > 1 && i >= NP) break;
                    const T sa = src ? (T)a.src_amps[L.step] * sv[i] : T(0);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        Sg[c * NP + i] += (o4 ? dt * X[c * NP + i] : T(0)) + Z[c * NP + i] + (c < 2 ? sa : T(0));
                }
                break;
            }
            default:
                break;
            }
        }
        if (L.partner >= 0) ++j;  // the exterior loop ran with its interior loop
        __syncthreads();
    }
    // scatter what this tile wrote and others (or later sub-chains) need
    for (int s = tid; s < nfoot; s += NT) {
        const int64_t x = sfoot[s];
        const uint16_t fl = flags[s];
        T *row = lds + (size_t)s * NR;
        stage_field<K, T, 0>(row, a, x, fl, false, shot);
        stage_field<K, T, 1>(row, a, x, fl, false, shot);
        stage_field<K, T, 2>(row, a, x, fl, false, shot);
        stage_field<K, T, 3>(row, a, x, fl, false, shot);
        stage_field<K, T, 4>(row, a, x, fl, false, shot);
    }
}

}  // namespace dgt
