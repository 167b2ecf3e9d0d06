#pragma once
// Tile executor for degrees k >= 3 on the matrix cores (gfx950 MFMA).
//
// The per-cell contractions of an operator application (the derivative
// matrices of the cell-integral loop and the lift of the facet loops, with the
// block-diagonal solve folded in) are small dense products of an Np x Np or
// Np x 3(k+1) reference matrix with the cells' nodal values.  Taken over 16
// cells at a time they are 16 x 16 x 4 matrix products: the reference matrix
// is the A operand (rows = output nodes, padded to 16), the cells' values the
// B operand (one column per cell), and the result stays in the accumulator
// registers of the wave, one column per cell.  Per-cell factors (geometry,
// material, the loop's scale) and the masks of the tile's iteration sets are
// applied to the B columns, so cells whose iteration belongs to another tile
// contribute nothing.
//
// Data of a tile: the fields some operator of the sub-chain reads through a
// facet (its operand and its penalty field) live in LDS for every footprint
// slot, [component][node][slot]; fields only produced and consumed by the same
// cell (the last output, consumed by the update, and the updated field) stay in
// the accumulator layout and go straight to and from HBM.  A sub-chain may hold
// several consecutive operator applications (half a time step of the fourth-order
// scheme), with a barrier between them; the updated field is not read again
// inside such a sub-chain, so the update writes it to HBM only.  The gather,
// increment and write-back rules are those of the other tile kernels, so the
// result is the chain's.
#include <hip/hip_runtime.h>

#include <utility>

#include "dg_kernels.h"
#include "refconst.h"
#include "tile_args.h"
#include "tile_chain.h"

namespace dgt {

template <typename T>
struct Mfma;
// Operand layouts (one wave, checked on the device): A[i][k] in lane i + 16 k, B[k][j]
// in lane j + 16 k; the accumulator's register r of lane l holds D[row(l / 16, r)][l % 16].
template <>
struct Mfma<float> {
    typedef float V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ V4 mma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    typedef double V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
    static __device__ __forceinline__ V4 mma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// the 16 x 4 blocks of the reference matrices held by one lane: A[i][k] with
// i = lane % 16 (output node) and k = 4 t + lane / 16
template <int K, typename T>
struct MfmaRef {
    static constexpr int NP = np_of(K), NFP = K + 1, NQ = 3 * NFP;
    static constexpr int KS = (NP + 3) / 4, KQ = (NQ + 3) / 4;
    T dr[KS], ds[KS], lf[KQ];
    __device__ __forceinline__ void load(const RefC<K, T> &Rf, int lane) {
        const int i = lane & 15, kk = lane >> 4;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const int k = 4 * t + kk;
            const bool ok = i < NP && k < NP;
            dr[t] = ok ? Rf.Dr[(ok ? i : 0) * NP + (ok ? k : 0)] : T(0);
            ds[t] = ok ? Rf.Ds[(ok ? i : 0) * NP + (ok ? k : 0)] : T(0);
        }
#pragma unroll
        for (int t = 0; t < KQ; ++t) {
            const int q = 4 * t + kk;
            const bool ok = i < NP && q < NQ;
            const int p = ok ? q / NFP : 0, m = ok ? q % NFP : 0;
            lf[t] = ok ? Rf.lift[(p * NP + (ok ? i : 0)) * NFP + m] : T(0);
        }
    }
};

// per-slot tile data in LDS behind the field and geometry regions
template <typename T>
struct MfmaTile {
    T *f;              // field regions and geometry, [rows][S]
    uint32_t *acc;     // [S] loop bits
    int32_t *x;        // [S] exec cell id
    uint16_t *fl;      // [S] gather (bits 0-7) and write-back (bits 8-15) flags per field
    uint32_t *nb;      // [operator][local facet][S] neighbour codes of the tile's facet loops
    int S, nfoot, f0, tile, shot;
};

// one operator application of the sub-chain on the wave's 16-cell groups
template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int O, int NT>
__device__ __forceinline__ void mfma_op(const MfmaRef<K, T> &Ar, const TileArgs &a, const MfmaTile<T> &tl) {
    using V4 = typename Mfma<T>::V4;
    constexpr int NP = np_of(K), NFP = K + 1, NQ = 3 * NFP;
    constexpr int KS = MfmaRef<K, T>::KS, KQ = MfmaRef<K, T>::KQ;
    constexpr OpDesc D = op_desc(ORDER, O);
    constexpr int NI = D.vel ? 3 : 2, NO = D.vel ? 2 : 3;
    constexpr int j0 = op_first_loop(ORDER, O) - op_first_loop(ORDER, O0);
    constexpr int ju = op_upd_loop(ORDER, O) - op_first_loop(ORDER, O0);
    constexpr int QF = D.vel ? F_V : F_S;  // field the update writes
    const int S = tl.S, nfoot = tl.nfoot;
    const bool pen = D.pen >= 0 && a.loops[j0 + 1].pen >= 0;
    const int tid = threadIdx.x;
    const uint32_t nc32 = (uint32_t)a.nc;  // component-node rows of a field fit in 32 bits (host check)

    // gather the LDS fields whose first use in the sub-chain is this operator
#pragma unroll
    for (int f = 0; f < F_COUNT; ++f) {
        if (field_first_op(ORDER, O0, NOPS, f) != O || a.lds_row[f] < 0) continue;
        const int nr = field_ncomp(f) * NP;
        const T *F = reinterpret_cast<const T *>(a.F[f]) + tl.shot * a.fshot[f];
        const bool coh = a.persist && field_last_write(ORDER, O0, NOPS, f) >= 0;
        T *dst = tl.f + a.lds_row[f];
        for (int s = tid; s < nfoot; s += NT) {
            if (!((tl.fl[s] >> f) & 1)) continue;
            const T *Fx = F + tl.x[s];
            T v[3 * NP];
#pragma unroll
            for (int r = 0; r < 3 * NP; ++r)
                if (r < nr) v[r] = load_field(Fx + (uint32_t)r * nc32, coh);
#pragma unroll
            for (int r = 0; r < 3 * NP; ++r)
                if (r < nr) dst[(size_t)r * S + s] = v[r];
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int jc = lane & 15, g = lane >> 4;  // B/D column (cell) and row block
    constexpr int NW = NT / 64;
    const int ngroups = (nfoot + 15) >> 4;
    const T scale = sizeof(T) == 8 ? (T)a.loops[j0].scale_d : (T)a.loops[j0].scale_f;
    const T fscale = sizeof(T) == 8 ? (T)a.loops[j0 + 1].scale_d : (T)a.loops[j0 + 1].scale_f;
    const T psc = pen ? (sizeof(T) == 8 ? (T)a.loops[j0 + 1].pscale_d : (T)a.loops[j0 + 1].pscale_f) : T(0);
    const T *gr = tl.f + a.nrow;  // geometry rows
    const T *fin = tl.f + a.lds_row[D.in];
    const T *fpn = tl.f + (pen ? a.lds_row[D.pen < 0 ? 0 : D.pen] : 0);
    const T dt = (T)a.dt;

    const T *nrm = gr + G_NROWS * S;  // per local facet: outward unit normal and |facet| / |J|
    // the facet points this lane evaluates: q = 4 t + g -> local facet, node on it, cell node
    int pt_p[KQ], pt_m[KQ], pt_n0[KQ];
#pragma unroll
    for (int t = 0; t < KQ; ++t) {
        const int q = 4 * t + g;
        pt_p[t] = q < NQ ? q / NFP : 3;
        pt_m[t] = q < NQ ? q % NFP : 0;
        pt_n0[t] = q < NQ ? fnode(K, pt_p[t], pt_m[t]) : 0;
    }

    for (int grp = wave; grp < ngroups; grp += NW) {
        const int s = grp * 16 + jc;
        const bool valid = s < nfoot;
        const int sv = valid ? s : 0;
        const uint32_t acc = valid ? tl.acc[sv] : 0u;
        const uint16_t fl = valid ? tl.fl[sv] : (uint16_t)0;
        const int64_t x = tl.x[sv];
        const bool vol = (acc >> j0) & 1u;
        const T rx = gr[G_RX * S + sv], ry = gr[G_RY * S + sv], sx = gr[G_SX * S + sv], sy = gr[G_SY * S + sv];

        // operands of the update that are not in LDS, loaded now so that their latency
        // hides behind the contractions
        constexpr int NU = D.upd != 0 ? NO : 1;
        T qpre[NU][4], ppre[NU][4];
        bool upd = false;
        if constexpr (D.upd != 0) {
            upd = valid && ju < a.nloops && ((acc >> ju) & 1u);
            const T *Q = reinterpret_cast<const T *>(a.F[QF]) + tl.shot * a.fshot[QF];
            const T *PF = reinterpret_cast<const T *>(a.F[D.part < 0 ? 0 : D.part]) +
                          tl.shot * a.fshot[D.part < 0 ? 0 : D.part];
            const bool q_glob = a.lds_row[QF] < 0;
            const bool p_glob = D.part >= 0 && a.lds_row[D.part < 0 ? 0 : D.part] < 0;
            const bool p_coh = a.persist && D.part >= 0 && field_last_write(ORDER, O0, NOPS, D.part) >= 0;
#pragma unroll
            for (int c = 0; c < NU; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = Mfma<T>::row(g, r);
                    const uint32_t gi = (uint32_t)(c * NP + (i < NP ? i : 0)) * nc32;
                    qpre[c][r] = (upd && i < NP && q_glob) ? load_field(Q + x + gi, a.persist) : T(0);
                    ppre[c][r] = (upd && i < NP && p_glob) ? load_field(PF + x + gi, p_coh) : T(0);
                }
        }

        // accumulators: one 16 x 16 block per output component, rows = nodes, columns = cells;
        // a cell whose volume loop is not in this tile starts from its partial sum
        V4 o[NO];
#pragma unroll
        for (int c = 0; c < NO; ++c) o[c] = V4{0, 0, 0, 0};
        const bool init = valid && !vol && ((fl >> D.out) & 1);
        if (__ballot(init)) {
            if (a.lds_row[D.out] >= 0) {
                const T *src = tl.f + a.lds_row[D.out];
#pragma unroll
                for (int c = 0; c < NO; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = Mfma<T>::row(g, r);
                        if (i < NP && init) o[c][r] = src[(size_t)(c * NP + i) * S + sv];
                    }
            } else {
                const T *F = reinterpret_cast<const T *>(a.F[D.out]) + tl.shot * a.fshot[D.out];
                const bool coh = a.persist;
#pragma unroll
                for (int c = 0; c < NO; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = Mfma<T>::row(g, r);
                        if (i < NP && init) o[c][r] = load_field(F + x + (uint32_t)(c * NP + i) * nc32, coh);
                    }
            }
        }

        // cell-integral loop: o += Dr B_r + Ds B_s with the cell's factors folded into the columns
        if (__ballot(valid && vol)) {
            const T w = vol ? scale : T(0);
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const int k = 4 * t + g;
                T u[NI];
#pragma unroll
                for (int c = 0; c < NI; ++c) u[c] = (k < NP && vol) ? fin[(size_t)(c * NP + (k < NP ? k : 0)) * S + sv] : T(0);
                if constexpr (D.vel) {
                    const T wr = w * gr[G_IRHO * S + sv];
                    // rates of vx and vy: rho^-1 (Dx sxx + Dy sxy, Dx sxy + Dy syy)
                    const T br0 = wr * (rx * u[0] + ry * u[2]), bs0 = wr * (sx * u[0] + sy * u[2]);
                    const T br1 = wr * (rx * u[2] + ry * u[1]), bs1 = wr * (sx * u[2] + sy * u[1]);
                    o[0] = Mfma<T>::mma(Ar.dr[t], br0, o[0]);
                    o[1] = Mfma<T>::mma(Ar.dr[t], br1, o[1]);
                    o[0] = Mfma<T>::mma(Ar.ds[t], bs0, o[0]);
                    o[1] = Mfma<T>::mma(Ar.ds[t], bs1, o[1]);
                } else {
                    // C eps(v): (lam+2mu) exx + lam eyy, lam exx + (lam+2mu) eyy, 2 mu exy
                    const T lam = gr[G_LAM * S + sv], mu = gr[G_MU * S + sv];
                    const T l2 = w * (lam + 2 * mu), lw = w * lam, mw = w * mu;
                    const T br0 = l2 * rx * u[0] + lw * ry * u[1], bs0 = l2 * sx * u[0] + lw * sy * u[1];
                    const T br1 = lw * rx * u[0] + l2 * ry * u[1], bs1 = lw * sx * u[0] + l2 * sy * u[1];
                    const T br2 = mw * (ry * u[0] + rx * u[1]), bs2 = mw * (sy * u[0] + sx * u[1]);
                    o[0] = Mfma<T>::mma(Ar.dr[t], br0, o[0]);
                    o[1] = Mfma<T>::mma(Ar.dr[t], br1, o[1]);
                    o[2] = Mfma<T>::mma(Ar.dr[t], br2, o[2]);
                    o[0] = Mfma<T>::mma(Ar.ds[t], bs0, o[0]);
                    o[1] = Mfma<T>::mma(Ar.ds[t], bs1, o[1]);
                    o[2] = Mfma<T>::mma(Ar.ds[t], bs2, o[2]);
                }
            }
        }

        // facet loops of this tile: the flux at facet point q = 4 t + g of the column's cell
        // (its own side), lifted by LIFT (A) x flux (B)
        uint32_t nb[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) nb[p] = tl.nb[((O - O0) * 3 + p) * S + sv];
        if (__ballot((nb[0] | nb[1] | nb[2]) & NB_VALID)) {
            const T zp0 = gr[G_ZP * S + sv], zs0 = gr[G_ZS * S + sv];
            const T irho = gr[G_IRHO * S + sv], lam = gr[G_LAM * S + sv], mu = gr[G_MU * S + sv];
#pragma unroll
            for (int t = 0; t < KQ; ++t) {
                const int p = pt_p[t], m = pt_m[t];
                const uint32_t code = p == 0 ? nb[0] : (p == 1 ? nb[1] : (p == 2 ? nb[2] : 0u));
                T gq[3] = {0, 0, 0};
                if (code & NB_VALID) {
                    const T nx = nrm[(3 * p) * S + s], ny = nrm[(3 * p + 1) * S + s], fs = nrm[(3 * p + 2) * S + s];
                    const int n0 = pt_n0[t];
                    T a0[NI], p0[NO];
#pragma unroll
                    for (int c = 0; c < NI; ++c) a0[c] = fin[(size_t)(c * NP + n0) * S + s];
#pragma unroll
                    for (int c = 0; c < NO; ++c) p0[c] = pen ? fpn[(size_t)(c * NP + n0) * S + s] : T(0);
                    if (code & NB_BND) {
                        const bool fr = code & NB_FREE;
                        if constexpr (D.vel)
                            flux_v_ext<T, UPW, true>(a0, p0, fr, nx, ny, zp0, zs0, fs * irho, fscale, psc, gq);
                        else
                            flux_s_ext<T, UPW, true>(a0, p0, fr, nx, ny, zp0, zs0, lam, mu, fs, fscale, psc, gq);
                    } else {
                        // this cell's side through the jumps across the facet (as in the
                        // register-resident chain kernel)
                        const int s1 = code & 0x3fff, l1 = (code >> 14) & 3;
                        const int n1 = fnode(K, l1, K - m);
                        const T zp1 = gr[G_ZP * S + s1], zs1 = gr[G_ZS * S + s1];
                        const T nn = nx * nx, mm = ny * ny, nm = nx * ny, nd = nn - mm;
                        const T ip = T(1) / (zp0 + zp1), is = T(1) / (zs0 + zs1);
                        T d[NI];
#pragma unroll
                        for (int c = 0; c < NI; ++c) d[c] = fin[(size_t)(c * NP + n1) * S + s1] - a0[c];
                        if constexpr (D.vel) {
                            const T w0 = fs * irho;
                            if (UPW) {
                                T An = w0 * fscale * zp0 * ip * ((d[0] * nn + d[1] * mm) + d[2] * (2 * nm));
                                T At = w0 * fscale * zs0 * is * (d[2] * nd + nm * (d[1] - d[0]));
                                if constexpr (D.pen >= 0) {
                                    if (pen) {
                                        const T ex = fpn[(size_t)n1 * S + s1] - p0[0];
                                        const T ey = fpn[(size_t)(NP + n1) * S + s1] - p0[1];
                                        An += w0 * psc * zp0 * zp1 * ip * (ex * nx + ey * ny);
                                        At += w0 * psc * zs0 * zs1 * is * (ey * nx - ex * ny);
                                    }
                                }
                                gq[0] = An * nx - At * ny;
                                gq[1] = An * ny + At * nx;
                            } else {
                                const T kn = T(0.5) * w0 * fscale;
                                gq[0] = kn * (d[0] * nx + d[2] * ny);
                                gq[1] = kn * (d[2] * nx + d[1] * ny);
                            }
                        } else {
                            const T l2m = fs * (lam + 2 * mu), lw = fs * lam, mw = fs * mu;
                            if (UPW) {
                                T En = fscale * zp1 * ip * (d[0] * nx + d[1] * ny);
                                T Et = fscale * zs1 * is * (d[1] * nx - d[0] * ny);
                                if constexpr (D.pen >= 0) {
                                    if (pen) {
                                        const T dxx = fpn[(size_t)n1 * S + s1] - p0[0];
                                        const T dyy = fpn[(size_t)(NP + n1) * S + s1] - p0[1];
                                        const T dxy = fpn[(size_t)(2 * NP + n1) * S + s1] - p0[2];
                                        En += psc * ip * ((dxx * nn + dyy * mm) + dxy * (2 * nm));
                                        Et += psc * is * (dxy * nd + nm * (dyy - dxx));
                                    }
                                }
                                gq[0] = En * (l2m * nn + lw * mm) + Et * (-2 * mw * nm);
                                gq[1] = En * (lw * nn + l2m * mm) + Et * (2 * mw * nm);
                                gq[2] = En * (2 * mw * nm) + Et * (mw * nd);
                            } else {
                                const T kc = T(0.5) * fscale;
                                gq[0] = kc * (l2m * nx * d[0] + lw * ny * d[1]);
                                gq[1] = kc * (lw * nx * d[0] + l2m * ny * d[1]);
                                gq[2] = kc * (mw * ny * d[0] + mw * nx * d[1]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NO; ++c) o[c] = Mfma<T>::mma(Ar.lf[t], gq[c], o[c]);
            }
        }

        // the operator's output: into LDS when a later operator reads it through a facet,
        // to HBM after its last write in the sub-chain (write-back rule of the tile kernels)
        const bool wb_out = field_last_write(ORDER, O0, NOPS, D.out) == O && ((fl >> (8 + D.out)) & 1);
        if (a.lds_row[D.out] >= 0) {
            T *dst = tl.f + a.lds_row[D.out];
#pragma unroll
            for (int c = 0; c < NO; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = Mfma<T>::row(g, r);
                    if (i < NP && valid) dst[(size_t)(c * NP + i) * S + s] = o[c][r];
                }
        }
        if (wb_out) {
            T *F = reinterpret_cast<T *>(a.F[D.out]) + tl.shot * a.fshot[D.out];
#pragma unroll
            for (int c = 0; c < NO; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = Mfma<T>::row(g, r);
                    if (i < NP) store_field(F + x + (uint32_t)(c * NP + i) * nc32, o[c][r], a.persist);
                }
        }

        // the update consuming this operator's output (leapfrog, fourth or second order)
        if constexpr (D.upd != 0) {
            if (__ballot(upd)) {
                T *Q = reinterpret_cast<T *>(a.F[QF]) + tl.shot * a.fshot[QF];
                const bool q_lds = a.lds_row[QF] >= 0;
                const bool p_lds = D.part >= 0 && a.lds_row[D.part < 0 ? 0 : D.part] >= 0;
                const bool wb_q = field_last_write(ORDER, O0, NOPS, QF) == O && ((fl >> (8 + QF)) & 1);
                const bool src = !D.vel && x == a.src_cells[tl.shot];
                const T *svec = reinterpret_cast<const T *>(a.src_vec) + tl.shot * NP;
#pragma unroll
                for (int c = 0; c < NO; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = Mfma<T>::row(g, r);
                        if (i >= NP || !upd) continue;
                        const size_t li = (size_t)(c * NP + i) * S + s;
                        const uint32_t gi = (uint32_t)(c * NP + i) * nc32;
                        T add = o[c][r];
                        if constexpr (D.upd == 1) {
                            const T pv = p_lds ? tl.f[a.lds_row[D.part] + li] : ppre[c][r];
                            add = dt * pv + add;
                        }
                        if (src && c < 2) add += (T)a.src_amp * svec[i];
                        // the old value may sit in LDS (the operator's penalty field, which other
                        // waves still read as neighbour traces): the new one goes to HBM only
                        T qv = q_lds ? tl.f[a.lds_row[QF] + li] : qpre[c][r];
                        qv += add;
                        if (wb_q) store_field(Q + x + gi, qv, a.persist);
                    }
            }
        }
    }
    __syncthreads();
}

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
__device__ __forceinline__ void mfma_tile(const MfmaRef<K, T> &Ar, const TileArgs &a, unsigned char *smem, int tile,
                                          int f0, int nfoot, int b0, int shot) {
    MfmaTile<T> tl;
    tl.S = a.stride;
    tl.f = reinterpret_cast<T *>(smem);
    tl.acc = reinterpret_cast<uint32_t *>(tl.f + (size_t)a.nrow + (size_t)(G_NROWS + 9) * tl.S);
    tl.x = reinterpret_cast<int32_t *>(tl.acc + tl.S);
    tl.fl = reinterpret_cast<uint16_t *>(tl.x + tl.S);
    tl.nb = reinterpret_cast<uint32_t *>(tl.fl + tl.S + (tl.S & 1));
    tl.tile = tile;
    tl.shot = shot;
    tl.f0 = f0;
    tl.nfoot = nfoot;
    const int tid = threadIdx.x;
    // the tile's cells, loop bits, gather / write-back flags and geometry
    {
        const T *geo = reinterpret_cast<const T *>(a.geo);
        T *gr = tl.f + a.nrow;
        for (int s = tid; s < tl.nfoot; s += NT) {
            const uint32_t acc = a.facc[tl.f0 + s];
            const int32_t x = a.foot[tl.f0 + s];
            const bool single = acc >> 31;
            uint16_t fl = 0;
#pragma unroll
            for (int f = 0; f < F_COUNT; ++f) {
                const uint32_t m = acc & a.loops_mask[f];
                if (m && ((m & (~m + 1u)) & a.rfirst_mask[f])) fl |= 1u << f;
                if ((acc & a.writes_mask[f]) && (((a.persistent_mask >> f) & 1) || !single)) fl |= 1u << (8 + f);
            }
            tl.acc[s] = acc;
            tl.x[s] = x;
            tl.fl[s] = fl;
            T gv[G_NROWS];
#pragma unroll
            for (int r = 0; r < G_NROWS; ++r) gv[r] = geo[(int64_t)r * a.nc + x];
#pragma unroll
            for (int r = 0; r < G_NROWS; ++r) gr[(size_t)r * tl.S + s] = gv[r];
            // facet normals and scales, shared by the sub-chain's operators and by the four
            // lanes that evaluate points of a facet
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                T nx, ny, fs;
                facet_normal<T>(p, gv[G_RX], gv[G_RY], gv[G_SX], gv[G_SY], nx, ny, fs);
                gr[(size_t)(G_NROWS + 3 * p) * tl.S + s] = nx;
                gr[(size_t)(G_NROWS + 3 * p + 1) * tl.S + s] = ny;
                gr[(size_t)(G_NROWS + 3 * p + 2) * tl.S + s] = fs;
            }
        }
        // slots past the footprint in the last 16-cell group read as a valid empty cell
        for (int s = tl.nfoot + tid; s < ((tl.nfoot + 15) & ~15); s += NT) {
            tl.acc[s] = 0u;
            tl.x[s] = 0;
            tl.fl[s] = 0;
#pragma unroll
            for (int q = 0; q < 3 * NOPS; ++q) tl.nb[q * tl.S + s] = 0u;
        }
        // the neighbour tables of the tile's facet loops ([operator][facet][slot])
        for (int i = tid; i < 3 * NOPS * tl.nfoot; i += NT) {
            const int q = i / tl.nfoot, s = i - q * tl.nfoot;
            tl.nb[q * tl.S + s] = a.tnb[b0 + i];
        }
    }
    [&]<int... Q>(std::integer_sequence<int, Q...>) {
        (mfma_op<K, T, UPW, ORDER, O0, NOPS, O0 + Q, NT>(Ar, a, tl), ...);
    }(std::make_integer_sequence<int, NOPS>{});
}

template <int K, typename T, bool UPW, int ORDER, int O0, int NOPS, int NT>
__global__ __launch_bounds__(NT) void k_tile_mfma(const TileArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_next, s_shot, s_f0, s_nfoot, s_b0;
    MfmaRef<K, T> Ar;
    Ar.load(R<K, T>(), threadIdx.x & 63);
    if (!a.persist) {  // one launch per colour
        const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
        const TileMeta m = tile_meta(a, a.tile_base + item / a.nshots);
        mfma_tile<K, T, UPW, ORDER, O0, NOPS, NT>(Ar, a, smem, m.x, m.y, m.z, m.w, item % a.nshots);
        return;
    }
    for (;;) {  // dependence-driven schedule, as in the register-resident chain kernel
        if (threadIdx.x == 0) {
            const uint32_t ticket = atomicAdd(a.head, 1u) - a.head_base;
            s_next = -1;
            if (ticket < (uint32_t)a.nexec * (uint32_t)a.nshots) {
                const TileMeta m = tile_meta(a, (int)(ticket / (uint32_t)a.nshots));
                const int shot = (int)(ticket % (uint32_t)a.nshots);
                s_shot = shot;
                s_f0 = m.y;
                s_nfoot = m.z;
                s_b0 = m.w;
                if (wait_preds(a, m.x, shot, a.epoch)) s_next = m.x;  // -1 also when the wait gave up
            }
        }
        __syncthreads();
        const int tile = s_next, shot = s_shot;
        if (tile < 0) return;
        mfma_tile<K, T, UPW, ORDER, O0, NOPS, NT>(Ar, a, smem, tile, s_f0, s_nfoot, s_b0, shot);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = a.succ_off[tile]; k < a.succ_off[tile + 1]; ++k)
                __hip_atomic_fetch_add(a.cnt + (int64_t)shot * a.ntiles + a.succ[k], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace dgt
