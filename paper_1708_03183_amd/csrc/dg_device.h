#pragma once
// DG velocity-stress elastic solver of libdgtile on gfx950: the untiled loop
// chain (one kernel per loop), the executor plan (local maps), permutations
// and the FP64 energy reduction.  The tiled executor's kernels are in
// tile_kernel.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"
#include "dg_kernels.h"
#include "inspector.h"
#include "mesh.h"
#include "refconst.h"
#include "refelem.h"
#include "tile_args.h"

namespace dgt {

// ------------------------------------------------------------ untiled kernels (one per loop)
// blockIdx.y selects a shot: every field and facet buffer is offset by its shot stride

// volume term of the velocity (VEL) or stress operator: out = scale * vol(in)
template <int K, typename T, bool VEL>
__global__ __launch_bounds__(256) void k_vol(const T *__restrict__ in, T *__restrict__ out,
                                             const T *__restrict__ geo, int64_t nc, T scale, int64_t ish,
                                             int64_t osh) {
    constexpr int NP = np_of(K);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * NP) return;
    in += blockIdx.y * ish;
    out += blockIdx.y * osh;
    const int64_t c = t / NP;  // nodes of one cell are adjacent lanes: its inputs are read once
    const int i = (int)(t - c * NP);
    const auto &Rf = R<K, T>();
    const T rx = geo[G_RX * nc + c], ry = geo[G_RY * nc + c], sx = geo[G_SX * nc + c], sy = geo[G_SY * nc + c];
    constexpr int NCI = VEL ? 3 : 2;
    T ar[NCI], as[NCI];
#pragma unroll
    for (int q = 0; q < NCI; ++q) { ar[q] = 0; as[q] = 0; }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const T dr = Rf.Dr[i * NP + j], ds = Rf.Ds[i * NP + j];
#pragma unroll
        for (int q = 0; q < NCI; ++q) {
            const T u = in[((int64_t)q * NP + j) * nc + c];
            ar[q] += dr * u;
            as[q] += ds * u;
        }
    }
    if constexpr (VEL) {
        const T irho = geo[G_IRHO * nc + c];
        const T dxx = rx * ar[0] + sx * as[0];  // d/dx sxx
        const T dyy = ry * ar[1] + sy * as[1];  // d/dy syy
        const T dxy_x = rx * ar[2] + sx * as[2], dxy_y = ry * ar[2] + sy * as[2];
        out[((int64_t)0 * NP + i) * nc + c] = scale * irho * (dxx + dxy_y);
        out[((int64_t)1 * NP + i) * nc + c] = scale * irho * (dxy_x + dyy);
    } else {
        const T lam = geo[G_LAM * nc + c], mu = geo[G_MU * nc + c];
        const T exx = rx * ar[0] + sx * as[0], eyy = ry * ar[1] + sy * as[1];
        const T exy = T(0.5) * ((ry * ar[0] + sy * as[0]) + (rx * ar[1] + sx * as[1]));
        out[((int64_t)0 * NP + i) * nc + c] = scale * ((lam + 2 * mu) * exx + lam * eyy);
        out[((int64_t)1 * NP + i) * nc + c] = scale * (lam * exx + (lam + 2 * mu) * eyy);
        out[((int64_t)2 * NP + i) * nc + c] = scale * (2 * mu * exy);
    }
}

// interior-facet flux: one thread per (facet, facet node); writes the lifted
// input G[side][comp][m'][f] in each side's own facet-node order
template <int K, typename T, bool VEL, bool UPW, bool PEN>
__global__ __launch_bounds__(256) void k_flux_int(const T *__restrict__ in, const T *__restrict__ pin,
                                                  const int32_t *__restrict__ f2c, const uint8_t *__restrict__ f2l,
                                                  const T *__restrict__ geo, int64_t nc, int64_t nf, T scale,
                                                  T pscale, T *__restrict__ G, int64_t ish, int64_t psh,
                                                  int64_t gsh) {
    constexpr int NP = np_of(K), NFP = K + 1, NCO = VEL ? 2 : 3;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nf * NFP) return;
    in += blockIdx.y * ish;
    if (PEN) pin += blockIdx.y * psh;
    G += blockIdx.y * gsh;
    const int m = (int)(t / nf);
    const int64_t f = t - (int64_t)m * nf;
    const auto &Rf = R<K, T>();
    const int64_t c0 = f2c[2 * f], c1 = f2c[2 * f + 1];
    const int l0 = f2l[f] & 3, l1 = (f2l[f] >> 2) & 3;
    const int n0 = Rf.fn[l0 * NFP + m], n1 = Rf.fn[l1 * NFP + (K - m)];
    T nx, ny, fs0, fs1, tmpx, tmpy;
    facet_normal<T>(l0, geo[G_RX * nc + c0], geo[G_RY * nc + c0], geo[G_SX * nc + c0], geo[G_SY * nc + c0], nx, ny,
                    fs0);
    facet_normal<T>(l1, geo[G_RX * nc + c1], geo[G_RY * nc + c1], geo[G_SX * nc + c1], geo[G_SY * nc + c1], tmpx,
                    tmpy, fs1);
    const T zp0 = geo[G_ZP * nc + c0], zs0 = geo[G_ZS * nc + c0], zp1 = geo[G_ZP * nc + c1],
            zs1 = geo[G_ZS * nc + c1];
    T g0[3], g1[3];
    if (VEL) {
        T s0[3], s1[3], v0[2] = {0, 0}, v1[2] = {0, 0};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            s0[q] = in[((int64_t)q * NP + n0) * nc + c0];
            s1[q] = in[((int64_t)q * NP + n1) * nc + c1];
        }
        if (PEN) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                v0[q] = pin[((int64_t)q * NP + n0) * nc + c0];
                v1[q] = pin[((int64_t)q * NP + n1) * nc + c1];
            }
        }
        flux_v_int<T, UPW, PEN>(s0, s1, v0, v1, nx, ny, zp0, zs0, zp1, zs1, fs0 * geo[G_IRHO * nc + c0],
                                fs1 * geo[G_IRHO * nc + c1], scale, pscale, g0, g1);
    } else {
        T v0[2], v1[2], s0[3] = {0, 0, 0}, s1[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            v0[q] = in[((int64_t)q * NP + n0) * nc + c0];
            v1[q] = in[((int64_t)q * NP + n1) * nc + c1];
        }
        if (PEN) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                s0[q] = pin[((int64_t)q * NP + n0) * nc + c0];
                s1[q] = pin[((int64_t)q * NP + n1) * nc + c1];
            }
        }
        flux_s_int<T, UPW, PEN>(v0, v1, s0, s1, nx, ny, zp0, zs0, zp1, zs1, geo[G_LAM * nc + c0],
                                geo[G_MU * nc + c0], geo[G_LAM * nc + c1], geo[G_MU * nc + c1], fs0, fs1, scale,
                                pscale, g0, g1);
    }
#pragma unroll
    for (int q = 0; q < NCO; ++q) {
        G[((int64_t)(0 * NCO + q) * NFP + m) * nf + f] = g0[q];
        G[((int64_t)(1 * NCO + q) * NFP + (K - m)) * nf + f] = g1[q];
    }
}

template <int K, typename T, bool VEL, bool UPW, bool PEN>
__global__ __launch_bounds__(256) void k_flux_ext(const T *__restrict__ in, const T *__restrict__ pin,
                                                  const int32_t *__restrict__ b2c, const uint8_t *__restrict__ b2l,
                                                  const T *__restrict__ geo, int64_t nc, int64_t nb, T scale,
                                                  T pscale, T *__restrict__ G, int64_t ish, int64_t psh,
                                                  int64_t gsh) {
    constexpr int NP = np_of(K), NFP = K + 1, NCO = VEL ? 2 : 3;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * NFP) return;
    in += blockIdx.y * ish;
    if (PEN) pin += blockIdx.y * psh;
    G += blockIdx.y * gsh;
    const int m = (int)(t / nb);
    const int64_t b = t - (int64_t)m * nb;
    const auto &Rf = R<K, T>();
    const int64_t c = b2c[b];
    const int l = b2l[b] & 3;
    const bool fr = (b2l[b] >> 2) & 1;
    const int nd = Rf.fn[l * NFP + m];
    T nx, ny, fs;
    facet_normal<T>(l, geo[G_RX * nc + c], geo[G_RY * nc + c], geo[G_SX * nc + c], geo[G_SY * nc + c], nx, ny, fs);
    const T zp = geo[G_ZP * nc + c], zs = geo[G_ZS * nc + c];
    T g[3];
    if (VEL) {
        T s[3], v[2] = {0, 0};
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] = in[((int64_t)q * NP + nd) * nc + c];
        if (PEN) {
#pragma unroll
            for (int q = 0; q < 2; ++q) v[q] = pin[((int64_t)q * NP + nd) * nc + c];
        }
        flux_v_ext<T, UPW, PEN>(s, v, fr, nx, ny, zp, zs, fs * geo[G_IRHO * nc + c], scale, pscale, g);
    } else {
        T v[2], s[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) v[q] = in[((int64_t)q * NP + nd) * nc + c];
        if (PEN) {
#pragma unroll
            for (int q = 0; q < 3; ++q) s[q] = pin[((int64_t)q * NP + nd) * nc + c];
        }
        flux_s_ext<T, UPW, PEN>(v, s, fr, nx, ny, zp, zs, geo[G_LAM * nc + c], geo[G_MU * nc + c], fs, scale,
                                pscale, g);
    }
#pragma unroll
    for (int q = 0; q < NCO; ++q) G[((int64_t)q * NFP + m) * nb + b] = g[q];
}

// lift of the facet terms into the cell's accumulator (increments of the
// interior- and exterior-facet loops), local facets in order 0, 1, 2
template <int K, typename T, bool VEL>
__global__ __launch_bounds__(256) void k_lift(T *__restrict__ out, const int32_t *__restrict__ c2f,
                                              const T *__restrict__ G, const T *__restrict__ Gx, int64_t nc,
                                              int64_t nf, int64_t nb, int64_t osh, int64_t gsh, int64_t gxsh) {
    constexpr int NP = np_of(K), NFP = K + 1, NCO = VEL ? 2 : 3;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * NP) return;
    out += blockIdx.y * osh;
    G += blockIdx.y * gsh;
    Gx += blockIdx.y * gxsh;
    const int64_t c = t / NP;
    const int i = (int)(t - c * NP);
    const auto &Rf = R<K, T>();
    T acc[NCO];
#pragma unroll
    for (int q = 0; q < NCO; ++q) acc[q] = 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int32_t code = c2f[(int64_t)p * nc + c];
        if (code >= 0) {
            const int64_t f = code >> 1;
            const int s = code & 1;
#pragma unroll
            for (int q = 0; q < NCO; ++q)
#pragma unroll
                for (int m = 0; m < NFP; ++m)
                    acc[q] += Rf.lift[(p * NP + i) * NFP + m] * G[((int64_t)(s * NCO + q) * NFP + m) * nf + f];
        } else {
            const int64_t b = -(int64_t)code - 1;
#pragma unroll
            for (int q = 0; q < NCO; ++q)
#pragma unroll
                for (int m = 0; m < NFP; ++m)
                    acc[q] += Rf.lift[(p * NP + i) * NFP + m] * Gx[((int64_t)q * NFP + m) * nb + b];
        }
    }
#pragma unroll
    for (int q = 0; q < NCO; ++q) out[((int64_t)q * NP + i) * nc + c] += acc[q];
}

// One whole operator application per cell (volume term, the cell's side of its three
// facets, lift) in one pass: out = scale * op(in) (+ pscale * the upwind penalty of pin).
// The same arithmetic as k_vol, k_flux_int / k_flux_ext and k_lift: each facet's flux
// is evaluated from the cell's own side (its outward normal, the neighbour's trace at the
// matching node as the other side), which is the other side's value of the facet-loop
// form with the two cells and the sign of the normal exchanged.  One thread per cell;
// the facet terms never leave registers.  blockIdx.y selects a shot.
template <int K, typename T, bool VEL, bool UPW, bool PEN>
__global__ __launch_bounds__(256) void k_op_cell(const T *__restrict__ in, const T *__restrict__ pin,
                                                 T *__restrict__ out, const int32_t *__restrict__ c2f,
                                                 const int32_t *__restrict__ f2c, const uint8_t *__restrict__ f2l,
                                                 const uint8_t *__restrict__ b2l, const T *__restrict__ geo,
                                                 int64_t nc, T scale, T pscale, int64_t ish, int64_t osh,
                                                 int64_t psh) {
    constexpr int NP = np_of(K), NFP = K + 1, NCI = VEL ? 3 : 2, NCO = VEL ? 2 : 3;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    in += blockIdx.y * ish;
    out += blockIdx.y * osh;
    if (PEN) pin += blockIdx.y * psh;
    const auto &Rf = R<K, T>();
    const T rx = geo[G_RX * nc + c], ry = geo[G_RY * nc + c], sx = geo[G_SX * nc + c], sy = geo[G_SY * nc + c];
    const T zp0 = geo[G_ZP * nc + c], zs0 = geo[G_ZS * nc + c];
    T u[NCI][NP], o[NCO][NP];
#pragma unroll
    for (int q = 0; q < NCI; ++q)
#pragma unroll
        for (int j = 0; j < NP; ++j) u[q][j] = in[((int64_t)q * NP + j) * nc + c];
    // volume term
    const T irho = VEL ? geo[G_IRHO * nc + c] : T(0);
    const T lam = VEL ? T(0) : geo[G_LAM * nc + c], mu = VEL ? T(0) : geo[G_MU * nc + c];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        T ar[NCI], as[NCI];
#pragma unroll
        for (int q = 0; q < NCI; ++q) ar[q] = as[q] = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const T dr = Rf.Dr[i * NP + j], ds = Rf.Ds[i * NP + j];
#pragma unroll
            for (int q = 0; q < NCI; ++q) {
                ar[q] += dr * u[q][j];
                as[q] += ds * u[q][j];
            }
        }
        if constexpr (VEL) {
            const T dxx = rx * ar[0] + sx * as[0], dyy = ry * ar[1] + sy * as[1];
            const T dxy_x = rx * ar[2] + sx * as[2], dxy_y = ry * ar[2] + sy * as[2];
            o[0][i] = scale * irho * (dxx + dxy_y);
            o[1][i] = scale * irho * (dxy_x + dyy);
        } else {
            const T exx = rx * ar[0] + sx * as[0], eyy = ry * ar[1] + sy * as[1];
            const T exy = T(0.5) * ((ry * ar[0] + sy * as[0]) + (rx * ar[1] + sx * as[1]));
            o[0][i] = scale * ((lam + 2 * mu) * exx + lam * eyy);
            o[1][i] = scale * (lam * exx + (lam + 2 * mu) * eyy);
            o[2][i] = scale * (2 * mu * exy);
        }
    }
    // facet terms, lifted at once
    T lacc[NCO][NP];
#pragma unroll
    for (int q = 0; q < NCO; ++q)
#pragma unroll
        for (int i = 0; i < NP; ++i) lacc[q][i] = 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        T nx, ny, fs;
        facet_normal<T>(p, rx, ry, sx, sy, nx, ny, fs);
        const int32_t code = c2f[(int64_t)p * nc + c];
        T g[NFP][3];
        if (code >= 0) {
            const int64_t f = code >> 1;
            const int side = code & 1;
            const int64_t c1 = f2c[2 * f + (1 - side)];
            const int l1 = side == 0 ? (f2l[f] >> 2) & 3 : f2l[f] & 3;
            const T zp1 = geo[G_ZP * nc + c1], zs1 = geo[G_ZS * nc + c1];
#pragma unroll
            for (int m = 0; m < NFP; ++m) {
                const int n0 = fnode(K, p, m), n1 = Rf.fn[l1 * NFP + (K - m)];
                T a0[3], a1[3], p0[3] = {0, 0, 0}, p1[3] = {0, 0, 0}, g1[3];
#pragma unroll
                for (int q = 0; q < NCI; ++q) {
                    a0[q] = u[q][n0];
                    a1[q] = in[((int64_t)q * NP + n1) * nc + c1];
                }
                if (PEN) {
#pragma unroll
                    for (int q = 0; q < NCO; ++q) {
                        p0[q] = pin[((int64_t)q * NP + n0) * nc + c];
                        p1[q] = pin[((int64_t)q * NP + n1) * nc + c1];
                    }
                }
                if constexpr (VEL)
                    flux_v_int<T, UPW, PEN>(a0, a1, p0, p1, nx, ny, zp0, zs0, zp1, zs1, fs * irho, T(0), scale,
                                            pscale, g[m], g1);
                else
                    flux_s_int<T, UPW, PEN>(a0, a1, p0, p1, nx, ny, zp0, zs0, zp1, zs1, lam, mu, lam, mu, fs, T(0),
                                            scale, pscale, g[m], g1);
            }
        } else {
            const int64_t b = -(int64_t)code - 1;
            const bool fr = (b2l[b] >> 2) & 1;
#pragma unroll
            for (int m = 0; m < NFP; ++m) {
                const int n0 = fnode(K, p, m);
                T a0[3], p0[3] = {0, 0, 0};
#pragma unroll
                for (int q = 0; q < NCI; ++q) a0[q] = u[q][n0];
                if (PEN) {
#pragma unroll
                    for (int q = 0; q < NCO; ++q) p0[q] = pin[((int64_t)q * NP + n0) * nc + c];
                }
                if constexpr (VEL)
                    flux_v_ext<T, UPW, PEN>(a0, p0, fr, nx, ny, zp0, zs0, fs * irho, scale, pscale, g[m]);
                else
                    flux_s_ext<T, UPW, PEN>(a0, p0, fr, nx, ny, zp0, zs0, lam, mu, fs, scale, pscale, g[m]);
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int q = 0; q < NCO; ++q)
#pragma unroll
                for (int m = 0; m < NFP; ++m) lacc[q][i] += Rf.lift[(p * NP + i) * NFP + m] * g[m][q];
    }
#pragma unroll
    for (int q = 0; q < NCO; ++q)
#pragma unroll
        for (int i = 0; i < NP; ++i) out[((int64_t)q * NP + i) * nc + c] = o[q][i] + lacc[q][i];
}

// v += dt*U + Z (order 4) ; v += Z (order 2, dt folded into Z)
template <typename T>
__global__ __launch_bounds__(256) void k_upd_v(T *__restrict__ V, const T *__restrict__ U, const T *__restrict__ Z,
                                               int64_t n, T dt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    V[t] += (U ? dt * U[t] : T(0)) + Z[t];
}

// s += dt*X + Z + dt r(t) Mk^-1 phi(x_s) on sxx, syy of the source cell
template <int K, typename T>
__global__ __launch_bounds__(256) void k_upd_s(T *__restrict__ S, const T *__restrict__ X, const T *__restrict__ Z,
                                               int64_t nc, T dt, int64_t src_cell, T src_amp,
                                               const T *__restrict__ src_vec) {
    constexpr int NP = np_of(K);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * NP * nc) return;
    const int64_t row = t / nc, c = t - row * nc;
    T add = (X ? dt * X[t] : T(0)) + Z[t];
    if (c == src_cell && row < 2 * NP) add += src_amp * src_vec[row % NP];
    S[t] += add;
}

// ------------------------------------------------------------ plan kernels (local maps)

__global__ void k_rank_keys(const int32_t *__restrict__ foot_off, const int32_t *__restrict__ foot,
                            const int32_t *__restrict__ rank, int32_t ntiles, int64_t len,
                            uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    // tile of entry i by binary search in foot_off
    int lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (foot_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    keys[i] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)rank[foot[i]];
}

__global__ void k_split_keys(const uint64_t *__restrict__ keys, int64_t len, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] = (int32_t)(keys[i] & 0xffffffffull);
}

__device__ __forceinline__ int slot_of(const int32_t *__restrict__ foot, int b, int e, int32_t x) {
    int lo = b, hi = e;  // first position with foot >= x
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (foot[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo - b;
}

// kind: 0 cell loop, 1 interior facet loop, 2 exterior facet loop
// (iterations of tile skip, the never-executed tile of a region-aware schedule, get 0)
__global__ void k_lmap(int kind, const int32_t *__restrict__ it_off, const int32_t *__restrict__ iters, int32_t ntiles,
                       int32_t skip, int64_t n, const int32_t *__restrict__ foot_off, const int32_t *__restrict__ efoot,
                       const int32_t *__restrict__ rank, const int32_t *__restrict__ f2c,
                       const int8_t *__restrict__ f2l, const int32_t *__restrict__ b2c,
                       const int8_t *__restrict__ b2l, const uint8_t *__restrict__ bfree,
                       uint32_t *__restrict__ lmap, int32_t *__restrict__ err) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (it_off[mid] <= q) lo = mid;
        else hi = mid;
    }
    if (lo == skip) {
        lmap[q] = 0u;
        return;
    }
    const int b = foot_off[lo], e = foot_off[lo + 1];
    const int32_t it = iters[q];
    uint32_t code = 0;
    if (kind == 0) {
        const int s = slot_of(efoot, b, e, rank[it]);
        if (s >= e - b || efoot[b + s] != rank[it] || s > 0x3fff) atomicExch(err, 1);
        code = (uint32_t)s;
    } else if (kind == 1) {
        const int32_t x0 = rank[f2c[2 * it]], x1 = rank[f2c[2 * it + 1]];
        const int s0 = slot_of(efoot, b, e, x0), s1 = slot_of(efoot, b, e, x1);
        if (s0 >= e - b || s1 >= e - b || efoot[b + s0] != x0 || efoot[b + s1] != x1 || s0 > 0x3fff || s1 > 0x3fff)
            atomicExch(err, 1);
        code = (uint32_t)s0 | ((uint32_t)s1 << 14) | ((uint32_t)f2l[2 * it] << 28) | ((uint32_t)f2l[2 * it + 1] << 30);
    } else {
        const int32_t x = rank[b2c[it]];
        const int s = slot_of(efoot, b, e, x);
        if (s >= e - b || efoot[b + s] != x || s > 0x3fff) atomicExch(err, 1);
        code = (uint32_t)s | ((uint32_t)b2l[it] << 28) | ((uint32_t)bfree[it] << 30);
    }
    lmap[q] = code;
}

// ------------------------------------------------------------ permutation and energy

template <typename T>
__global__ void k_permute_rows(const T *__restrict__ src, T *__restrict__ dst, const int32_t *__restrict__ map,
                               int64_t rows, int64_t nc, int to_exec) {
    // to_exec: dst[r][rank[c]] = src[r][c] with map = rank; else dst[r][c] = src[r][rank[c]]
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * nc) return;
    const int64_t r = t / nc, c = t - r * nc;
    if (to_exec) dst[r * nc + map[c]] = src[t];
    else dst[t] = src[r * nc + map[c]];
}

// Halo buffers: buf[q][r][i] = field[q][r][rank[cells[i]]] (pack) or the reverse
// (unpack), for nshots copies of `rows` rows; cells were checked against nc.
template <typename T>
__global__ void k_halo_copy(T *__restrict__ fld, T *__restrict__ buf, const int32_t *__restrict__ rank,
                            const int32_t *__restrict__ cells, int64_t n, int64_t rows, int64_t nc, int64_t total,
                            int unpack) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t qr = t / n, i = t - qr * n;  // qr = shot * rows + row
    const int64_t f = qr * nc + rank[cells[i]];
    if (unpack) fld[f] = buf[t];
    else buf[t] = fld[f];
}

template <int K, typename T>
__global__ __launch_bounds__(256) void k_energy(const T *__restrict__ v, const T *__restrict__ sn,
                                                const T *__restrict__ so, const T *__restrict__ geo,
                                                const int32_t *__restrict__ rank, int64_t nc,
                                                double *__restrict__ partial) {
    constexpr int NP = np_of(K);
    __shared__ double red[256];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (c < nc) {
        const auto &Rf = R<K, T>();
        const int64_t x = rank[c];
        const double lam = geo[G_LAM * nc + x], mu = geo[G_MU * nc + x], rho = 1.0 / (double)geo[G_IRHO * nc + x];
        const double det = geo[G_DET * nc + x];
        const double cA = (lam + 2 * mu) / (4 * mu * (lam + mu)), cB = -lam / (4 * mu * (lam + mu)), cC = 1.0 / mu;
        for (int i = 0; i < NP; ++i)
            for (int j = 0; j < NP; ++j) {
                const double M = (double)Rf.M[i * NP + j];
                const double ke = (double)v[(int64_t)i * nc + c] * v[(int64_t)j * nc + c] +
                                  (double)v[((int64_t)NP + i) * nc + c] * v[((int64_t)NP + j) * nc + c];
                const double axx = sn[(int64_t)i * nc + c], ayy = sn[((int64_t)NP + i) * nc + c],
                             axy = sn[((int64_t)2 * NP + i) * nc + c];
                const double bxx = so[(int64_t)j * nc + c], byy = so[((int64_t)NP + j) * nc + c],
                             bxy = so[((int64_t)2 * NP + j) * nc + c];
                const double se = cA * (axx * bxx + ayy * byy) + cB * (axx * byy + ayy * bxx) + cC * axy * bxy;
                e += M * (rho * ke + se);
            }
        e *= 0.5 * det;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double *__restrict__ p, int64_t n, double *__restrict__ out) {
    __shared__ double red[256];
    double e = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) e += p[i];
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// geometry rows in exec order (input-order arrays permuted by rank)
template <typename T>
__global__ void k_geometry(const double *__restrict__ xy, const int32_t *__restrict__ c2v,
                           const double *__restrict__ lam, const double *__restrict__ mu,
                           const double *__restrict__ rho, const int32_t *__restrict__ rank, int64_t nc,
                           T *__restrict__ geo) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *p0 = xy + 2 * c2v[3 * c], *p1 = xy + 2 * c2v[3 * c + 1], *p2 = xy + 2 * c2v[3 * c + 2];
    const double xr = p1[0] - p0[0], xs = p2[0] - p0[0], yr = p1[1] - p0[1], ys = p2[1] - p0[1];
    const double det = xr * ys - xs * yr;
    const int64_t x = rank[c];
    geo[G_RX * nc + x] = (T)(ys / det);
    geo[G_RY * nc + x] = (T)(-xs / det);
    geo[G_SX * nc + x] = (T)(-yr / det);
    geo[G_SY * nc + x] = (T)(xr / det);
    geo[G_LAM * nc + x] = (T)lam[c];
    geo[G_MU * nc + x] = (T)mu[c];
    geo[G_IRHO * nc + x] = (T)(1.0 / rho[c]);
    geo[G_ZP * nc + x] = (T)sqrt(rho[c] * (lam[c] + 2.0 * mu[c]));
    geo[G_ZS * nc + x] = (T)sqrt(rho[c] * mu[c]);
    geo[G_DET * nc + x] = (T)det;
}

__global__ void k_centroids(const double *__restrict__ xy, const int32_t *__restrict__ c2v, int64_t nc,
                            double *__restrict__ cxy) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *p0 = xy + 2 * c2v[3 * c], *p1 = xy + 2 * c2v[3 * c + 1], *p2 = xy + 2 * c2v[3 * c + 2];
    // ((x0 + x1) + x2) / 3 with no contraction: the seed order depends on these bits
    cxy[2 * c] = __ddiv_rn(__dadd_rn(__dadd_rn(p0[0], p1[0]), p2[0]), 3.0);
    cxy[2 * c + 1] = __ddiv_rn(__dadd_rn(__dadd_rn(p0[1], p1[1]), p2[1]), 3.0);
}

}  // namespace dgt
