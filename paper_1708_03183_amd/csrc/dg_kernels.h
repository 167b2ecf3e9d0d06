// Device arithmetic of the DG velocity-stress operators (gfx950), shared by
// the untiled per-loop kernels and the fused tiled executor.
//
// Folded strong form on affine cells (the block-diagonal inverse mass of the
// paper's solver loops, Sec. 7.2, is folded into the operators):
//   A(S)  = rho^-1 (Dx Sxx + Dy Sxy, Dx Sxy + Dy Syy) + sum_f fs_f rho^-1 LIFT_f (T* - T^-)
//   B(V)  = C eps(V) + sum_f fs_f LIFT_f C sym((v* - v^-) x n)
// with Dx = r_x Dr + s_x Ds, LIFT_f = Mhat^-1 E_f M1, fs_f = |facet| / |J|.
// Upwind fluxes are split into the part driven by the operated field and the
// lagged penalty driven by the other field.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgt {

constexpr int np_of(int k) { return (k + 1) * (k + 2) / 2; }

// cell node of facet node t on local facet p (facet p joins local vertices p
// and p+1, its nodes run from vertex p; cell nodes (i/K, j/K) ordered by j then i)
__host__ __device__ constexpr int fnode(int K, int p, int t) {
    return p == 0 ? t : (p == 1 ? t * (K + 1) - t * (t - 1) / 2 + (K - t) : (K - t) * (K + 1) - (K - t) * (K - t - 1) / 2);
}

template <int K, typename T>
struct RefC {
    static constexpr int NP = np_of(K), NFP = K + 1;
    T Dr[NP * NP];
    T Ds[NP * NP];
    T lift[3 * NP * NFP];
    T M[NP * NP];
    int fn[3 * NFP];
};

// geometry rows per cell (exec order, row-major [row][cell])
enum { G_RX = 0, G_RY, G_SX, G_SY, G_LAM, G_MU, G_IRHO, G_ZP, G_ZS, G_NROWS, G_DET = G_NROWS };

// data fields of the GPU chain
enum { F_V = 0, F_S, F_U, F_X, F_Z, F_COUNT };
__host__ __device__ constexpr int field_ncomp(int f) { return (f == F_V || f == F_U) ? 2 : 3; }

// kinds of loops in the GPU chain
enum LoopKind : int8_t {
    KV_VOL_V = 0, KV_VOL_S, KV_INT_V, KV_INT_S, KV_EXT_V, KV_EXT_S, KV_SOLVE,
    KV_UPD_V, KV_UPD_S, KV_UPD2_V, KV_UPD2_S
};

// scaled outward normal of local facet l from J^{-1}: m = (|e|/|J|) n
template <typename T>
__device__ __forceinline__ void facet_normal(int l, T rx, T ry, T sx, T sy, T &nx, T &ny, T &fs) {
    T mx, my;
    if (l == 0) { mx = -sx; my = -sy; }
    else if (l == 1) { mx = rx + sx; my = ry + sy; }
    else { mx = -rx; my = -ry; }
    fs = sqrt(mx * mx + my * my);
    const T inv = T(1) / fs;
    nx = mx * inv;
    ny = my * inv;
}

// interior flux of the velocity operator at one facet node.
// s0/s1: stress-like input traces (xx, yy, xy); v0/v1: penalty velocity traces.
// Outputs the traction differences already scaled by fs/rho per side.
template <typename T, bool UPW, bool PEN>
__device__ __forceinline__ void flux_v_int(const T *s0, const T *s1, const T *v0, const T *v1, T nx, T ny,
                                           T zp0, T zs0, T zp1, T zs1, T w0, T w1, T scale, T pscale,
                                           T *g0, T *g1) {
    const T T0x = s0[0] * nx + s0[2] * ny, T0y = s0[2] * nx + s0[1] * ny;
    const T T1x = s1[0] * nx + s1[2] * ny, T1y = s1[2] * nx + s1[1] * ny;
    T tsx, tsy;
    const T tx = -ny, ty = nx;
    if (!UPW) {
        tsx = T(0.5) * (T0x + T1x);
        tsy = T(0.5) * (T0y + T1y);
    } else {
        // reciprocals of the impedance sums: the same for every node of a facet, so
        // they are computed once per facet where the nodes are unrolled
        const T ip = T(1) / (zp0 + zp1), is = T(1) / (zs0 + zs1);
        const T tn = (zp1 * (T0x * nx + T0y * ny) + zp0 * (T1x * nx + T1y * ny)) * ip;
        const T tt = (zs1 * (T0x * tx + T0y * ty) + zs0 * (T1x * tx + T1y * ty)) * is;
        tsx = tn * nx + tt * tx;
        tsy = tn * ny + tt * ty;
    }
    T px = 0, py = 0;
    if (UPW && PEN) {
        const T a = zp0 * zp1 * (T(1) / (zp0 + zp1)) * ((v1[0] - v0[0]) * nx + (v1[1] - v0[1]) * ny);
        const T b = zs0 * zs1 * (T(1) / (zs0 + zs1)) * ((v1[0] - v0[0]) * tx + (v1[1] - v0[1]) * ty);
        px = a * nx + b * tx;
        py = a * ny + b * ty;
    }
    g0[0] = w0 * (scale * (tsx - T0x) + pscale * px);
    g0[1] = w0 * (scale * (tsy - T0y) + pscale * py);
    g1[0] = w1 * (scale * (T1x - tsx) - pscale * px);
    g1[1] = w1 * (scale * (T1y - tsy) - pscale * py);
}

// C sym(e x n) for isotropic (lam, mu), scaled by w
template <typename T>
__device__ __forceinline__ void csym(T ex, T ey, T nx, T ny, T lam, T mu, T w, T *out) {
    const T exx = ex * nx, eyy = ey * ny, exy = T(0.5) * (ex * ny + ey * nx);
    out[0] = w * ((lam + 2 * mu) * exx + lam * eyy);
    out[1] = w * (lam * exx + (lam + 2 * mu) * eyy);
    out[2] = w * (2 * mu * exy);
}

// interior flux of the stress operator at one facet node.
// v0/v1: velocity-like input traces; s0/s1: penalty stress traces.
template <typename T, bool UPW, bool PEN>
__device__ __forceinline__ void flux_s_int(const T *v0, const T *v1, const T *s0, const T *s1, T nx, T ny,
                                           T zp0, T zs0, T zp1, T zs1, T lam0, T mu0, T lam1, T mu1, T w0, T w1,
                                           T scale, T pscale, T *g0, T *g1) {
    const T tx = -ny, ty = nx;
    T vsx, vsy;
    if (!UPW) {
        vsx = T(0.5) * (v0[0] + v1[0]);
        vsy = T(0.5) * (v0[1] + v1[1]);
    } else {
        const T ip = T(1) / (zp0 + zp1), is = T(1) / (zs0 + zs1);
        const T vn = (zp0 * (v0[0] * nx + v0[1] * ny) + zp1 * (v1[0] * nx + v1[1] * ny)) * ip;
        const T vt = (zs0 * (v0[0] * tx + v0[1] * ty) + zs1 * (v1[0] * tx + v1[1] * ty)) * is;
        vsx = vn * nx + vt * tx;
        vsy = vn * ny + vt * ty;
    }
    T px = 0, py = 0;
    if (UPW && PEN) {
        const T T0x = s0[0] * nx + s0[2] * ny, T0y = s0[2] * nx + s0[1] * ny;
        const T T1x = s1[0] * nx + s1[2] * ny, T1y = s1[2] * nx + s1[1] * ny;
        const T a = ((T1x - T0x) * nx + (T1y - T0y) * ny) * (T(1) / (zp0 + zp1));
        const T b = ((T1x - T0x) * tx + (T1y - T0y) * ty) * (T(1) / (zs0 + zs1));
        px = a * nx + b * tx;
        py = a * ny + b * ty;
    }
    const T e0x = scale * (vsx - v0[0]) + pscale * px, e0y = scale * (vsy - v0[1]) + pscale * py;
    const T e1x = scale * (vsx - v1[0]) + pscale * px, e1y = scale * (vsy - v1[1]) + pscale * py;
    csym(e0x, e0y, nx, ny, lam0, mu0, w0, g0);
    csym(e1x, e1y, -nx, -ny, lam1, mu1, w1, g1);
}

// exterior facet of the velocity operator: free surface (mirror ghost) or
// absorbing (zero ghost, always upwind)
template <typename T, bool UPW, bool PEN>
__device__ __forceinline__ void flux_v_ext(const T *s, const T *v, bool free_surf, T nx, T ny, T zp, T zs, T w,
                                           T scale, T pscale, T *g) {
    const T Tx = s[0] * nx + s[2] * ny, Ty = s[2] * nx + s[1] * ny;
    if (free_surf) {
        g[0] = w * scale * (-Tx);
        g[1] = w * scale * (-Ty);
        return;
    }
    T px = 0, py = 0;
    if (PEN) {
        const T tx = -ny, ty = nx;
        const T vn = v[0] * nx + v[1] * ny, vt = v[0] * tx + v[1] * ty;
        px = T(-0.5) * (zp * vn * nx + zs * vt * tx);
        py = T(-0.5) * (zp * vn * ny + zs * vt * ty);
    }
    g[0] = w * (scale * T(-0.5) * Tx + pscale * px);
    g[1] = w * (scale * T(-0.5) * Ty + pscale * py);
}

template <typename T, bool UPW, bool PEN>
__device__ __forceinline__ void flux_s_ext(const T *v, const T *s, bool free_surf, T nx, T ny, T zp, T zs, T lam,
                                           T mu, T w, T scale, T pscale, T *g) {
    const T tx = -ny, ty = nx;
    T ex = 0, ey = 0;
    if (free_surf) {
        if (UPW && PEN) {
            const T Tx = s[0] * nx + s[2] * ny, Ty = s[2] * nx + s[1] * ny;
            const T a = -(Tx * nx + Ty * ny) * (T(1) / zp), b = -(Tx * tx + Ty * ty) * (T(1) / zs);
            ex = pscale * (a * nx + b * tx);
            ey = pscale * (a * ny + b * ty);
        }
    } else {
        ex = scale * T(-0.5) * v[0];
        ey = scale * T(-0.5) * v[1];
        if (PEN) {
            const T Tx = s[0] * nx + s[2] * ny, Ty = s[2] * nx + s[1] * ny;
            const T a = T(-0.5) * (Tx * nx + Ty * ny) * (T(1) / zp), b = T(-0.5) * (Tx * tx + Ty * ty) * (T(1) / zs);
            ex += pscale * (a * nx + b * tx);
            ey += pscale * (a * ny + b * ty);
        }
    }
    csym(ex, ey, nx, ny, lam, mu, w, g);
}

}  // namespace dgt
