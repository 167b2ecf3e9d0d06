// Gradient kernels of the full-waveform inversion for the upwind flux and absorbing
// boundaries (included by fwi_impl.h; an extension beyond the paper, which runs the
// forward chain only).
//
// Notation: A (stress -> velocity rate) and B (velocity -> stress rate) are the
// operator parts of the DG operators, Dv and Ds the penalties of the upwind flux
// (velocity-jump traction, traction-jump velocity).  In the energy inner product
// W = blockdiag(rho M_J, M_J C^-1) the operator parts are skew, W_v A = -(W_s B)^T, and
// the penalties self-adjoint, with the exact Riemann weights at impedance jumps and
// with free-surface or absorbing ghosts alike, so with alpha = W^-1 lambda the
// transposed step is
//   alpha_v <- alpha_v - (dt A + c A B A) alpha_s,   alpha_s <- alpha_s + dt Ds alpha_s,
//   then alpha_s <- alpha_s - (dt B + c B A B) alpha_v,   alpha_v <- alpha_v + dt Dv alpha_v
// (the second line with the alpha_v of the first; c = dt^3/24 at order 4, else 0).
//
// The gradient of one step is a sum of terms a^T W dOp b over pairs (a, b) of adjoint-
// and forward-side vectors, Op in {A, B, Dv, Ds}.  With Op = W^-1 Op~ each term splits
// into a cell part -a^T (dW) (Op b), dW_v/drho = M_J and dW_s/dm = -M_J (x) C^-1 C_m C^-1,
// and a facet part a^T dOp~ b: Op~ holds the material only in the facet weights of the
// flux, functions of the impedances Zp = sqrt(rho (lam + 2 mu)) and Zs = sqrt(rho mu) of
// the two cells (per facet, normal components with Zp, tangential ones with Zs; [x] =
// x(side 0) - x(side 1), T(s) = s n the traction with the normal n of side 0, S = Z0 + Z1):
//   A:  int [a] . T*,  T* = (Z1 T(b)0 + Z0 T(b)1) / S
//   B:  int [T(a)] . v*, v* = (Z0 b0 + Z1 b1) / S
//   Dv: -int (Z0 Z1 / S) [a] . [b]
//   Ds: -int [T(a)] . [T(b)] / S
// and at exterior facets, whose ghost has the cell's own impedances, Dv (absorbing)
// -int (Z/2) a . b, Ds -int T(a) . T(b) / Z (free surface) or / (2Z) (absorbing); A and B
// do not depend on the impedances there.  The integrals are exact on the facet nodes
// with the facet mass matrix, as in the forward flux.

namespace dgt {

enum FwiKind { FK_A = 0, FK_B = 1, FK_DV = 2, FK_DS = 3 };

// pairs (a, b) whose gradient terms one launch sums
constexpr int FWI_MAX_PAIRS = 12;

struct FacetMass {
    double m[25];  // [nfp][nfp] reference facet mass on [0, 1]
};

// out = c0 x0 + c1 x1 + c2 x2 + c3 x3 (null terms skipped; out may alias x0)
template <typename T>
__global__ __launch_bounds__(256) void k_fwi_lin(T *out, const T *x0, double c0, const T *x1, double c1, const T *x2,
                                                 double c2, const T *x3, double c3, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double v = c0 * (double)x0[t];
    if (x1) v += c1 * (double)x1[t];
    if (x2) v += c2 * (double)x2[t];
    if (x3) v += c3 * (double)x3[t];
    out[t] = (T)v;
}

// Cell parts of coef * a^T W dOp b for several pairs (a, ob = Op b) in one pass, one
// thread per cell and shot (blockIdx.y): velocity kinds (A, Dv) add -coef |J| a . M ob
// to d/drho, stress kinds (B, Ds) add coef |J| sum_j (C^-1 (M a)_j) . C_m (C^-1 ob_j)
// to d/dlam and d/dmu; the sums of all pairs are added to part once.
template <typename T>
struct FwiCellPairs {
    int n;
    int kind[FWI_MAX_PAIRS];
    const T *a[FWI_MAX_PAIRS];
    const T *ob[FWI_MAX_PAIRS];
    int64_t sh[FWI_MAX_PAIRS];
    double coef[FWI_MAX_PAIRS];
};

template <int K, typename T>
__global__ __launch_bounds__(256) void k_fwi_cell_pairs(const FwiCellPairs<T> P, const T *__restrict__ geo,
                                                        int64_t nc, double *__restrict__ part) {
    constexpr int NP = np_of(K);
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nc) return;
    const int q = blockIdx.y;
    const auto &Rf = R<K, T>();
    const double det = geo[G_DET * nc + x];
    const double lam = geo[G_LAM * nc + x], mu = geo[G_MU * nc + x];
    const double cA = (lam + 2 * mu) / (4 * mu * (lam + mu)), cB = -lam / (4 * mu * (lam + mu)), cC = 1.0 / mu;
    double gr = 0.0, gl = 0.0, gm = 0.0;
    for (int p = 0; p < P.n; ++p) {
        const T *a = P.a[p] + q * P.sh[p], *ob = P.ob[p] + q * P.sh[p];
        const double coef = P.coef[p];
        if (P.kind[p] == FK_A || P.kind[p] == FK_DV) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    double ma = 0.0;
#pragma unroll
                    for (int i = 0; i < NP; ++i)
                        ma += (double)a[(int64_t)(c * NP + i) * nc + x] * (double)Rf.M[i * NP + j];
                    acc += ma * (double)ob[(int64_t)(c * NP + j) * nc + x];
                }
            gr -= coef * det * acc;
        } else {
            double sl = 0.0, sm = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                double ma[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ma[c] = 0.0;
#pragma unroll
                    for (int i = 0; i < NP; ++i)
                        ma[c] += (double)a[(int64_t)(c * NP + i) * nc + x] * (double)Rf.M[i * NP + j];
                }
                const double b0 = (double)ob[(int64_t)(0 * NP + j) * nc + x],
                             b1 = (double)ob[(int64_t)(1 * NP + j) * nc + x],
                             b2 = (double)ob[(int64_t)(2 * NP + j) * nc + x];
                const double ax = cA * ma[0] + cB * ma[1], ay = cB * ma[0] + cA * ma[1], axy = cC * ma[2];
                const double ex = cA * b0 + cB * b1, ey = cB * b0 + cA * b1, exy = cC * b2;
                sl += (ax + ay) * (ex + ey);
                sm += 2 * (ax * ex + ay * ey) + axy * exy;
            }
            gl += coef * det * sl;
            gm += coef * det * sm;
        }
    }
    double *o = part + (int64_t)q * 3 * nc;
    o[x] += gl;
    o[nc + x] += gm;
    o[2 * nc + x] += gr;
}

// impedance derivatives of one side -> (d/dlam, d/dmu, d/drho)
__device__ __forceinline__ void fwi_chain_z(double dzp, double dzs, double lam, double mu, double rho, double zp,
                                            double zs, double *o) {
    o[0] += dzp * rho / (2 * zp);
    o[1] += dzp * rho / zp + (zs > 0 ? dzs * rho / (2 * zs) : 0.0);
    o[2] += dzp * (lam + 2 * mu) / (2 * zp) + (zs > 0 ? dzs * mu / (2 * zs) : 0.0);
}

// <x, y> with the facet mass over the facet nodes
template <int NFP>
__device__ __forceinline__ double fwi_fdot(const FacetMass &m1, const double (&x)[NFP], const double (&y)[NFP]) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NFP; ++i)
#pragma unroll
        for (int j = 0; j < NFP; ++j) s += x[i] * m1.m[i * NFP + j] * y[j];
    return s;
}

// Facet parts of coef * a^T dOp~ b at interior facets for several pairs (a, b) in one
// pass (one thread per facet and shot): the impedance derivatives of every pair are
// summed per facet side, then turned into (lam, mu, rho) derivatives and added to
// fb[shot][facet][side][lam, mu, rho] once (the conversion is linear), so fb is read and
// written once per reversed step.  Velocity-like fields have 2 components, stress-like
// ones 3 (a: the output kind of Op, b: its input kind).
template <typename T>
struct FwiPairs {
    int n;
    int kind[FWI_MAX_PAIRS];
    const T *a[FWI_MAX_PAIRS];
    const T *b[FWI_MAX_PAIRS];
    int64_t ash[FWI_MAX_PAIRS], bsh[FWI_MAX_PAIRS];
    double coef[FWI_MAX_PAIRS];
};

template <int K, typename T>
__global__ __launch_bounds__(256) void k_fwi_facet_pairs(const FwiPairs<T> P, const int32_t *__restrict__ ef2c,
                                                         const uint8_t *__restrict__ ef2l, const T *__restrict__ geo,
                                                         int64_t nc, int64_t nf, FacetMass m1,
                                                         double *__restrict__ fb) {
    constexpr int NP = np_of(K), NFP = K + 1;
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int q = blockIdx.y;
    const auto &Rf = R<K, T>();
    const int64_t c[2] = {ef2c[2 * f], ef2c[2 * f + 1]};
    const int l0 = ef2l[f] & 3, l1 = (ef2l[f] >> 2) & 3;
    T nxT, nyT, fsT;
    facet_normal<T>(l0, geo[G_RX * nc + c[0]], geo[G_RY * nc + c[0]], geo[G_SX * nc + c[0]], geo[G_SY * nc + c[0]], nxT,
                    nyT, fsT);
    const double nx = nxT, ny = nyT, tx = -ny, ty = nx;
    const double len = (double)fsT * (double)geo[G_DET * nc + c[0]];
    double zp[2], zs[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        zp[s] = geo[G_ZP * nc + c[s]];
        zs[s] = geo[G_ZS * nc + c[s]];
    }
    const double Sp = zp[0] + zp[1], Ss = zs[0] + zs[1];
    int node[2][NFP];
#pragma unroll
    for (int m = 0; m < NFP; ++m) {
        node[0][m] = Rf.fn[l0 * NFP + m];
        node[1][m] = Rf.fn[l1 * NFP + (K - m)];
    }
    // velocity-like field at node m of side s: components along n and t; stress-like:
    // its traction with the normal of side 0, along n and t
    auto nt = [&](const T *F, bool stress, int s, int m, double &vn, double &vt) {
        const int64_t x = c[s];
        const int nd = node[s][m];
        double wx, wy;
        if (stress) {
            const double sxx = F[(int64_t)(0 * NP + nd) * nc + x], syy = F[(int64_t)(1 * NP + nd) * nc + x],
                         sxy = F[(int64_t)(2 * NP + nd) * nc + x];
            wx = sxx * nx + sxy * ny;
            wy = sxy * nx + syy * ny;
        } else {
            wx = F[(int64_t)(0 * NP + nd) * nc + x];
            wy = F[(int64_t)(1 * NP + nd) * nc + x];
        }
        vn = wx * nx + wy * ny;
        vt = wx * tx + wy * ty;
    };
    double dzp[2] = {0.0, 0.0}, dzs[2] = {0.0, 0.0};
    for (int i = 0; i < P.n; ++i) {
        const int kind = P.kind[i];
        const T *a = P.a[i] + q * P.ash[i], *b = P.b[i] + q * P.bsh[i];
        const bool as_ = kind == FK_B || kind == FK_DS, bs_ = kind == FK_A || kind == FK_DS;
        double xn[NFP], xt[NFP], yn[NFP], yt[NFP];
#pragma unroll
        for (int m = 0; m < NFP; ++m) {
            double a0n, a0t, a1n, a1t, b0n, b0t, b1n, b1t;
            nt(a, as_, 0, m, a0n, a0t);
            nt(a, as_, 1, m, a1n, a1t);
            nt(b, bs_, 0, m, b0n, b0t);
            nt(b, bs_, 1, m, b1n, b1t);
            xn[m] = a0n - a1n;
            xt[m] = a0t - a1t;
            yn[m] = kind == FK_A ? b1n - b0n : b0n - b1n;
            yt[m] = kind == FK_A ? b1t - b0t : b0t - b1t;
        }
        const double Pn = P.coef[i] * len * fwi_fdot<NFP>(m1, xn, yn), Pt = P.coef[i] * len * fwi_fdot<NFP>(m1, xt, yt);
        if (kind == FK_A || kind == FK_B) {
            dzp[0] += zp[1] * Pn / (Sp * Sp);
            dzp[1] += -zp[0] * Pn / (Sp * Sp);
            dzs[0] += Ss > 0 ? zs[1] * Pt / (Ss * Ss) : 0.0;
            dzs[1] += Ss > 0 ? -zs[0] * Pt / (Ss * Ss) : 0.0;
        } else if (kind == FK_DV) {
            dzp[0] += -zp[1] * zp[1] * Pn / (Sp * Sp);
            dzp[1] += -zp[0] * zp[0] * Pn / (Sp * Sp);
            dzs[0] += Ss > 0 ? -zs[1] * zs[1] * Pt / (Ss * Ss) : 0.0;
            dzs[1] += Ss > 0 ? -zs[0] * zs[0] * Pt / (Ss * Ss) : 0.0;
        } else {
            dzp[0] += Pn / (Sp * Sp);
            dzp[1] += Pn / (Sp * Sp);
            dzs[0] += Ss > 0 ? Pt / (Ss * Ss) : 0.0;
            dzs[1] += Ss > 0 ? Pt / (Ss * Ss) : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int64_t x = c[s];
        double o[3] = {0, 0, 0};
        fwi_chain_z(dzp[s], dzs[s], geo[G_LAM * nc + x], geo[G_MU * nc + x], 1.0 / (double)geo[G_IRHO * nc + x], zp[s],
                    zs[s], o);
        double *d = fb + (((int64_t)q * nf + f) * 2 + s) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] += o[k];
    }
}

// Exterior-facet part (penalties only): Dv at absorbing facets, Ds at absorbing facets
// and, with the upwind flux (upw), at free surfaces; added to eb[shot][facet][lam, mu, rho].
template <int K, typename T, int KIND>
__global__ __launch_bounds__(256) void k_fwi_ext_pair(const T *__restrict__ a, const T *__restrict__ b, int64_t sh,
                                                      const int32_t *__restrict__ eb2c, const uint8_t *__restrict__ eb2l,
                                                      const T *__restrict__ geo, int64_t nc, int64_t nb, FacetMass m1,
                                                      double coef, int upw, double *__restrict__ eb) {
    constexpr int NP = np_of(K), NFP = K + 1;
    constexpr bool ST = KIND == FK_DS;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb) return;
    const int q = blockIdx.y;
    a += q * sh;
    b += q * sh;
    const bool free_surf = (eb2l[e] >> 2) & 1;
    if (KIND == FK_DV && free_surf) return;  // the mirror ghost has no velocity jump
    if (free_surf && !upw) return;           // free surfaces take the central flux then: no penalty
    const auto &Rf = R<K, T>();
    const int64_t x = eb2c[e];
    const int l = eb2l[e] & 3;
    T nxT, nyT, fsT;
    facet_normal<T>(l, geo[G_RX * nc + x], geo[G_RY * nc + x], geo[G_SX * nc + x], geo[G_SY * nc + x], nxT, nyT, fsT);
    const double nx = nxT, ny = nyT, tx = -ny, ty = nx;
    const double len = (double)fsT * (double)geo[G_DET * nc + x];
    auto nt = [&](const T *F, int m, double &vn, double &vt) {
        const int node = Rf.fn[l * NFP + m];
        double wx, wy;
        if (ST) {
            const double sxx = F[(int64_t)(0 * NP + node) * nc + x], syy = F[(int64_t)(1 * NP + node) * nc + x],
                         sxy = F[(int64_t)(2 * NP + node) * nc + x];
            wx = sxx * nx + sxy * ny;
            wy = sxy * nx + syy * ny;
        } else {
            wx = F[(int64_t)(0 * NP + node) * nc + x];
            wy = F[(int64_t)(1 * NP + node) * nc + x];
        }
        vn = wx * nx + wy * ny;
        vt = wx * tx + wy * ty;
    };
    double xn[NFP], xt[NFP], yn[NFP], yt[NFP];
#pragma unroll
    for (int m = 0; m < NFP; ++m) {
        nt(a, m, xn[m], xt[m]);
        nt(b, m, yn[m], yt[m]);
    }
    const double Pn = coef * len * fwi_fdot<NFP>(m1, xn, yn), Pt = coef * len * fwi_fdot<NFP>(m1, xt, yt);
    const double zp = geo[G_ZP * nc + x], zs = geo[G_ZS * nc + x];
    double dzp, dzs;
    if (KIND == FK_DV) {  // -int (Z/2) a . b
        dzp = -0.5 * Pn;
        dzs = -0.5 * Pt;
    } else {  // -int T(a) . T(b) / (w Z): free w = 1, absorbing w = 2
        const double w = free_surf ? 1.0 : 2.0;
        dzp = Pn / (w * zp * zp);
        dzs = zs > 0 ? Pt / (w * zs * zs) : 0.0;
    }
    double o[3] = {0, 0, 0};
    fwi_chain_z(dzp, dzs, geo[G_LAM * nc + x], geo[G_MU * nc + x], 1.0 / (double)geo[G_IRHO * nc + x], zp, zs, o);
    double *d = eb + ((int64_t)q * nb + e) * 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] += o[k];
}

// g[m][x] += the facet parts of cell x, summed over its facets and the shots in order
__global__ __launch_bounds__(256) void k_fwi_facet_gather(const int32_t *__restrict__ c2f, const double *__restrict__ fb,
                                                          const double *__restrict__ eb, int64_t nc, int64_t nf,
                                                          int64_t nb, int nshots, double *__restrict__ g) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nc) return;
    double acc[3] = {0, 0, 0};
    for (int q = 0; q < nshots; ++q)
        for (int p = 0; p < 3; ++p) {
            const int32_t code = c2f[(int64_t)p * nc + x];
            const double *d = code >= 0 ? fb + (((int64_t)q * nf + (code >> 1)) * 2 + (code & 1)) * 3
                                        : eb + ((int64_t)q * nb + (-(int64_t)code - 1)) * 3;
            for (int m = 0; m < 3; ++m) acc[m] += d[m];
        }
    for (int m = 0; m < 3; ++m) g[m * nc + x] += acc[m];
}

}  // namespace dgt
