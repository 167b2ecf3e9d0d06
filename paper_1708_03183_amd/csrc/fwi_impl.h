// Full-waveform-inversion gradient of libdgtile (included at the end of solver.hip).
// The paper runs the forward chain only; this part extends the method to the
// gradient of a receiver misfit with respect to the per-cell material, and cites no
// passage of the paper.
//
// Forward: u_{n+1} = Phi(u_n) + s_n with u_n = (v^{n-1/2}, sigma^n), one step of the
// DG loop chain.  Receivers sample the velocity after every step, r_n = R u_{n+1};
// the misfit is J = 1/2 sum_n sum_r |r_n - d_n|^2.
//
// Adjoint: with the central flux and free-surface (or periodic) boundaries the
// semi-discrete operator is skew-adjoint in the discrete energy inner product, so
// Phi^T = T^-1 Phi(-dt) T with T = blockdiag(M_J^-1 P, M_J^-1 C) per cell (M_J the
// cell mass |J| M^, P = 1/rho, C the stiffness).  In the variables alpha = T a the
// adjoint recursion a_n = Phi^T a_{n+1} + R^T (r_{n-1} - d_{n-1}) is the forward
// chain run with -dt (on a second solver, tiled by the same inspector) plus the
// injection T R^T (r - d).  Per step the gradient needs the forward operator outputs
// (U = A sigma_n, X' = B U, Z = A X' of the velocity half, X1 = B v^{n+1/2}, Y = A X1,
// V2 = B Y of the stress half) and, at order 4, W = A B alpha_v, W' = B A alpha_s and
// their first halves; they come from single operator applications (untiled kernels).  With dA/drho_K =
// -(1/rho_K) E_K A and dB/dlam_K = C_lam C^-1 E_K B (E_K the restriction to cell K):
//   g_rho_K -= |J_K| sum [(dt av + c W) . M^ U + av . M^ (c Z) - c (A as) . M^ Y]
//   g_lam_K += |J_K| sum [(dt as + c W') . (M^ x S_lam) X1 + as . (M^ x S_lam) (c V2)
//                         - c (B av) . (M^ x S_lam) X']
// (and g_mu with S_mu), S_m = C^-1 C_m C^-1, c = dt^3/24 (0 at order 2), av the
// velocity part of alpha after the reversed step, as its stress part before it; the
// last terms of each line come from the material inside the other half's c A B A
// or c B A B.
// Forward states are recomputed from checkpoints by a binomial (revolve-style)
// reversal schedule.

#include "fwi_upwind.h"

namespace dgt {

// receiver r at step n of shot q: out[((q * nsteps + n) * nrec + r) * 2 + c]
template <int K, typename T>
__global__ __launch_bounds__(256) void k_fwi_sample(const T *__restrict__ v, int64_t nc, int64_t vsh, int nrec,
                                                    const int32_t *__restrict__ cell, const double *__restrict__ phi,
                                                    int64_t nsteps, int64_t n, const double *__restrict__ obs,
                                                    double *__restrict__ trace, double *__restrict__ res,
                                                    double *__restrict__ jacc) {
    constexpr int NP = np_of(K);
    __shared__ double red[256];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int t = threadIdx.x; t < 2 * nrec; t += blockDim.x) {
        const int k = t >> 1, c = t & 1;
        const int64_t x = cell[k];
        double r = 0.0;
        for (int i = 0; i < NP; ++i) r += phi[k * NP + i] * (double)v[q * vsh + (int64_t)(c * NP + i) * nc + x];
        const int64_t o = (((int64_t)q * nsteps + n) * nrec + k) * 2 + c;
        if (trace) trace[o] = r;
        if (obs) {
            const double d = r - obs[o];
            res[((int64_t)q * nrec + k) * 2 + c] = d;
            acc += d * d;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && jacc) jacc[q] += 0.5 * red[0];
}

// alpha_v += T R^T res: per receiver the weights (1/rho_K) M^-1 phi(x_r) / |J_K|.  One
// thread per (shot, component, node) runs over the receivers in order (receivers
// sharing a cell never race).
template <int K, typename T>
__global__ __launch_bounds__(256) void k_fwi_inject(T *__restrict__ av, int64_t nc, int64_t vsh, int nshots, int nrec,
                                                    const int32_t *__restrict__ cell, const double *__restrict__ mphi,
                                                    const T *__restrict__ geo, const double *__restrict__ res) {
    constexpr int NP = np_of(K);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nshots * 2 * NP) return;
    const int q = t / (2 * NP), c = (t / NP) % 2, i = t % NP;
    for (int k = 0; k < nrec; ++k) {
        const int64_t x = cell[k];
        const double w = mphi[k * NP + i] * (double)geo[G_IRHO * nc + x] / (double)geo[G_DET * nc + x];
        T &a = av[q * vsh + (int64_t)(c * NP + i) * nc + x];
        a = (T)((double)a + w * res[((int64_t)q * nrec + k) * 2 + c]);
    }
}

// v1 = v0 + (dt U + Z), the velocity update of the untiled chain
template <typename T>
__global__ __launch_bounds__(256) void k_fwi_vnext(T *__restrict__ v1, const T *__restrict__ v0,
                                                   const T *__restrict__ U, const T *__restrict__ Z, int64_t n, T dt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    v1[t] = v0[t] + (dt * U[t] + (Z ? Z[t] : T(0)));
}

// per-cell gradient terms of one step and one shot (blockIdx.y), in FP64, stored per
// shot in part[shot][3][nc]; k_fwi_grad_sum adds the shots in order (deterministic).
// 2-component fields (stride vsh per shot): av, U, Zs = c A B U, W = A B av,
// tV = A as, Y = A X1; 3-component (stride ssh): as, X1, V2s = c B A X1,
// Wp = B A as, tS = B av, Xp = B U.  The order-4 fields are null at order 2.
template <int K, typename T>
__global__ __launch_bounds__(256) void k_fwi_grad(int64_t nc, int nshots, const T *__restrict__ geo,
                                                  const T *__restrict__ av, const T *__restrict__ U,
                                                  const T *__restrict__ Zs, const T *__restrict__ W,
                                                  const T *__restrict__ tV, const T *__restrict__ Y, int64_t vsh,
                                                  const T *__restrict__ as, const T *__restrict__ X1,
                                                  const T *__restrict__ V2s, const T *__restrict__ Wp,
                                                  const T *__restrict__ tS, const T *__restrict__ Xp, int64_t ssh,
                                                  double dt, double c3, double *__restrict__ part) {
    constexpr int NP = np_of(K);
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nc) return;
    const int q = blockIdx.y;
    const auto &Rf = R<K, T>();
    const double lam = geo[G_LAM * nc + x], mu = geo[G_MU * nc + x], det = geo[G_DET * nc + x];
    // C^-1 on (xx, yy, xy): [[cA, cB, 0], [cB, cA, 0], [0, 0, 1/mu]]
    const double cA = (lam + 2 * mu) / (4 * mu * (lam + mu)), cB = -lam / (4 * mu * (lam + mu)), cC = 1.0 / mu;
    const bool o4 = W != nullptr;
    auto ld = [&](const T *f, int64_t o, int c, int i) { return (double)f[o + (int64_t)(c * NP + i) * nc]; };
    double gr = 0.0, gl = 0.0, gm = 0.0;
    {
        const int64_t ov = q * vsh + x, os = q * ssh + x;
        // left factors per node, read once: velocity (a = dt av + c W, av, -c A as) and
        // stress through C^-1 (dt as + c W', as, -c B av), the last two at order 4 only
        T la[2][NP], lb[2][NP], lc[2][NP], lp[3][NP], lg[3][NP], ls[3][NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                la[c][i] = (T)(dt * ld(av, ov, c, i) + (o4 ? c3 * ld(W, ov, c, i) : 0.0));
                lb[c][i] = o4 ? (T)ld(av, ov, c, i) : T(0);
                lc[c][i] = o4 ? (T)(-c3 * ld(tV, ov, c, i)) : T(0);
            }
            double p[3], h[3], t[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p[c] = dt * ld(as, os, c, i) + (o4 ? c3 * ld(Wp, os, c, i) : 0.0);
                h[c] = o4 ? ld(as, os, c, i) : 0.0;
                t[c] = o4 ? -c3 * ld(tS, os, c, i) : 0.0;
            }
            lp[0][i] = (T)(cA * p[0] + cB * p[1]); lp[1][i] = (T)(cB * p[0] + cA * p[1]); lp[2][i] = (T)(cC * p[2]);
            lg[0][i] = (T)(cA * h[0] + cB * h[1]); lg[1][i] = (T)(cB * h[0] + cA * h[1]); lg[2][i] = (T)(cC * h[2]);
            ls[0][i] = (T)(cA * t[0] + cB * t[1]); ls[1][i] = (T)(cB * t[0] + cA * t[1]); ls[2][i] = (T)(cC * t[2]);
        }
        // right factors streamed node by node: sum_i left_i M_ij right_j
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double mla[2] = {0, 0}, mlb[2] = {0, 0}, mlc[2] = {0, 0}, mlp[3] = {0, 0, 0}, mlg[3] = {0, 0, 0},
                   mls[3] = {0, 0, 0};
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const double M = (double)Rf.M[i * NP + j];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    mla[c] += M * (double)la[c][i];
                    if (o4) {
                        mlb[c] += M * (double)lb[c][i];
                        mlc[c] += M * (double)lc[c][i];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    mlp[c] += M * (double)lp[c][i];
                    if (o4) {
                        mlg[c] += M * (double)lg[c][i];
                        mls[c] += M * (double)ls[c][i];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                gr += mla[c] * ld(U, ov, c, j);
                if (o4) gr += mlb[c] * ld(Zs, ov, c, j) + mlc[c] * ld(Y, ov, c, j);
            }
            // strains E = C^-1 (field): lam term (b_xx + b_yy)(e_xx + e_yy), mu term
            // 2 (b_xx e_xx + b_yy e_yy) + b_xy e_xy
            auto strain = [&](const T *f, double (&e)[3]) {
                const double f0 = ld(f, os, 0, j), f1 = ld(f, os, 1, j), f2 = ld(f, os, 2, j);
                e[0] = cA * f0 + cB * f1;
                e[1] = cB * f0 + cA * f1;
                e[2] = cC * f2;
            };
            auto acc = [&](const double (&b)[3], const double (&e)[3]) {
                gl += (b[0] + b[1]) * (e[0] + e[1]);
                gm += 2 * (b[0] * e[0] + b[1] * e[1]) + b[2] * e[2];
            };
            double e[3];
            strain(X1, e);
            acc(mlp, e);
            if (o4) {
                strain(V2s, e);
                acc(mlg, e);
                strain(Xp, e);
                acc(mls, e);
            }
        }
    }
    double *o = part + (int64_t)q * 3 * nc;
    o[x] = det * gl;
    o[nc + x] = det * gm;
    o[2 * nc + x] = -det * gr;
}

__global__ __launch_bounds__(256) void k_fwi_grad_sum(int64_t nc, int nshots, const double *__restrict__ part,
                                                      double *__restrict__ g) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nc) return;
    double a = 0.0;
    for (int q = 0; q < nshots; ++q) a += part[(int64_t)q * 3 * nc + t];
    g[t] += a;
}

struct FwiReceivers {
    int nrec = 0;
    DBuf<int32_t> cell;  // exec id of each receiver's cell
    DBuf<double> phi;    // [nrec][Np] basis at the receiver
    DBuf<double> mphi;   // [nrec][Np] reference inverse mass times phi
};

static void fwi_receivers(dgt_solver *s, int nrec, const double *xy, FwiReceivers &R) {
    const int np = s->E.np;
    std::vector<int32_t> cell(nrec);
    std::vector<double> phi((size_t)nrec * np), mphi((size_t)nrec * np);
    for (int k = 0; k < nrec; ++k) {
        DGT_REQUIRE(std::isfinite(xy[2 * k]) && std::isfinite(xy[2 * k + 1]), DGT_EINVAL,
                    "receiver position is not finite");
        double rs = 0, ss = 0;
        const int64_t c = locate_point(s, xy[2 * k], xy[2 * k + 1], rs, ss);
        DGT_REQUIRE(c >= 0, DGT_EINVAL, "receiver outside the mesh");
        cell[k] = s->rank_h[c];
        s->E.phi(rs, ss, &phi[(size_t)k * np]);
        for (int i = 0; i < np; ++i) {
            double a = 0;
            for (int j = 0; j < np; ++j) a += s->E.Minv[i * np + j] * phi[(size_t)k * np + j];
            mphi[(size_t)k * np + i] = a;
        }
    }
    R.nrec = nrec;
    R.cell.upload(cell, s->st);
    R.phi.upload(phi, s->st);
    R.mphi.upload(mphi, s->st);
}

static void fwi_check(dgt_solver *s, const dgt_fwi_params *p) {
    DGT_REQUIRE(p->nrec >= 1 && p->rec_xy, DGT_EINVAL, "at least one receiver");
    DGT_REQUIRE(p->nsteps >= 1, DGT_EINVAL, "nsteps must be >= 1");
    DGT_REQUIRE(p->mode == 0 || p->mode == 1, DGT_EINVAL, "mode must be 0 or 1");
    DGT_REQUIRE(p->mode == 0 || (s->plan_status == DGT_OK && s->inspected), DGT_ESTATE,
                "tiled mode needs a successful dgt_solver_inspect");
    DGT_REQUIRE(p->mode == 0 || s->last_region.empty(), DGT_EUNSUPPORTED,
                "full-waveform inversion runs on a whole mesh, not on a region-aware part");
    DGT_REQUIRE(p->mode == 0 || s->fuse == 1, DGT_EUNSUPPORTED,
                "full-waveform inversion samples receivers after every step: no chain fused over steps");
}

template <int K, typename T>
static void fwi_advance(dgt_solver *s, int64_t n0, int64_t nsteps, int mode) {
    if (nsteps <= 0) return;
    int64_t launches = 0;
    // one call per step, so that every replay computes the source times alike
    for (int64_t n = n0; n < n0 + nsteps; ++n) {
        if (mode == 0) step_untiled<K, T>(s, 1, (double)n * s->p.dt, launches);
        else step_tiled<K, T>(s, 1, (double)n * s->p.dt, launches);
    }
}

// number of steps a binomial reversal reverses with `snaps` free checkpoints and
// `sweeps` forward sweeps: C(snaps + sweeps, snaps), capped
static int64_t binom_steps(int snaps, int sweeps, int64_t cap) {
    double b = 1.0;
    for (int i = 1; i <= snaps; ++i) {
        b = b * (double)(sweeps + i) / (double)i;
        if (b > (double)cap) return cap + 1;
    }
    return (int64_t)(b + 0.5);
}

template <int K, typename T>
struct FwiRun {
    dgt_solver *f = nullptr, *a = nullptr;  // forward (dt) and reversed (-dt) solvers
    const dgt_fwi_params *p = nullptr;
    const FwiReceivers *R = nullptr;
    const double *obs = nullptr;
    int S = 1;
    bool rec = false;  // intermediates from recorded tiled steps
    int64_t vsh = 0, ssh = 0, advanced = 0, reversed = 0;
    std::vector<DBuf<char>> snap;
    DBuf<T> U, Xp, Zs, V1, X1, Y, V2s, W, Wp, tV, tS, As;
    DBuf<double> res, g, part;
    // upwind flux or absorbing sides: the closed-form transposed step (fwi_upwind.h)
    bool upw = false;
    FacetMass m1{};
    DBuf<T> fU1, fX1, fZ1, fPV, fV1, fX2, fU2, fZ2, fPS;  // forward intermediates of a step
    DBuf<T> aA, aBA, aABA, aPS, aMu, aB, aAB, aBAB, aPV;  // adjoint-side vectors
    DBuf<double> fb, eb;                                  // facet parts per facet, side and shot

    void alloc_upwind() {
        const size_t nv = (size_t)vsh * S, ns = (size_t)ssh * S;
        for (auto *b : {&fU1, &fZ1, &fPV, &fV1, &fU2, &aA, &aABA, &aMu, &aAB, &aPV}) b->alloc(nv);
        for (auto *b : {&fX1, &fX2, &fZ2, &fPS, &aBA, &aPS, &aB, &aBAB}) b->alloc(ns);
        fb.alloc((size_t)S * std::max<int64_t>(f->nf, 1) * 6);
        eb.alloc((size_t)S * std::max<int64_t>(f->nb, 1) * 3);
        DGT_HIP(hipMemsetAsync(fb.p, 0, fb.n * sizeof(double), f->st));
        DGT_HIP(hipMemsetAsync(eb.p, 0, eb.n * sizeof(double), f->st));
        const int nfp = K + 1;
        for (int i = 0; i < nfp * nfp; ++i) m1.m[i] = f->E.M1[i];
    }
    // cell and interior-facet parts of the queued pairs, one launch each
    FwiCellPairs<T> cq{};
    FwiPairs<T> fq{};
    void flush_pairs() {
        if (cq.n)
            k_fwi_cell_pairs<K, T><<<dim3(blocks_for(f->nc, 256), S), 256, 0, f->st>>>(cq, (const T *)f->geo.p,
                                                                                      f->nc, part.p);
        if (fq.n)
            k_fwi_facet_pairs<K, T><<<dim3(blocks_for(f->nf, 256), S), 256, 0, f->st>>>(
                fq, f->ef2c.p, f->ef2l.p, (const T *)f->geo.p, f->nc, f->nf, m1, fb.p);
        cq.n = fq.n = 0;
    }
    // one term coef * a^T W dOp b (ob = Op b): cell part, and the facet part when the
    // flux weights of Op depend on the impedances
    template <int KIND>
    void pair(const T *a_, const T *b_, const T *ob, double coef) {
        hipStream_t st = f->st;
        const int64_t nc = f->nc, nf = f->nf, nb = f->nb;
        constexpr bool VEL = KIND == FK_A || KIND == FK_DV;  // kind of a and ob
        const int64_t sh = VEL ? vsh : ssh;
        const T *geo = (const T *)f->geo.p;
        // the cell and interior-facet parts are queued and summed in one pass each by
        // flush_pairs
        if (fq.n == FWI_MAX_PAIRS || cq.n == FWI_MAX_PAIRS) flush_pairs();
        const int k = cq.n++;
        cq.kind[k] = KIND;
        cq.a[k] = a_;
        cq.ob[k] = ob;
        cq.sh[k] = sh;
        cq.coef[k] = coef;
        // interior facets weigh by the impedances with the upwind flux only; exterior ones
        // only in the penalties (absorbing facets always, free surfaces with the upwind flux)
        if (f->upw && nf) {
            const int i = fq.n++;
            fq.kind[i] = KIND;
            fq.a[i] = a_;
            fq.b[i] = b_;
            fq.ash[i] = sh;
            fq.bsh[i] = (KIND == FK_A || KIND == FK_DS) ? ssh : vsh;
            fq.coef[i] = coef;
        }
        if ((KIND == FK_DV || KIND == FK_DS) && f->haspen && nb)
            k_fwi_ext_pair<K, T, KIND><<<dim3(blocks_for(nb, 256), S), 256, 0, st>>>(
                a_, b_, sh, f->eb2c.p, f->eb2l.p, geo, nc, nb, m1, coef, f->upw ? 1 : 0, eb.p);
    }
    // The reversal of step n with the upwind flux or absorbing sides: the forward state u_n
    // is in f, alpha_{n+1} in a.  Forward: U1 = A s, X1 = B U1, Z1 = A X1, PV = Dv v,
    // v' = v + dt U1 + c Z1 + dt PV, X2 = B v', U2 = A X2, Z2 = B U2, PS = Ds s.  Adjoint:
    // mu = alpha_v - dt A alpha_s - c A B A alpha_s (the velocity part after the first
    // transposed half).  Terms of the gradient, each coef * a^T W dOp b:
    //   (alpha_s, v') B dt, (alpha_s, U2) B c, (A alpha_s, X2) A -c, (B A alpha_s, v') B c,
    //   (alpha_s, s) Ds dt, (mu, s) A dt, (mu, X1) A c, (B mu, U1) B -c, (A B mu, s) A c,
    //   (mu, v) Dv dt
    // (from d(S2 S1) = dS2 S1 + S2 dS1 and W_v A = -(W_s B)^T).
    void step_back_upw(int64_t n) {
        hipStream_t st = f->st;
        const bool o4 = f->p.time_order == 4;
        const double dt = f->p.dt, c3 = o4 ? dt * dt * dt / 24.0 : 0.0;
        int64_t launches = 0;
        const int64_t nvS = vsh * S, nsS = ssh * S;
        const T *v0 = (const T *)f->fld[F_V].p, *s0 = (const T *)f->fld[F_S].p;
        T *av = (T *)a->fld[F_V].p, *as = (T *)a->fld[F_S].p;
        auto vop = [&](const T *in, T *out) { apply_op_cell<K, T>(f, true, in, out, 1.0, nullptr, 0.0, launches, S, ssh, vsh); };
        auto sop = [&](const T *in, T *out) { apply_op_cell<K, T>(f, false, in, out, 1.0, nullptr, 0.0, launches, S, vsh, ssh); };
        // penalties alone: the operator part scaled by zero (its input only needs finite values)
        auto vpen = [&](const T *pv, T *out) { apply_op_cell<K, T>(f, true, s0, out, 0.0, pv, 1.0, launches, S, ssh, vsh, vsh); };
        auto spen = [&](const T *ps, T *out) { apply_op_cell<K, T>(f, false, v0, out, 0.0, ps, 1.0, launches, S, vsh, ssh, ssh); };
        auto lin = [&](T *out, int64_t cnt, const T *x0, double c0, const T *x1, double c1, const T *x2, double c2,
                       const T *x3, double c3_) {
            k_fwi_lin<T><<<blocks_for(cnt, 256), 256, 0, st>>>(out, x0, c0, x1, c1, x2, c2, x3, c3_, cnt);
        };
        sample(n);
        const bool pen = f->haspen;
        // forward intermediates
        vop(s0, fU1.p);
        if (o4) {
            sop(fU1.p, fX1.p);
            vop(fX1.p, fZ1.p);
        }
        if (pen) vpen(v0, fPV.p);
        lin(fV1.p, nvS, v0, 1.0, fU1.p, dt, o4 ? fZ1.p : nullptr, c3, pen ? fPV.p : nullptr, dt);
        sop(fV1.p, fX2.p);
        if (o4) {
            vop(fX2.p, fU2.p);
            sop(fU2.p, fZ2.p);
        }
        if (pen) spen(s0, fPS.p);
        // adjoint-side vectors
        vop(as, aA.p);
        if (o4) {
            sop(aA.p, aBA.p);
            vop(aBA.p, aABA.p);
        }
        if (pen) spen(as, aPS.p);
        lin(aMu.p, nvS, av, 1.0, aA.p, -dt, o4 ? aABA.p : nullptr, -c3, nullptr, 0.0);
        sop(aMu.p, aB.p);
        if (o4) {
            vop(aB.p, aAB.p);
            sop(aAB.p, aBAB.p);
        }
        if (pen) vpen(aMu.p, aPV.p);
        // gradient terms of this step
        DGT_HIP(hipMemsetAsync(part.p, 0, part.n * sizeof(double), st));
        pair<FK_B>(as, fV1.p, fX2.p, dt);
        pair<FK_A>(aMu.p, s0, fU1.p, dt);
        if (o4) {
            pair<FK_B>(as, fU2.p, fZ2.p, c3);
            pair<FK_A>(aA.p, fX2.p, fU2.p, -c3);
            pair<FK_B>(aBA.p, fV1.p, fX2.p, c3);
            pair<FK_A>(aMu.p, fX1.p, fZ1.p, c3);
            pair<FK_B>(aB.p, fU1.p, fX1.p, -c3);
            pair<FK_A>(aAB.p, s0, fU1.p, c3);
        }
        if (pen) {
            pair<FK_DS>(as, s0, fPS.p, dt);
            pair<FK_DV>(aMu.p, v0, fPV.p, dt);
        }
        flush_pairs();
        k_fwi_grad_sum<<<blocks_for(3 * f->nc, 256), 256, 0, st>>>(f->nc, S, part.p, g.p);
        // the transposed step: alpha_s += dt Ds alpha_s - dt B mu - c B A B mu; alpha_v = mu + dt Dv mu
        lin(as, nsS, as, 1.0, pen ? aPS.p : nullptr, dt, aB.p, -dt, o4 ? aBAB.p : nullptr, -c3);
        lin(av, nvS, aMu.p, 1.0, pen ? aPV.p : nullptr, dt, nullptr, 0.0, nullptr, 0.0);
        ++reversed;
        add_residual(n);
    }

    void store(int slot) {
        const size_t bv = (size_t)vsh * S * sizeof(T), bs = (size_t)ssh * S * sizeof(T);
        if (snap[slot].n < bv + bs) snap[slot].alloc(bv + bs);
        DGT_HIP(hipMemcpyAsync(snap[slot].p, f->fld[F_V].p, bv, hipMemcpyDeviceToDevice, f->st));
        DGT_HIP(hipMemcpyAsync(snap[slot].p + bv, f->fld[F_S].p, bs, hipMemcpyDeviceToDevice, f->st));
    }
    void restore(int slot) {
        const size_t bv = (size_t)vsh * S * sizeof(T), bs = (size_t)ssh * S * sizeof(T);
        DGT_HIP(hipMemcpyAsync(f->fld[F_V].p, snap[slot].p, bv, hipMemcpyDeviceToDevice, f->st));
        DGT_HIP(hipMemcpyAsync(f->fld[F_S].p, snap[slot].p + bv, bs, hipMemcpyDeviceToDevice, f->st));
    }
    void advance(int64_t n0, int64_t n) {
        fwi_advance<K, T>(f, n0, n, p->mode);
        advanced += n;
    }
    // residual of the receivers at the forward state held (the observation after
    // step n - 1), then its injection into the adjoint velocity
    void sample(int64_t n) {
        if (n < 1) return;
        k_fwi_sample<K, T><<<S, 256, 0, f->st>>>((const T *)f->fld[F_V].p, f->nc, vsh, R->nrec, R->cell.p, R->phi.p,
                                               p->nsteps, n - 1, obs, nullptr, res.p, nullptr);
    }
    void add_residual(int64_t n) {
        if (n < 1) return;
        constexpr int NP = np_of(K);
        k_fwi_inject<K, T><<<blocks_for((int64_t)S * 2 * NP, 256), 256, 0, f->st>>>(
            (T *)a->fld[F_V].p, f->nc, vsh, S, R->nrec, R->cell.p, R->mphi.p, (const T *)f->geo.p, res.p);
    }
    void inject(int64_t n) {
        sample(n);
        add_residual(n);
    }
    // copy a field of every shot (ncomp components) into a buffer of shot stride dsh
    void copy_field(T *dst, int64_t dsh, const dgt_solver *s, int fld, int ncomp) {
        const int64_t w = (int64_t)ncomp * np_of(K) * s->nc;
        DGT_HIP(hipMemcpy2DAsync(dst, dsh * sizeof(T), s->fld[fld].p, s->fshot(fld) * sizeof(T), w * sizeof(T), S,
                                 hipMemcpyDeviceToDevice, s->st));
    }
    // Both half steps keep U, X, Z when the chain is split at the end of the velocity
    // half (loop 13 of the order-4 chain) and runs tiled: one forward step and one
    // reversed step then give every intermediate of the gradient, instead of ten
    // untiled operator applications.
    bool recordable() const {
        if (p->mode != 1 || f->p.time_order != 4) return false;
        for (const dgt_solver *s : {f, a}) {
            bool half = false;
            for (const auto &P : s->plan) half |= P.first + P.n == 13;
            if (!half) return false;
        }
        return true;
    }
    // one tiled step of solver s from time t0; after the velocity half its fields U, X, Z
    // go to vel[0], vel[1], vel[2], after the stress half to str[0..2] (null: not kept)
    void record_step(dgt_solver *s, double t0, T *const (&vel)[3], T *const (&str)[3]) {
        int64_t launches = 0;
        const std::function<void(size_t)> after = [&](size_t b) {
            const auto &P = s->plan[b];
            const int end = P.first + P.n;
            if (end != 13 && end != 26) return;
            T *const(&d)[3] = end == 13 ? vel : str;
            // velocity half: U = A s, X = B U, Z = c A X (2 components); stress half:
            // X = B v, U = A X, Z = c B U (3 components)
            if (d[0]) copy_field(d[0], vsh, s, F_U, 2);
            if (d[1]) copy_field(d[1], ssh, s, F_X, 3);
            if (d[2]) copy_field(d[2], end == 13 ? vsh : ssh, s, F_Z, end == 13 ? 2 : 3);
        };
        step_tiled<K, T>(s, 1, t0, launches, (1 << F_U) | (1 << F_X) | (1 << F_Z), &after);
    }
    // the forward state u_n is in f, alpha_{n+1} in a
    void step_back(int64_t n) {
        if (upw) return step_back_upw(n);
        hipStream_t st = f->st;
        const int64_t nc = f->nc;
        const bool o4 = f->p.time_order == 4;
        const double dt = f->p.dt, c3 = o4 ? dt * dt * dt / 24.0 : 0.0;
        int64_t launches = 0;
        if (rec) {
            sample(n);  // from u_n, before the recorded step advances the forward state
            // forward step: velocity half U = A s_n, X = B U, Z = c A X; stress half X = B v',
            // U = A X, Z = c B U  (record_step's slots: U, X, Z fields)
            record_step(f, (double)n * dt, {U.p, Xp.p, Zs.p}, {Y.p, X1.p, V2s.p});
            DGT_HIP(hipMemcpyAsync(As.p, a->fld[F_S].p, (size_t)ssh * S * sizeof(T), hipMemcpyDeviceToDevice, st));
            // reversed step: velocity half U = A as, X = B A as; stress half X = B av,
            // U = A B av
            record_step(a, 0.0, {tV.p, Wp.p, nullptr}, {W.p, tS.p, nullptr});
            ++reversed;
            k_fwi_grad<K, T><<<dim3(blocks_for(nc, 256), S), 256, 0, st>>>(
                nc, S, (const T *)f->geo.p, (const T *)a->fld[F_V].p, U.p, Zs.p, W.p, tV.p, Y.p, vsh, As.p, X1.p,
                V2s.p, Wp.p, tS.p, Xp.p, ssh, dt, c3, part.p);
            k_fwi_grad_sum<<<blocks_for(3 * nc, 256), 256, 0, st>>>(nc, S, part.p, g.p);
            add_residual(n);
            return;
        }
        const T *v0 = (const T *)f->fld[F_V].p, *s0 = (const T *)f->fld[F_S].p;
        // every operator application covers all shots in one launch per kernel
        auto vop = [&](const T *in, T *out, double sc) { apply_op_cell<K, T>(f, true, in, out, sc, nullptr, 0.0, launches, S, ssh, vsh); };
        auto sop = [&](const T *in, T *out, double sc) { apply_op_cell<K, T>(f, false, in, out, sc, nullptr, 0.0, launches, S, vsh, ssh); };
        vop(s0, U.p, 1.0);
        if (o4) {
            sop(U.p, Xp.p, 1.0);
            vop(Xp.p, Zs.p, c3);
        }
        k_fwi_vnext<T><<<blocks_for(vsh * S, 256), 256, 0, st>>>(V1.p, v0, U.p, o4 ? Zs.p : nullptr, vsh * S, (T)dt);
        sop(V1.p, X1.p, 1.0);
        if (o4) {
            vop(X1.p, Y.p, 1.0);
            sop(Y.p, V2s.p, c3);
        }
        // alpha_s before the reversed step, then the step itself
        DGT_HIP(hipMemcpyAsync(As.p, a->fld[F_S].p, (size_t)ssh * S * sizeof(T), hipMemcpyDeviceToDevice, st));
        fwi_advance<K, T>(a, 0, 1, p->mode);
        ++reversed;
        const T *av = (const T *)a->fld[F_V].p;
        if (o4) {
            sop(av, tS.p, 1.0);
            vop(tS.p, W.p, 1.0);
            vop(As.p, tV.p, 1.0);
            sop(tV.p, Wp.p, 1.0);
        }
        k_fwi_grad<K, T><<<dim3(blocks_for(nc, 256), S), 256, 0, st>>>(
            nc, S, (const T *)f->geo.p, av, U.p, o4 ? Zs.p : nullptr, o4 ? W.p : nullptr, o4 ? tV.p : nullptr,
            o4 ? Y.p : nullptr, vsh, As.p, X1.p, o4 ? V2s.p : nullptr, o4 ? Wp.p : nullptr, o4 ? tS.p : nullptr,
            o4 ? Xp.p : nullptr, ssh, dt, c3, part.p);
        k_fwi_grad_sum<<<blocks_for(3 * nc, 256), 256, 0, st>>>(nc, S, part.p, g.p);
        inject(n);
    }
    // reverse steps [l, r): u_l is in checkpoint `slot`, `free` checkpoints above it
    void reverse(int64_t l, int64_t r, int slot, int free) {
        if (r - l == 1) {
            restore(slot);
            step_back(l);
            return;
        }
        if (free == 0) {
            for (int64_t j = r - 1; j >= l; --j) {
                restore(slot);
                advance(l, j - l);
                step_back(j);
            }
            return;
        }
        const int64_t n = r - l;
        int t = 1;
        while (binom_steps(free, t, n) < n) ++t;
        int64_t right = binom_steps(free - 1, t, n);
        right = std::max<int64_t>(1, std::min<int64_t>(right, n - 1));
        const int64_t m = r - right;
        restore(slot);
        advance(l, m - l);
        store(slot + 1);
        reverse(m, r, slot + 1, free - 1);
        reverse(l, m, slot, free);
    }
};

// a second solver on the same mesh and material running the chain with -dt, the
// same shots (no sources) and the same inspection and schedule
static std::unique_ptr<dgt_solver> fwi_adjoint_solver(dgt_solver *s, const dgt_mesh *mh) {
    const int64_t nc = s->nc;
    std::vector<double> lam(nc), mu(nc), rho(nc);
    DGT_HIP(hipMemcpyAsync(lam.data(), s->lam.p, 8 * nc, hipMemcpyDeviceToHost, s->st));
    DGT_HIP(hipMemcpyAsync(mu.data(), s->mu.p, 8 * nc, hipMemcpyDeviceToHost, s->st));
    DGT_HIP(hipMemcpyAsync(rho.data(), s->rho.p, 8 * nc, hipMemcpyDeviceToHost, s->st));
    DGT_HIP(hipStreamSynchronize(s->st));
    dgt_solver_params q = s->p;
    q.dt = -s->p.dt;
    auto a = new_solver(mh, lam.data(), mu.data(), rho.data(), &q, (void *)s->st);
    if (s->nshots > 1) {
        a->nshots = s->nshots;
        alloc_fields(a.get());
        a->src_in.assign(s->nshots, -1);
        a->src_vec.alloc((size_t)s->nshots * s->E.np * s->esz);
        DGT_HIP(hipMemsetAsync(a->src_vec.p, 0, a->src_vec.n, s->st));
        set_source_exec(a.get());
    }
    if (s->inspected) {
        dgt_inspect_params ip = s->last_ip;
        ip.splits = s->last_splits.data();
        ip.nsplits = (int32_t)s->last_splits.size();
        ip.sub_tile_sizes = s->last_sub_ts.empty() ? nullptr : s->last_sub_ts.data();
        solver_inspect_once(a.get(), &ip, s->last_cap);
        DGT_REQUIRE(a->plan_status == DGT_OK && a->rank_h == s->rank_h, DGT_ESTATE,
                    "the reversed chain's inspection differs from the forward one");
        a->sched_mode = s->sched_mode;
    } else {
        DGT_REQUIRE(a->rank_h == s->rank_h, DGT_ESTATE, "cell orders differ");
    }
    return a;
}

template <int K, typename T>
static void fwi_forward_run(dgt_solver *s, const dgt_fwi_params *p, const FwiReceivers &R, const double *obs,
                            double *trace, double *jacc) {
    const int64_t vsh = s->fshot(F_V);
    for (int f = 0; f < F_COUNT; ++f) DGT_HIP(hipMemsetAsync(s->fld[f].p, 0, s->fld[f].n, s->st));
    DBuf<double> res((size_t)s->nshots * R.nrec * 2);
    for (int64_t n = 0; n < p->nsteps; ++n) {
        fwi_advance<K, T>(s, n, 1, p->mode);
        k_fwi_sample<K, T><<<s->nshots, 256, 0, s->st>>>((const T *)s->fld[F_V].p, s->nc, vsh, R.nrec, R.cell.p,
                                                       R.phi.p, p->nsteps, n, obs, trace, res.p, jacc);
    }
}

}  // namespace dgt

extern "C" {

dgt_status dgt_fwi_forward(dgt_solver *s, const dgt_fwi_params *p, double *traces) {
    return guard([&] {
        DGT_REQUIRE(s && p && traces, DGT_EINVAL, "NULL argument");
        fwi_check(s, p);
        FwiReceivers R;
        fwi_receivers(s, p->nrec, p->rec_xy, R);
        if (p->mode == 1) prepare_tiled(s);
        dispatch(s, [&]<int K, typename T>() { fwi_forward_run<K, T>(s, p, R, nullptr, traces, nullptr); });
        DGT_HIP(hipGetLastError());
        DGT_HIP(hipStreamSynchronize(s->st));
        if (p->mode == 1) check_graphs(s);
        s->state_valid = true;  // the state after the run
    });
}

dgt_status dgt_fwi_gradient(dgt_solver *s, const dgt_fwi_params *p, const double *observed, double *misfit,
                            double *g_lam, double *g_mu, double *g_rho) {
    return guard([&] {
        DGT_REQUIRE(s && p && observed && misfit && g_lam && g_mu && g_rho, DGT_EINVAL, "NULL argument");
        fwi_check(s, p);
        DGT_REQUIRE(p->nsnap >= 1, DGT_EINVAL, "nsnap must be >= 1");
        // the reversed chain is the transposed step for the central flux with free or
        // periodic boundaries; otherwise the closed-form transposed step of fwi_upwind.h
        bool any_absorbing = false;
        {
            const auto bf = s->bfree.download(s->st, std::max<int64_t>(s->nb, 1));
            for (int64_t b = 0; b < s->nb; ++b) any_absorbing |= bf[b] == 0;
        }
        const bool upw_path = s->upw || s->haspen || any_absorbing || std::getenv("DGT_FWI_CLOSED_FORM");
        FwiReceivers R;
        fwi_receivers(s, p->nrec, p->rec_xy, R);
        auto adj = fwi_adjoint_solver(s, s->mesh_handle);
        hipStream_t st = s->st;
        const int S = s->nshots;
        const int64_t nc = s->nc;
        DBuf<double> jacc(S);
        DGT_HIP(hipMemsetAsync(jacc.p, 0, 8 * S, st));
        if (p->mode == 1) {
            prepare_tiled(s);
            prepare_tiled(adj.get());
        }
        double J = 0;
        dispatch(s, [&]<int K, typename T>() {
            FwiRun<K, T> run;
            run.f = s;
            run.a = adj.get();
            run.p = p;
            run.R = &R;
            run.obs = observed;
            run.S = S;
            run.vsh = s->fshot(F_V);
            run.ssh = s->fshot(F_S);
            const size_t nv = (size_t)run.vsh * S, ns = (size_t)run.ssh * S;
            for (auto *b : {&run.U, &run.Zs, &run.V1, &run.Y, &run.W, &run.tV}) b->alloc(nv);
            for (auto *b : {&run.Xp, &run.X1, &run.V2s, &run.Wp, &run.tS, &run.As}) b->alloc(ns);
            run.res.alloc((size_t)S * R.nrec * 2);
            run.g.alloc((size_t)3 * nc);
            run.part.alloc((size_t)3 * nc * S);
            DGT_HIP(hipMemsetAsync(run.g.p, 0, 8 * 3 * nc, st));
            run.snap.resize(p->nsnap);
            run.upw = upw_path;
            if (run.upw) run.alloc_upwind();
            run.rec = !run.upw && run.recordable() && !std::getenv("DGT_FWI_UNTILED_INTERMEDIATES");
            // forward sweep from rest: misfit; the start state is the first checkpoint
            for (int f = 0; f < F_COUNT; ++f) DGT_HIP(hipMemsetAsync(s->fld[f].p, 0, s->fld[f].n, st));
            run.store(0);
            fwi_forward_run<K, T>(s, p, R, observed, nullptr, jacc.p);
            run.advanced += p->nsteps;
            // adjoint start: alpha_N = T R^T (r_{N-1} - d_{N-1}), from the final state
            for (int f = 0; f < F_COUNT; ++f) DGT_HIP(hipMemsetAsync(adj->fld[f].p, 0, adj->fld[f].n, st));
            run.inject(p->nsteps);
            run.reverse(0, p->nsteps, 0, p->nsnap - 1);
            if (run.upw)
                k_fwi_facet_gather<<<blocks_for(nc, 256), 256, 0, st>>>(s->c2f.p, run.fb.p, run.eb.p, nc, s->nf, s->nb,
                                                                       S, run.g.p);
            // gradient into the mesh numbering
            for (int m = 0; m < 3; ++m)
                k_permute_rows<double><<<blocks_for(nc, 256), 256, 0, st>>>(
                    run.g.p + m * nc, m == 0 ? g_lam : (m == 1 ? g_mu : g_rho), s->rank.p, 1, nc, 0);
            s->last_launches = run.advanced + run.reversed;
        });
        DGT_HIP(hipGetLastError());
        const auto jh = jacc.download(st);
        for (int q = 0; q < S; ++q) J += jh[q];
        if (p->mode == 1) {
            check_graphs(s);
            check_graphs(adj.get());
        }
        *misfit = J;
        s->state_valid = false;  // the fields hold the reversal's last forward state
    });
}

}  // extern "C"
