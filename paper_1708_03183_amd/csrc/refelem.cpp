// Nodal P_k reference triangle of libdgtile (host, set-up only).
//
// The paper's DG discretisation (Sec. 7.1) is not printed; the element used is
// Lagrange P_k, k = 1..4, on the equispaced nodes (i/k, j/k), i+j <= k, of the
// triangle {(0,0),(1,0),(0,1)}, nodes ordered by j then i.  Each basis
// function is built symbolically with Silvester's product formula in
// barycentric coordinates, so derivatives are exact polynomial derivatives and
// integrals use the exact monomial moments int r^a s^b = a! b! / (a+b+2)!.
// The expanded P4 coefficients alternate in sign and the equispaced P4 mass
// matrix is ill-conditioned (about 1e5), so every step runs in IEEE binary128
// (113-bit significand) and each table is rounded to double once: the tables
// are then the exactly rounded values of the exact rationals.
#include "refelem.h"

#include <cmath>
#include <stdexcept>

namespace dgt {

namespace {

using xf = __float128;

xf xabs(xf v) { return v < 0 ? -v : v; }
constexpr int D = 9;  // degree bound + 1 for products of two P4 polynomials

struct Poly {  // sum c[a][b] r^a s^b
    xf c[D][D] = {};
    static Poly constant(xf v) {
        Poly p;
        p.c[0][0] = v;
        return p;
    }
    Poly operator*(const Poly &o) const {
        Poly r;
        for (int a = 0; a < D; ++a)
            for (int b = 0; a + b < D; ++b) {
                if (c[a][b] == 0) continue;
                for (int a2 = 0; a + a2 < D; ++a2)
                    for (int b2 = 0; a + a2 + b + b2 < D; ++b2) r.c[a + a2][b + b2] += c[a][b] * o.c[a2][b2];
            }
        return r;
    }
    Poly dr() const {
        Poly r;
        for (int a = 1; a < D; ++a)
            for (int b = 0; a + b < D; ++b) r.c[a - 1][b] = a * c[a][b];
        return r;
    }
    Poly ds() const {
        Poly r;
        for (int a = 0; a < D; ++a)
            for (int b = 1; a + b < D; ++b) r.c[a][b - 1] = b * c[a][b];
        return r;
    }
    xf eval(xf r, xf s) const {
        xf v = 0, rp = 1;
        for (int a = 0; a < D; ++a, rp *= r) {
            xf sp = 1;
            for (int b = 0; a + b < D; ++b, sp *= s) v += c[a][b] * rp * sp;
        }
        return v;
    }
};

xf fact(int n) {
    xf f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// exact integral over the reference triangle
xf integrate(const Poly &p) {
    xf v = 0;
    for (int a = 0; a < D; ++a)
        for (int b = 0; a + b < D; ++b)
            if (p.c[a][b] != 0) v += p.c[a][b] * fact(a) * fact(b) / fact(a + b + 2);
    return v;
}

// linear factor (k*lambda - m) / (n - m) with lambda = c0 + cr r + cs s
Poly factor(int k, xf c0, xf cr, xf cs, int m, int n) {
    Poly p;
    const xf den = (xf)(n - m);
    p.c[0][0] = (k * c0 - m) / den;
    p.c[1][0] = k * cr / den;
    p.c[0][1] = k * cs / den;
    return p;
}

// Silvester: phi for barycentric multi-index (i0 on lambda0=1-r-s, i1 on r, i2 on s)
Poly silvester(int k, int i1, int i2) {
    const int i0 = k - i1 - i2;
    Poly p = Poly::constant(1);
    for (int m = 0; m < i1; ++m) p = p * factor(k, 0, 1, 0, m, i1);
    for (int m = 0; m < i2; ++m) p = p * factor(k, 0, 0, 1, m, i2);
    for (int m = 0; m < i0; ++m) p = p * factor(k, 1, -1, -1, m, i0);
    return p;
}

// LU factorisation with partial pivoting, then inverse by column solves
std::vector<xf> lu_inverse(const std::vector<xf> &A, int n) {
    std::vector<xf> lu(A);
    std::vector<int> piv(n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (xabs(lu[r * n + c]) > xabs(lu[p * n + c])) p = r;
        if (lu[p * n + c] == 0) throw std::runtime_error("singular reference matrix");
        piv[c] = p;
        if (p != c)
            for (int j = 0; j < n; ++j) std::swap(lu[c * n + j], lu[p * n + j]);
        for (int r = c + 1; r < n; ++r) {
            lu[r * n + c] /= lu[c * n + c];
            for (int j = c + 1; j < n; ++j) lu[r * n + j] -= lu[r * n + c] * lu[c * n + j];
        }
    }
    std::vector<xf> inv(n * n, 0);
    for (int col = 0; col < n; ++col) {
        std::vector<xf> x(n, 0);
        x[col] = 1;
        for (int c = 0; c < n; ++c) std::swap(x[c], x[piv[c]]);
        for (int r = 0; r < n; ++r)
            for (int j = 0; j < r; ++j) x[r] -= lu[r * n + j] * x[j];
        for (int r = n - 1; r >= 0; --r) {
            for (int j = r + 1; j < n; ++j) x[r] -= lu[r * n + j] * x[j];
            x[r] /= lu[r * n + r];
        }
        for (int r = 0; r < n; ++r) inv[r * n + col] = x[r];
    }
    return inv;
}

std::vector<double> to_double(const std::vector<xf> &v) {
    std::vector<double> d(v.size());
    for (size_t i = 0; i < v.size(); ++i) d[i] = (double)v[i];
    return d;
}

}  // namespace

RefElem make_refelem(int k) {
    if (k < 1 || k > 4) throw std::runtime_error("degree must be 1..4");
    RefElem E;
    E.k = k;
    E.np = (k + 1) * (k + 2) / 2;
    E.nfp = k + 1;
    const int np = E.np, nfp = E.nfp;
    std::vector<Poly> phi;
    std::vector<xf> nodes;
    int idx[5][5];
    for (int j = 0; j <= k; ++j)
        for (int i = 0; i <= k - j; ++i) {
            idx[i][j] = (int)phi.size();
            phi.push_back(silvester(k, i, j));
            nodes.push_back((xf)i / k);
            nodes.push_back((xf)j / k);
        }
    E.nodes = to_double(nodes);
    std::vector<xf> M(np * np), Dr(np * np), Ds(np * np);
    for (int a = 0; a < np; ++a) {
        const Poly pr = phi[a].dr(), ps = phi[a].ds();
        for (int i = 0; i < np; ++i) {
            Dr[i * np + a] = pr.eval(nodes[2 * i], nodes[2 * i + 1]);
            Ds[i * np + a] = ps.eval(nodes[2 * i], nodes[2 * i + 1]);
        }
        for (int b = 0; b < np; ++b) M[a * np + b] = integrate(phi[a] * phi[b]);
    }
    const std::vector<xf> Minv = lu_inverse(M, np);
    E.M = to_double(M);
    E.Minv = to_double(Minv);
    E.Dr = to_double(Dr);
    E.Ds = to_double(Ds);
    // facet f joins local vertices f and f+1 (mod 3); nodes from the first vertex
    E.fnodes.assign(3 * nfp, 0);
    for (int t = 0; t <= k; ++t) {
        E.fnodes[0 * nfp + t] = idx[t][0];
        E.fnodes[1 * nfp + t] = idx[k - t][t];
        E.fnodes[2 * nfp + t] = idx[0][k - t];
    }
    // 1-D facet mass on [0,1] with the equispaced Lagrange basis (exact moments)
    std::vector<xf> M1(nfp * nfp, 0);
    {
        std::vector<std::vector<xf>> coef(nfp);
        for (int m = 0; m < nfp; ++m) {
            std::vector<xf> c(1, 1);
            for (int q = 0; q < nfp; ++q) {
                if (q == m) continue;
                const xf den = (xf)(m - q) / k;
                std::vector<xf> nc(c.size() + 1, 0);
                for (size_t e = 0; e < c.size(); ++e) {
                    nc[e + 1] += c[e] / den;
                    nc[e] -= c[e] * ((xf)q / k) / den;
                }
                c = nc;
            }
            coef[m] = c;
        }
        for (int a = 0; a < nfp; ++a)
            for (int b = 0; b < nfp; ++b) {
                xf v = 0;
                for (size_t e1 = 0; e1 < coef[a].size(); ++e1)
                    for (size_t e2 = 0; e2 < coef[b].size(); ++e2) v += coef[a][e1] * coef[b][e2] / (xf)(e1 + e2 + 1);
                M1[a * nfp + b] = v;
            }
    }
    E.M1 = to_double(M1);
    // LIFT_f = Mhat^{-1} E_f M1 : [3][Np][Nfp]
    E.lift.assign(3 * np * nfp, 0.0);
    for (int f = 0; f < 3; ++f)
        for (int i = 0; i < np; ++i)
            for (int m = 0; m < nfp; ++m) {
                xf v = 0;
                for (int q = 0; q < nfp; ++q) v += Minv[i * np + E.fnodes[f * nfp + q]] * M1[q * nfp + m];
                E.lift[(f * np + i) * nfp + m] = (double)v;
            }
    E.phi = [phi](double r, double s, double *out) {
        for (size_t i = 0; i < phi.size(); ++i) out[i] = (double)phi[i].eval((xf)r, (xf)s);
    };
    return E;
}

}  // namespace dgt
