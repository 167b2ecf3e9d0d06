/*
 * refelem.c -- oracle reference triangle (test infrastructure only).
 *
 * The paper discretises the elastic equations with discontinuous Galerkin in
 * space (Sec. 7.1) but prints no element; the reading used here is nodal
 * Lagrange P_k (k = 1..4) on the equispaced nodes (i/k, j/k), i+j <= k, of the
 * reference triangle {(0,0),(1,0),(0,1)}, nodes ordered by j then i.
 *
 * Everything is built the plain way: a monomial Vandermonde matrix inverted by
 * Gauss-Jordan elimination gives the Lagrange basis, and integrals use a
 * collapsed (Duffy) product of Gauss-Legendre rules that is exact for the
 * polynomial degrees involved.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int or_np(int k) { return (k + 1) * (k + 2) / 2; }

/*
 * Precision.  Every table of the element (quadrature rules, monomial
 * coefficients of the basis, mass matrices and their inverse, derivative
 * matrices) is computed in IEEE binary128 (gcc's __float128: soft-float
 * arithmetic, 113-bit significand) and rounded to double once, when it leaves
 * this file.  In double precision the equispaced P4 Vandermonde and mass
 * inversions lose about two digits, which put the tables 1e-14 away from the
 * exact rationals; with 113 bits the rounding to double is the only error
 * left in them.
 */
typedef __float128 qreal;

static qreal qabs(qreal x) { return x < 0 ? -x : x; }

/* Gauss-Legendre rule with n points on [0,1]: Newton on P_n from the
 * Chebyshev-like guess cos(pi (i + 3/4) / (n + 1/2)), iterated in binary128. */
static void gauss_legendre01_q(int n, qreal *x, qreal *w) {
    for (int i = 0; i < n; i++) {
        qreal z = (qreal)cos(M_PI * (i + 0.75) / (n + 0.5));
        qreal pn = 0, dp = 1;
        for (int it = 0; it < 200; it++) {
            qreal p0 = 1, p1 = z;
            for (int m = 2; m <= n; m++) {
                qreal p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? z : p1;
            qreal pnm1 = (n == 1) ? 1 : p0;
            dp = n * (z * pn - pnm1) / (z * z - 1);
            qreal dz = pn / dp;
            z -= dz;
            if (qabs(dz) < (qreal)1e-33) break;
        }
        qreal p0 = 1, p1 = z;
        for (int m = 2; m <= n; m++) {
            qreal p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        qreal pnm1 = (n == 1) ? 1 : p0;
        pn = (n == 1) ? z : p1;
        dp = n * (z * pn - pnm1) / (z * z - 1);
        x[i] = (1 - z) / 2;
        w[i] = 1 / ((1 - z * z) * dp * dp); /* 2/((1-z^2)P'^2) scaled by 1/2 */
    }
}

static void gauss_legendre01(int n, double *x, double *w) {
    qreal xq[16], wq[16];
    gauss_legendre01_q(n, xq, wq);
    for (int i = 0; i < n; i++) {
        x[i] = (double)xq[i];
        w[i] = (double)wq[i];
    }
}

/* collapsed (Duffy) product rule on the reference triangle, n*n points */
static int tri_quad_q(int n, qreal *pts, qreal *w) {
    qreal u[16], wu[16];
    gauss_legendre01_q(n, u, wu);
    int q = 0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            /* (r, s) = (u_a, (1-u_a) u_b), Jacobian (1-u_a) */
            pts[2 * q] = u[a];
            pts[2 * q + 1] = (1 - u[a]) * u[b];
            w[q] = wu[a] * wu[b] * (1 - u[a]);
            q++;
        }
    return q;
}

int or_tri_quad(int n, double *pts, double *w) {
    if (n < 1 || n > 16) return -1;
    qreal pq[2 * 256], wq[256];
    int q = tri_quad_q(n, pq, wq);
    for (int i = 0; i < q; i++) {
        pts[2 * i] = (double)pq[2 * i];
        pts[2 * i + 1] = (double)pq[2 * i + 1];
        w[i] = (double)wq[i];
    }
    return q;
}

/* monomial exponent list, a+b <= k */
static void mono_exps(int k, int *ea, int *eb) {
    int m = 0;
    for (int d = 0; d <= k; d++)
        for (int b = 0; b <= d; b++) {
            ea[m] = d - b;
            eb[m] = b;
            m++;
        }
}

static qreal ipow(qreal x, int e) {
    qreal r = 1;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 if singular. */
static int invert(int n, const qreal *A, qreal *Ainv) {
    qreal a[15 * 30];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++)
            a[i * 2 * n + j] = (j < n) ? A[i * n + j] : (j - n == i ? 1 : 0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (qabs(a[r * 2 * n + c]) > qabs(a[p * 2 * n + c])) p = r;
        if (qabs(a[p * 2 * n + c]) < (qreal)1e-300) return 0;
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                qreal t = a[c * 2 * n + j];
                a[c * 2 * n + j] = a[p * 2 * n + j];
                a[p * 2 * n + j] = t;
            }
        qreal d = a[c * 2 * n + c];
        for (int j = 0; j < 2 * n; j++) a[c * 2 * n + j] /= d;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            qreal f = a[r * 2 * n + c];
            if (f != 0)
                for (int j = 0; j < 2 * n; j++) a[r * 2 * n + j] -= f * a[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = a[i * 2 * n + n + j];
    return 1;
}

static void ref_nodes(int k, qreal *nodes) {
    int m = 0;
    for (int j = 0; j <= k; j++)
        for (int i = 0; i <= k - j; i++) {
            nodes[2 * m] = (qreal)i / k;
            nodes[2 * m + 1] = (qreal)j / k;
            m++;
        }
}

/* Coefficients C[m*Np+i] of phi_i in the monomial basis: C = V^{-1}. */
static int lagrange_coeffs(int k, qreal *C) {
    int np = or_np(k);
    int ea[15], eb[15];
    qreal nodes[30];
    mono_exps(k, ea, eb);
    ref_nodes(k, nodes);
    qreal V[225];
    for (int n = 0; n < np; n++)
        for (int m = 0; m < np; m++) V[n * np + m] = ipow(nodes[2 * n], ea[m]) * ipow(nodes[2 * n + 1], eb[m]);
    return invert(np, V, C);
}

static void eval_basis(int k, const qreal *C, qreal r, qreal s, qreal *phi, qreal *dr, qreal *ds) {
    int np = or_np(k);
    int ea[15], eb[15];
    mono_exps(k, ea, eb);
    for (int i = 0; i < np; i++) {
        qreal p = 0, pr = 0, ps = 0;
        for (int m = 0; m < np; m++) {
            qreal c = C[m * np + i];
            p += c * ipow(r, ea[m]) * ipow(s, eb[m]);
            if (ea[m] > 0) pr += c * ea[m] * ipow(r, ea[m] - 1) * ipow(s, eb[m]);
            if (eb[m] > 0) ps += c * eb[m] * ipow(r, ea[m]) * ipow(s, eb[m] - 1);
        }
        if (phi) phi[i] = p;
        if (dr) dr[i] = pr;
        if (ds) ds[i] = ps;
    }
}

static void round_out(int n, const qreal *q, double *d) {
    if (d)
        for (int i = 0; i < n; i++) d[i] = (double)q[i];
}

int or_basis(int k, double r, double s, double *phi) {
    if (k < 1 || k > 4) return -1;
    qreal C[225], p[15];
    if (!lagrange_coeffs(k, C)) return -2;
    eval_basis(k, C, r, s, p, NULL, NULL);
    round_out(or_np(k), p, phi);
    return 0;
}

/* Internal: basis values + derivatives (used by dg.c). */
int or_basis_full(int k, double r, double s, double *phi, double *dr, double *ds) {
    qreal C[225], p[15], pr[15], ps[15];
    if (!lagrange_coeffs(k, C)) return -2;
    eval_basis(k, C, r, s, p, pr, ps);
    round_out(or_np(k), p, phi);
    round_out(or_np(k), pr, dr);
    round_out(or_np(k), ps, ds);
    return 0;
}

int or_refelem(int k, double *nodes, double *M, double *Minv, double *Dr, double *Ds, double *M1,
               int32_t *fnodes) {
    if (k < 1 || k > 4) return -1;
    int np = or_np(k), nfp = k + 1;
    qreal C[225], nd[30];
    if (!lagrange_coeffs(k, C)) return -2;
    ref_nodes(k, nd);
    round_out(2 * np, nd, nodes);
    qreal Mloc[225], Mi[225];
    {
        int nq1 = k + 2;
        qreal pts[2 * 36], w[36], phi[15];
        int nq = tri_quad_q(nq1, pts, w);
        for (int i = 0; i < np * np; i++) Mloc[i] = 0;
        for (int q = 0; q < nq; q++) {
            eval_basis(k, C, pts[2 * q], pts[2 * q + 1], phi, NULL, NULL);
            for (int i = 0; i < np; i++)
                for (int j = 0; j < np; j++) Mloc[i * np + j] += w[q] * phi[i] * phi[j];
        }
    }
    round_out(np * np, Mloc, M);
    if (Minv) {
        if (!invert(np, Mloc, Mi)) return -2;
        round_out(np * np, Mi, Minv);
    }
    if (Dr || Ds) {
        qreal phi[15], pr[15], ps[15];
        for (int i = 0; i < np; i++) {
            eval_basis(k, C, nd[2 * i], nd[2 * i + 1], phi, pr, ps);
            for (int j = 0; j < np; j++) {
                if (Dr) Dr[i * np + j] = (double)pr[j];
                if (Ds) Ds[i * np + j] = (double)ps[j];
            }
        }
    }
    if (M1) {
        /* 1-D Lagrange basis on t_m = m/k, facet mass by Gauss-Legendre */
        qreal V[25], Ci[25], x[8], w[8], Mf[25];
        for (int a = 0; a < nfp; a++)
            for (int m = 0; m < nfp; m++) V[a * nfp + m] = ipow((qreal)a / k, m);
        if (!invert(nfp, V, Ci)) return -2;
        int nq = k + 2;
        gauss_legendre01_q(nq, x, w);
        for (int i = 0; i < nfp * nfp; i++) Mf[i] = 0;
        for (int q = 0; q < nq; q++) {
            qreal psi[5];
            for (int a = 0; a < nfp; a++) {
                qreal p = 0;
                for (int m = 0; m < nfp; m++) p += Ci[m * nfp + a] * ipow(x[q], m);
                psi[a] = p;
            }
            for (int a = 0; a < nfp; a++)
                for (int b = 0; b < nfp; b++) Mf[a * nfp + b] += w[q] * psi[a] * psi[b];
        }
        round_out(nfp * nfp, Mf, M1);
    }
    if (fnodes) {
        /* facet f joins local vertices f and f+1 (mod 3); its nodes run from the
         * first vertex to the second. */
        int idx[5][5];
        int m = 0;
        for (int j = 0; j <= k; j++)
            for (int i = 0; i <= k - j; i++) idx[i][j] = m++;
        for (int t = 0; t <= k; t++) {
            fnodes[0 * nfp + t] = idx[t][0];
            fnodes[1 * nfp + t] = idx[k - t][t];
            fnodes[2 * nfp + t] = idx[0][k - t];
        }
    }
    return 0;
}

/* Gauss-Legendre on [0,1] for dg.c */
void or_gl01(int n, double *x, double *w) { gauss_legendre01(n, x, w); }
