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

/* Gauss-Legendre rule with n points on [0,1] (Newton on P_n). */
static void gauss_legendre01(int n, double *x, double *w) {
    for (int i = 0; i < n; i++) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; m++) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1;
            double pnm1 = (n == 1) ? 1.0 : p0;
            double dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; m++) {
            double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        double pn = (n == 1) ? z : p1, pnm1 = (n == 1) ? 1.0 : p0;
        double dp = n * (z * pn - pnm1) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp); /* 2/((1-z^2)P'^2) scaled by 1/2 */
    }
}

int or_tri_quad(int n, double *pts, double *w) {
    double *u = malloc(sizeof(double) * n), *wu = malloc(sizeof(double) * n);
    gauss_legendre01(n, u, wu);
    int q = 0;
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) {
            /* (r, s) = (u_a, (1-u_a) u_b), Jacobian (1-u_a) */
            pts[2 * q] = u[a];
            pts[2 * q + 1] = (1.0 - u[a]) * u[b];
            w[q] = wu[a] * wu[b] * (1.0 - u[a]);
            q++;
        }
    free(u);
    free(wu);
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

static double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

/* Gauss-Jordan inverse with partial pivoting; returns 0 if singular. */
static int invert(int n, const double *A, double *Ainv) {
    double *a = malloc(sizeof(double) * n * 2 * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++)
            a[i * 2 * n + j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(a[r * 2 * n + c]) > fabs(a[p * 2 * n + c])) p = r;
        if (fabs(a[p * 2 * n + c]) < 1e-300) {
            free(a);
            return 0;
        }
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                double t = a[c * 2 * n + j];
                a[c * 2 * n + j] = a[p * 2 * n + j];
                a[p * 2 * n + j] = t;
            }
        double d = a[c * 2 * n + c];
        for (int j = 0; j < 2 * n; j++) a[c * 2 * n + j] /= d;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double f = a[r * 2 * n + c];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; j++) a[r * 2 * n + j] -= f * a[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = a[i * 2 * n + n + j];
    free(a);
    return 1;
}

static void ref_nodes(int k, double *nodes) {
    int m = 0;
    for (int j = 0; j <= k; j++)
        for (int i = 0; i <= k - j; i++) {
            nodes[2 * m] = (double)i / k;
            nodes[2 * m + 1] = (double)j / k;
            m++;
        }
}

/* Coefficients C[m*Np+i] of phi_i in the monomial basis: C = V^{-1}. */
static int lagrange_coeffs(int k, double *C) {
    int np = or_np(k);
    int ea[15], eb[15];
    double nodes[30];
    mono_exps(k, ea, eb);
    ref_nodes(k, nodes);
    double V[225];
    for (int n = 0; n < np; n++)
        for (int m = 0; m < np; m++) V[n * np + m] = ipow(nodes[2 * n], ea[m]) * ipow(nodes[2 * n + 1], eb[m]);
    return invert(np, V, C);
}

static void eval_basis(int k, const double *C, double r, double s, double *phi, double *dr, double *ds) {
    int np = or_np(k);
    int ea[15], eb[15];
    mono_exps(k, ea, eb);
    for (int i = 0; i < np; i++) {
        double p = 0, pr = 0, ps = 0;
        for (int m = 0; m < np; m++) {
            double c = C[m * np + i];
            p += c * ipow(r, ea[m]) * ipow(s, eb[m]);
            if (ea[m] > 0) pr += c * ea[m] * ipow(r, ea[m] - 1) * ipow(s, eb[m]);
            if (eb[m] > 0) ps += c * eb[m] * ipow(r, ea[m]) * ipow(s, eb[m] - 1);
        }
        if (phi) phi[i] = p;
        if (dr) dr[i] = pr;
        if (ds) ds[i] = ps;
    }
}

int or_basis(int k, double r, double s, double *phi) {
    if (k < 1 || k > 4) return -1;
    double C[225];
    if (!lagrange_coeffs(k, C)) return -2;
    eval_basis(k, C, r, s, phi, NULL, NULL);
    return 0;
}

/* Internal: basis values + derivatives (used by dg.c). */
int or_basis_full(int k, double r, double s, double *phi, double *dr, double *ds) {
    double C[225];
    if (!lagrange_coeffs(k, C)) return -2;
    eval_basis(k, C, r, s, phi, dr, ds);
    return 0;
}

int or_refelem(int k, double *nodes, double *M, double *Minv, double *Dr, double *Ds, double *M1,
               int32_t *fnodes) {
    if (k < 1 || k > 4) return -1;
    int np = or_np(k), nfp = k + 1;
    double C[225], nd[30];
    if (!lagrange_coeffs(k, C)) return -2;
    ref_nodes(k, nd);
    if (nodes) memcpy(nodes, nd, sizeof(double) * 2 * np);
    double Mloc[225];
    {
        int nq1 = k + 2;
        double pts[2 * 36], w[36], phi[15];
        int nq = or_tri_quad(nq1, pts, w);
        memset(Mloc, 0, sizeof(Mloc));
        for (int q = 0; q < nq; q++) {
            eval_basis(k, C, pts[2 * q], pts[2 * q + 1], phi, NULL, NULL);
            for (int i = 0; i < np; i++)
                for (int j = 0; j < np; j++) Mloc[i * np + j] += w[q] * phi[i] * phi[j];
        }
    }
    if (M) memcpy(M, Mloc, sizeof(double) * np * np);
    if (Minv && !invert(np, Mloc, Minv)) return -2;
    if (Dr || Ds) {
        double phi[15], pr[15], ps[15];
        for (int i = 0; i < np; i++) {
            eval_basis(k, C, nd[2 * i], nd[2 * i + 1], phi, pr, ps);
            for (int j = 0; j < np; j++) {
                if (Dr) Dr[i * np + j] = pr[j];
                if (Ds) Ds[i * np + j] = ps[j];
            }
        }
    }
    if (M1) {
        /* 1-D Lagrange basis on t_m = m/k, facet mass by Gauss-Legendre */
        double V[25], Ci[25];
        for (int a = 0; a < nfp; a++)
            for (int m = 0; m < nfp; m++) V[a * nfp + m] = ipow((double)a / k, m);
        if (!invert(nfp, V, Ci)) return -2;
        int nq = k + 2;
        double x[8], w[8];
        gauss_legendre01(nq, x, w);
        memset(M1, 0, sizeof(double) * nfp * nfp);
        for (int q = 0; q < nq; q++) {
            double psi[5];
            for (int a = 0; a < nfp; a++) {
                double p = 0;
                for (int m = 0; m < nfp; m++) p += Ci[m * nfp + a] * ipow(x[q], m);
                psi[a] = p;
            }
            for (int a = 0; a < nfp; a++)
                for (int b = 0; b < nfp; b++) M1[a * nfp + b] += w[q] * psi[a] * psi[b];
        }
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
