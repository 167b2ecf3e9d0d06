/*
 * dg.c -- oracle velocity-stress DG loop chain (test infrastructure only).
 *
 * The paper's application (Sec. 7.1-7.2) is a velocity-stress elastic solver,
 * DG in space, with a fourth-order explicit leapfrog from a truncated Taylor
 * series in time; each step is a chain of cell, interior-facet and exterior-
 * facet assembly loops followed by element-local inverse-mass solves.  The
 * paper prints no equations, so the following readings are fixed here and
 * written out in the plainest form (quadrature on every integral, then a
 * block-diagonal solve):
 *
 *  PDE      rho dv/dt = div(sigma),  dsigma/dt = lam tr(eps) I + 2 mu eps,
 *           eps = sym grad v (2-D, fields vx, vy, sxx, syy, sxy).
 *  Space    strong-form nodal DG P_k, affine cells:
 *             rho M_K U = int_K phi div(S) + sum_f int_f phi (T* - T^-)
 *                 M_K X = int_K phi C eps(V) + sum_f int_f phi C sym((v* - v^-) x n)
 *  Flux     central: averages; upwind: exact isotropic Riemann state.  Upwind
 *           is split into the part driven by the operated field (kept in the
 *           operators A, B) and the part driven by the other field (the
 *           penalties D_v, D_s), which is lagged in time.
 *  BCs      free surface: mirror ghost (sigma+ = -sigma-, v+ = v-);
 *           absorbing: zero ghost with the upwind formula.
 *  Time     staggered; v at half steps, sigma at integer steps:
 *             v^{n+1/2} = v^{n-1/2} + dt (A s^n + D_v v^{n-1/2}) + dt^3/24 A B A s^n
 *             s^{n+1}   = s^n + dt (B v^{n+1/2} + D_s s^n) + dt^3/24 B A B v^{n+1/2}
 *                         + dt r(t^{n+1/2}) M_K^{-1} phi(x_s) on sxx, syy
 *           (order 2 drops the dt^3 terms).
 * Loops iterate in ascending id; increments are applied in that order.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* from refelem.c / mesh.c */
int or_basis_full(int k, double r, double s, double *phi, double *dr, double *ds);
void or_gl01(int n, double *x, double *w);
const double *or_mesh_xy(const or_mesh *m);
const int32_t *or_mesh_c2v(const or_mesh *m);
const int32_t *or_mesh_f2c(const or_mesh *m);
const int8_t *or_mesh_f2l(const or_mesh *m);
const int32_t *or_mesh_b2c(const or_mesh *m);
const int8_t *or_mesh_b2l(const or_mesh *m);
const int8_t *or_mesh_bside(const or_mesh *m);

/* data spaces on the cells */
enum { D_V, D_S, D_BV, D_PV, D_BS, D_PS, D_U1, D_S1, D_U2, D_PVS, D_V1, D_W1, D_S2, D_PSS, D_COUNT };
static const int ds_ncomp[D_COUNT] = {2, 3, 2, 2, 3, 3, 2, 3, 2, 2, 3, 2, 3, 3};

enum { K_VOL_V, K_INT_V, K_EXT_V, K_SOLVE_V, K_VOL_S, K_INT_S, K_EXT_S, K_SOLVE_S, K_UPD_V, K_UPD_S,
       K_SOLUPD_V, K_SOLUPD_S };

typedef struct {
    int kind, in, out, pin, pout;
} dg_loop;

struct or_dg {
    const or_mesh *mesh;
    int k, np, nfp;
    int64_t nc, nf, nb;
    const int32_t *f2c, *b2c;
    const int8_t *f2l, *b2l, *bside;
    double *J;    /* [nc*4]  x_r, x_s, y_r, y_s */
    double *Ji;   /* [nc*4]  r_x, r_y, s_x, s_y */
    double *det;  /* [nc] */
    double *x0;   /* [nc*2] */
    double *lam, *mu, *rho;
    double *Minv; /* Np*Np */
    /* triangle quadrature with basis tables */
    int nq;
    double *qw, *qphi, *qdr, *qds; /* [nq], [nq*Np] */
    /* facet quadrature: per local facet f and orientation o (0: forward, 1: reversed), basis at points */
    int nq1;
    double *q1w;   /* [nq1] */
    double *q1phi; /* [3][2][nq1][Np] */
    int flux, order, free_sides, has_pen;
    double dt;
    /* source */
    int src_cell;
    double src_f0, src_t0, src_amp;
    double *src_vec; /* [Np] = M_K^{-1} phi(x_s) */
    /* chain */
    int nloops;
    dg_loop loops[26];
    double *data[D_COUNT];
    double t_half; /* source time of the current step */
};

double or_ricker(double t, double f0, double t0, double amp) {
    double a = M_PI * M_PI * f0 * f0 * (t - t0) * (t - t0);
    return amp * (1.0 - 2.0 * a) * exp(-a);
}

static void facet_point(int l, double t, double *r, double *s) {
    if (l == 0) { *r = t; *s = 0.0; }
    else if (l == 1) { *r = 1.0 - t; *s = t; }
    else { *r = 0.0; *s = 1.0 - t; }
}

double or_cfl_dt(const or_mesh *m, int k, const double *lam, const double *mu, const double *rho, double cfl) {
    const double *xy = or_mesh_xy(m);
    const int32_t *c2v = or_mesh_c2v(m);
    int64_t nc;
    or_mesh_counts(m, &nc, NULL, NULL);
    double hmin = INFINITY, cmax = 0.0;
    for (int64_t c = 0; c < nc; c++) {
        const double *p[3] = {xy + 2 * c2v[3 * c], xy + 2 * c2v[3 * c + 1], xy + 2 * c2v[3 * c + 2]};
        double area = 0.5 * ((p[1][0] - p[0][0]) * (p[2][1] - p[0][1]) - (p[2][0] - p[0][0]) * (p[1][1] - p[0][1]));
        double per = 0.0;
        for (int i = 0; i < 3; i++) per += hypot(p[(i + 1) % 3][0] - p[i][0], p[(i + 1) % 3][1] - p[i][1]);
        double h = 4.0 * area / per; /* twice the inradius */
        if (h < hmin) hmin = h;
        double cp = sqrt((lam[c] + 2.0 * mu[c]) / rho[c]);
        if (cp > cmax) cmax = cp;
    }
    return cfl * hmin / ((2.0 * k + 1.0) * cmax);
}

static void build_chain(or_dg *d) {
    int n = 0;
    int pv = d->has_pen ? D_PV : -1, ps = d->has_pen ? D_PS : -1;
    int pvs = d->has_pen ? D_PVS : -1, pss = d->has_pen ? D_PSS : -1;
    if (d->order == 2) {
        d->loops[n++] = (dg_loop){K_VOL_V, D_S, D_BV, -1, pv};
        d->loops[n++] = (dg_loop){K_INT_V, D_S, D_BV, d->has_pen ? D_V : -1, pv};
        d->loops[n++] = (dg_loop){K_EXT_V, D_S, D_BV, d->has_pen ? D_V : -1, pv};
        d->loops[n++] = (dg_loop){K_SOLUPD_V, D_BV, D_V, pv, -1};
        d->loops[n++] = (dg_loop){K_VOL_S, D_V, D_BS, -1, ps};
        d->loops[n++] = (dg_loop){K_INT_S, D_V, D_BS, d->has_pen ? D_S : -1, ps};
        d->loops[n++] = (dg_loop){K_EXT_S, D_V, D_BS, d->has_pen ? D_S : -1, ps};
        d->loops[n++] = (dg_loop){K_SOLUPD_S, D_BS, D_S, ps, -1};
    } else {
        /* velocity half step */
        d->loops[n++] = (dg_loop){K_VOL_V, D_S, D_BV, -1, pv};
        d->loops[n++] = (dg_loop){K_INT_V, D_S, D_BV, d->has_pen ? D_V : -1, pv};
        d->loops[n++] = (dg_loop){K_EXT_V, D_S, D_BV, d->has_pen ? D_V : -1, pv};
        d->loops[n++] = (dg_loop){K_SOLVE_V, D_BV, D_U1, pv, pvs};
        d->loops[n++] = (dg_loop){K_VOL_S, D_U1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_INT_S, D_U1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_EXT_S, D_U1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_SOLVE_S, D_BS, D_S1, -1, -1};
        d->loops[n++] = (dg_loop){K_VOL_V, D_S1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_INT_V, D_S1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_EXT_V, D_S1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_SOLVE_V, D_BV, D_U2, -1, -1};
        d->loops[n++] = (dg_loop){K_UPD_V, -1, D_V, -1, -1};
        /* stress half step */
        d->loops[n++] = (dg_loop){K_VOL_S, D_V, D_BS, -1, ps};
        d->loops[n++] = (dg_loop){K_INT_S, D_V, D_BS, d->has_pen ? D_S : -1, ps};
        d->loops[n++] = (dg_loop){K_EXT_S, D_V, D_BS, d->has_pen ? D_S : -1, ps};
        d->loops[n++] = (dg_loop){K_SOLVE_S, D_BS, D_V1, ps, pss};
        d->loops[n++] = (dg_loop){K_VOL_V, D_V1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_INT_V, D_V1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_EXT_V, D_V1, D_BV, -1, -1};
        d->loops[n++] = (dg_loop){K_SOLVE_V, D_BV, D_W1, -1, -1};
        d->loops[n++] = (dg_loop){K_VOL_S, D_W1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_INT_S, D_W1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_EXT_S, D_W1, D_BS, -1, -1};
        d->loops[n++] = (dg_loop){K_SOLVE_S, D_BS, D_S2, -1, -1};
        d->loops[n++] = (dg_loop){K_UPD_S, -1, D_S, -1, -1};
    }
    d->nloops = n;
}

int or_dg_create(const or_mesh *m, int k, const double *lam, const double *mu, const double *rho, int flux,
                 int order, double dt, int free_sides, or_dg **out) {
    *out = NULL;
    if (k < 1 || k > 4 || (order != 2 && order != 4) || (flux != 0 && flux != 1)) return -1;
    or_dg *d = calloc(1, sizeof(*d));
    d->mesh = m;
    d->k = k;
    d->np = or_np(k);
    d->nfp = k + 1;
    or_mesh_counts(m, &d->nc, &d->nf, &d->nb);
    d->f2c = or_mesh_f2c(m);
    d->f2l = or_mesh_f2l(m);
    d->b2c = or_mesh_b2c(m);
    d->b2l = or_mesh_b2l(m);
    d->bside = or_mesh_bside(m);
    d->flux = flux;
    d->order = order;
    d->dt = dt;
    d->free_sides = free_sides;
    int64_t nc = d->nc, np = d->np;
    const double *xy = or_mesh_xy(m);
    const int32_t *c2v = or_mesh_c2v(m);
    d->J = malloc(sizeof(double) * 4 * (nc + 1));
    d->Ji = malloc(sizeof(double) * 4 * (nc + 1));
    d->det = malloc(sizeof(double) * (nc + 1));
    d->x0 = malloc(sizeof(double) * 2 * (nc + 1));
    d->lam = malloc(sizeof(double) * (nc + 1));
    d->mu = malloc(sizeof(double) * (nc + 1));
    d->rho = malloc(sizeof(double) * (nc + 1));
    for (int64_t c = 0; c < nc; c++) {
        const double *p0 = xy + 2 * c2v[3 * c], *p1 = xy + 2 * c2v[3 * c + 1], *p2 = xy + 2 * c2v[3 * c + 2];
        double xr = p1[0] - p0[0], xs = p2[0] - p0[0], yr = p1[1] - p0[1], ys = p2[1] - p0[1];
        double det = xr * ys - xs * yr;
        d->J[4 * c + 0] = xr; d->J[4 * c + 1] = xs; d->J[4 * c + 2] = yr; d->J[4 * c + 3] = ys;
        d->Ji[4 * c + 0] = ys / det;   /* r_x */
        d->Ji[4 * c + 1] = -xs / det;  /* r_y */
        d->Ji[4 * c + 2] = -yr / det;  /* s_x */
        d->Ji[4 * c + 3] = xr / det;   /* s_y */
        d->det[c] = det;
        d->x0[2 * c] = p0[0];
        d->x0[2 * c + 1] = p0[1];
        d->lam[c] = lam[c];
        d->mu[c] = mu[c];
        d->rho[c] = rho[c];
    }
    d->Minv = malloc(sizeof(double) * np * np);
    or_refelem(k, NULL, NULL, d->Minv, NULL, NULL, NULL, NULL);
    /* triangle quadrature of degree >= 2k+1 */
    int n1 = k + 2;
    d->nq = n1 * n1;
    double *pts = malloc(sizeof(double) * 2 * d->nq);
    d->qw = malloc(sizeof(double) * d->nq);
    or_tri_quad(n1, pts, d->qw);
    d->qphi = malloc(sizeof(double) * d->nq * np);
    d->qdr = malloc(sizeof(double) * d->nq * np);
    d->qds = malloc(sizeof(double) * d->nq * np);
    for (int q = 0; q < d->nq; q++)
        or_basis_full(k, pts[2 * q], pts[2 * q + 1], d->qphi + q * np, d->qdr + q * np, d->qds + q * np);
    free(pts);
    d->nq1 = k + 2;
    double x1[8];
    d->q1w = malloc(sizeof(double) * d->nq1);
    or_gl01(d->nq1, x1, d->q1w);
    d->q1phi = malloc(sizeof(double) * 3 * 2 * d->nq1 * np);
    for (int l = 0; l < 3; l++)
        for (int o = 0; o < 2; o++)
            for (int q = 0; q < d->nq1; q++) {
                double r, s;
                facet_point(l, o ? 1.0 - x1[q] : x1[q], &r, &s);
                or_basis_full(k, r, s, d->q1phi + ((l * 2 + o) * d->nq1 + q) * np, NULL, NULL);
            }
    d->has_pen = (flux == 1);
    for (int64_t b = 0; b < d->nb; b++)
        if (!(d->bside[b] >= 0 && ((free_sides >> d->bside[b]) & 1))) d->has_pen = 1;
    for (int i = 0; i < D_COUNT; i++) d->data[i] = calloc((size_t)ds_ncomp[i] * np * nc + 1, sizeof(double));
    d->src_cell = -1;
    d->src_vec = calloc(np, sizeof(double));
    build_chain(d);
    *out = d;
    return 0;
}

void or_dg_free(or_dg *d) {
    if (!d) return;
    free(d->J); free(d->Ji); free(d->det); free(d->x0); free(d->lam); free(d->mu); free(d->rho);
    free(d->Minv); free(d->qw); free(d->qphi); free(d->qdr); free(d->qds); free(d->q1w); free(d->q1phi);
    free(d->src_vec);
    for (int i = 0; i < D_COUNT; i++) free(d->data[i]);
    free(d);
}

int or_dg_set_source(or_dg *d, double x, double y, double f0, double t0, double amp) {
    d->src_cell = -1;
    /* lowest cell id whose barycentric coordinates are all >= -1e-12 */
    for (int64_t c = 0; c < d->nc; c++) {
        double dx = x - d->x0[2 * c], dy = y - d->x0[2 * c + 1];
        double r = d->Ji[4 * c + 0] * dx + d->Ji[4 * c + 1] * dy;
        double s = d->Ji[4 * c + 2] * dx + d->Ji[4 * c + 3] * dy;
        if (r >= -1e-12 && s >= -1e-12 && 1.0 - r - s >= -1e-12) {
            double phi[15];
            or_basis_full(d->k, r, s, phi, NULL, NULL);
            for (int i = 0; i < d->np; i++) {
                double a = 0.0;
                for (int j = 0; j < d->np; j++) a += d->Minv[i * d->np + j] * phi[j];
                d->src_vec[i] = a / d->det[c];
            }
            d->src_cell = (int)c;
            break;
        }
    }
    d->src_f0 = f0;
    d->src_t0 = t0;
    d->src_amp = amp;
    return d->src_cell >= 0 ? 0 : -1;
}

int or_dg_source_cell(const or_dg *d) { return d->src_cell; }

/* --------------------------------------------------------------------- */
/* fluxes: inside state (-), outside state (+), outward normal n of inside */

typedef struct {
    double sxx, syy, sxy, vx, vy;
} pstate;

static void imped(const or_dg *d, int64_t c, double *zp, double *zs) {
    *zp = sqrt(d->rho[c] * (d->lam[c] + 2.0 * d->mu[c]));
    *zs = sqrt(d->rho[c] * d->mu[c]);
}

/* T* - T^- from the stress field (the operator part). */
static void flux_v_sigma(int upw, const pstate *in, const pstate *ou, const double *n, double zpi, double zsi,
                         double zpo, double zso, double *g) {
    double Ti[2] = {in->sxx * n[0] + in->sxy * n[1], in->sxy * n[0] + in->syy * n[1]};
    double To[2] = {ou->sxx * n[0] + ou->sxy * n[1], ou->sxy * n[0] + ou->syy * n[1]};
    double Ts[2];
    if (!upw) {
        Ts[0] = 0.5 * (Ti[0] + To[0]);
        Ts[1] = 0.5 * (Ti[1] + To[1]);
    } else {
        double t[2] = {-n[1], n[0]};
        double tni = Ti[0] * n[0] + Ti[1] * n[1], tno = To[0] * n[0] + To[1] * n[1];
        double tti = Ti[0] * t[0] + Ti[1] * t[1], tto = To[0] * t[0] + To[1] * t[1];
        double tn = (zpo * tni + zpi * tno) / (zpi + zpo);
        double tt = (zso * tti + zsi * tto) / (zsi + zso);
        Ts[0] = tn * n[0] + tt * t[0];
        Ts[1] = tn * n[1] + tt * t[1];
    }
    g[0] = Ts[0] - Ti[0];
    g[1] = Ts[1] - Ti[1];
}

/* upwind traction driven by the velocity jump (the lagged penalty part). */
static void flux_v_pen(int upw, const pstate *in, const pstate *ou, const double *n, double zpi, double zsi,
                       double zpo, double zso, double *g) {
    g[0] = g[1] = 0.0;
    if (!upw) return;
    double t[2] = {-n[1], n[0]};
    double vni = in->vx * n[0] + in->vy * n[1], vno = ou->vx * n[0] + ou->vy * n[1];
    double vti = in->vx * t[0] + in->vy * t[1], vto = ou->vx * t[0] + ou->vy * t[1];
    double a = zpi * zpo / (zpi + zpo) * (vno - vni);
    double b = zsi * zso / (zsi + zso) * (vto - vti);
    g[0] = a * n[0] + b * t[0];
    g[1] = a * n[1] + b * t[1];
}

/* v* - v^- from the velocity field (the operator part). */
static void flux_s_vel(int upw, const pstate *in, const pstate *ou, const double *n, double zpi, double zsi,
                       double zpo, double zso, double *dv) {
    double vs[2];
    if (!upw) {
        vs[0] = 0.5 * (in->vx + ou->vx);
        vs[1] = 0.5 * (in->vy + ou->vy);
    } else {
        double t[2] = {-n[1], n[0]};
        double vni = in->vx * n[0] + in->vy * n[1], vno = ou->vx * n[0] + ou->vy * n[1];
        double vti = in->vx * t[0] + in->vy * t[1], vto = ou->vx * t[0] + ou->vy * t[1];
        double vn = (zpi * vni + zpo * vno) / (zpi + zpo);
        double vt = (zsi * vti + zso * vto) / (zsi + zso);
        vs[0] = vn * n[0] + vt * t[0];
        vs[1] = vn * n[1] + vt * t[1];
    }
    dv[0] = vs[0] - in->vx;
    dv[1] = vs[1] - in->vy;
}

/* upwind velocity driven by the traction jump (the lagged penalty part). */
static void flux_s_pen(int upw, const pstate *in, const pstate *ou, const double *n, double zpi, double zsi,
                       double zpo, double zso, double *dv) {
    dv[0] = dv[1] = 0.0;
    if (!upw) return;
    double t[2] = {-n[1], n[0]};
    double Ti[2] = {in->sxx * n[0] + in->sxy * n[1], in->sxy * n[0] + in->syy * n[1]};
    double To[2] = {ou->sxx * n[0] + ou->sxy * n[1], ou->sxy * n[0] + ou->syy * n[1]};
    double a = ((To[0] - Ti[0]) * n[0] + (To[1] - Ti[1]) * n[1]) / (zpi + zpo);
    double b = ((To[0] - Ti[0]) * t[0] + (To[1] - Ti[1]) * t[1]) / (zsi + zso);
    dv[0] = a * n[0] + b * t[0];
    dv[1] = a * n[1] + b * t[1];
}

/* --------------------------------------------------------------------- */
/* per-iteration kernels */

#define IDX(d, comp, i, c) (((int64_t)(comp) * (d)->np + (i)) * (d)->nc + (c))

static void eval_at(const or_dg *d, const double *phi, int64_t c, int field, double *out, int ncomp) {
    const double *a = d->data[field];
    for (int comp = 0; comp < ncomp; comp++) {
        double v = 0.0;
        for (int j = 0; j < d->np; j++) v += a[IDX(d, comp, j, c)] * phi[j];
        out[comp] = v;
    }
}

static void kernel_vol(or_dg *d, int64_t c, int vel, int in, int out, int pout) {
    int np = d->np;
    /* the penalty accumulator has no volume term: this loop starts it at zero */
    if (pout >= 0)
        for (int comp = 0; comp < (vel ? 2 : 3); comp++)
            for (int i = 0; i < np; i++) d->data[pout][IDX(d, comp, i, c)] = 0.0;
    const double *ji = d->Ji + 4 * c;
    double detJ = d->det[c];
    const double *a = d->data[in];
    double *b = d->data[out];
    int nco = vel ? 2 : 3;
    for (int comp = 0; comp < nco; comp++)
        for (int i = 0; i < np; i++) b[IDX(d, comp, i, c)] = 0.0;
    for (int q = 0; q < d->nq; q++) {
        const double *pr = d->qdr + q * np, *ps = d->qds + q * np, *ph = d->qphi + q * np;
        double wq = d->qw[q] * detJ;
        double val[3];
        if (vel) {
            /* div(S): (dx sxx + dy sxy, dx sxy + dy syy) */
            double g[3][2] = {{0, 0}, {0, 0}, {0, 0}};
            for (int comp = 0; comp < 3; comp++)
                for (int j = 0; j < np; j++) {
                    double u = a[IDX(d, comp, j, c)];
                    g[comp][0] += u * (pr[j] * ji[0] + ps[j] * ji[2]);
                    g[comp][1] += u * (pr[j] * ji[1] + ps[j] * ji[3]);
                }
            val[0] = g[0][0] + g[2][1];
            val[1] = g[2][0] + g[1][1];
        } else {
            double g[2][2] = {{0, 0}, {0, 0}};
            for (int comp = 0; comp < 2; comp++)
                for (int j = 0; j < np; j++) {
                    double u = a[IDX(d, comp, j, c)];
                    g[comp][0] += u * (pr[j] * ji[0] + ps[j] * ji[2]);
                    g[comp][1] += u * (pr[j] * ji[1] + ps[j] * ji[3]);
                }
            double exx = g[0][0], eyy = g[1][1], exy = 0.5 * (g[0][1] + g[1][0]);
            double l = d->lam[c], mu = d->mu[c];
            val[0] = (l + 2 * mu) * exx + l * eyy;
            val[1] = l * exx + (l + 2 * mu) * eyy;
            val[2] = 2 * mu * exy;
        }
        for (int comp = 0; comp < nco; comp++)
            for (int i = 0; i < np; i++) b[IDX(d, comp, i, c)] += wq * ph[i] * val[comp];
    }
}

static void get_state(const or_dg *d, const double *phi, int64_t c, int fs, int fv, pstate *p) {
    double s[3] = {0, 0, 0}, v[2] = {0, 0};
    if (fs >= 0) eval_at(d, phi, c, fs, s, 3);
    if (fv >= 0) eval_at(d, phi, c, fv, v, 2);
    p->sxx = s[0]; p->syy = s[1]; p->sxy = s[2]; p->vx = v[0]; p->vy = v[1];
}

static void add_face(or_dg *d, int64_t c, const double *phi, double wl, int vel, int out, const double *g,
                     const double *n) {
    double *b = d->data[out];
    int np = d->np;
    if (vel) {
        for (int comp = 0; comp < 2; comp++)
            for (int i = 0; i < np; i++) b[IDX(d, comp, i, c)] += wl * phi[i] * g[comp];
    } else {
        double exx = g[0] * n[0], eyy = g[1] * n[1], exy = 0.5 * (g[0] * n[1] + g[1] * n[0]);
        double l = d->lam[c], mu = d->mu[c];
        double val[3] = {(l + 2 * mu) * exx + l * eyy, l * exx + (l + 2 * mu) * eyy, 2 * mu * exy};
        for (int comp = 0; comp < 3; comp++)
            for (int i = 0; i < np; i++) b[IDX(d, comp, i, c)] += wl * phi[i] * val[comp];
    }
}

static void facet_geom(const or_dg *d, int64_t c, int l, double *n, double *len) {
    const double *xy = or_mesh_xy(d->mesh);
    const int32_t *c2v = or_mesh_c2v(d->mesh);
    const double *pa = xy + 2 * c2v[3 * c + l], *pb = xy + 2 * c2v[3 * c + (l + 1) % 3];
    double dx = pb[0] - pa[0], dy = pb[1] - pa[1];
    double L = hypot(dx, dy);
    n[0] = dy / L;
    n[1] = -dx / L;
    *len = L;
}

/* interior facet f: both sides, each with its own outward normal */
static void kernel_int(or_dg *d, int64_t f, int vel, int in, int out, int pin, int pout) {
    int64_t c[2] = {d->f2c[2 * f], d->f2c[2 * f + 1]};
    int l[2] = {d->f2l[2 * f], d->f2l[2 * f + 1]};
    double n0[2], L;
    facet_geom(d, c[0], l[0], n0, &L);
    double zp[2], zs[2];
    imped(d, c[0], &zp[0], &zs[0]);
    imped(d, c[1], &zp[1], &zs[1]);
    int upw = d->flux == 1;
    for (int q = 0; q < d->nq1; q++) {
        const double *phi[2] = {d->q1phi + ((l[0] * 2 + 0) * d->nq1 + q) * d->np,
                                d->q1phi + ((l[1] * 2 + 1) * d->nq1 + q) * d->np};
        pstate st[2];
        for (int s = 0; s < 2; s++) {
            int fs = vel ? in : (pin >= 0 ? pin : -1);
            int fv = vel ? (pin >= 0 ? pin : -1) : in;
            get_state(d, phi[s], c[s], fs, fv, &st[s]);
        }
        double wl = d->q1w[q] * L;
        for (int s = 0; s < 2; s++) {
            int o = 1 - s;
            double n[2] = {s == 0 ? n0[0] : -n0[0], s == 0 ? n0[1] : -n0[1]};
            double g[2];
            if (vel) {
                flux_v_sigma(upw, &st[s], &st[o], n, zp[s], zs[s], zp[o], zs[o], g);
                add_face(d, c[s], phi[s], wl, 1, out, g, n);
                if (pout >= 0) {
                    flux_v_pen(upw, &st[s], &st[o], n, zp[s], zs[s], zp[o], zs[o], g);
                    add_face(d, c[s], phi[s], wl, 1, pout, g, n);
                }
            } else {
                flux_s_vel(upw, &st[s], &st[o], n, zp[s], zs[s], zp[o], zs[o], g);
                add_face(d, c[s], phi[s], wl, 0, out, g, n);
                if (pout >= 0) {
                    flux_s_pen(upw, &st[s], &st[o], n, zp[s], zs[s], zp[o], zs[o], g);
                    add_face(d, c[s], phi[s], wl, 0, pout, g, n);
                }
            }
        }
    }
}

/* exterior facet b: ghost state from the boundary condition */
static void kernel_ext(or_dg *d, int64_t b, int vel, int in, int out, int pin, int pout) {
    int64_t c = d->b2c[b];
    int l = d->b2l[b];
    double n[2], L;
    facet_geom(d, c, l, n, &L);
    double zp, zs;
    imped(d, c, &zp, &zs);
    int free_surf = d->bside[b] >= 0 && ((d->free_sides >> d->bside[b]) & 1);
    int upw = free_surf ? (d->flux == 1) : 1;
    for (int q = 0; q < d->nq1; q++) {
        const double *phi = d->q1phi + ((l * 2 + 0) * d->nq1 + q) * d->np;
        pstate in_s, gh;
        int fs = vel ? in : (pin >= 0 ? pin : -1);
        int fv = vel ? (pin >= 0 ? pin : -1) : in;
        get_state(d, phi, c, fs, fv, &in_s);
        if (free_surf) {
            gh.sxx = -in_s.sxx; gh.syy = -in_s.syy; gh.sxy = -in_s.sxy; gh.vx = in_s.vx; gh.vy = in_s.vy;
        } else {
            gh.sxx = gh.syy = gh.sxy = gh.vx = gh.vy = 0.0;
        }
        double wl = d->q1w[q] * L, g[2];
        if (vel) {
            flux_v_sigma(upw, &in_s, &gh, n, zp, zs, zp, zs, g);
            add_face(d, c, phi, wl, 1, out, g, n);
            if (pout >= 0) {
                flux_v_pen(upw, &in_s, &gh, n, zp, zs, zp, zs, g);
                add_face(d, c, phi, wl, 1, pout, g, n);
            }
        } else {
            flux_s_vel(upw, &in_s, &gh, n, zp, zs, zp, zs, g);
            add_face(d, c, phi, wl, 0, out, g, n);
            if (pout >= 0) {
                flux_s_pen(upw, &in_s, &gh, n, zp, zs, zp, zs, g);
                add_face(d, c, phi, wl, 0, pout, g, n);
            }
        }
    }
}

/* x = (w |J|)^{-1} Mhat^{-1} b for every component */
static void solve_into(const or_dg *d, int64_t c, int vel, const double *b, double *x) {
    int np = d->np, nco = vel ? 2 : 3;
    double w = (vel ? d->rho[c] : 1.0) * d->det[c];
    for (int comp = 0; comp < nco; comp++)
        for (int i = 0; i < np; i++) {
            double a = 0.0;
            for (int j = 0; j < np; j++) a += d->Minv[i * np + j] * b[IDX(d, comp, j, c)];
            x[comp * np + i] = a / w;
        }
}

static void kernel_solve(or_dg *d, int64_t c, int vel, int in, int out, int pin, int pout) {
    double x[45];
    int np = d->np, nco = vel ? 2 : 3;
    solve_into(d, c, vel, d->data[in], x);
    for (int comp = 0; comp < nco; comp++)
        for (int i = 0; i < np; i++) d->data[out][IDX(d, comp, i, c)] = x[comp * np + i];
    if (pin >= 0 && pout >= 0) {
        solve_into(d, c, vel, d->data[pin], x);
        for (int comp = 0; comp < nco; comp++)
            for (int i = 0; i < np; i++) d->data[pout][IDX(d, comp, i, c)] = x[comp * np + i];
    }
}

static void kernel_update(or_dg *d, int64_t c, int vel) {
    int np = d->np;
    double dt = d->dt, c3 = dt * dt * dt / 24.0;
    if (vel) {
        for (int comp = 0; comp < 2; comp++)
            for (int i = 0; i < np; i++) {
                int64_t id = IDX(d, comp, i, c);
                double u = d->data[D_U1][id];
                if (d->has_pen) u += d->data[D_PVS][id];
                d->data[D_V][id] += dt * u + c3 * d->data[D_U2][id];
            }
    } else {
        double r = (c == d->src_cell) ? or_ricker(d->t_half, d->src_f0, d->src_t0, d->src_amp) : 0.0;
        for (int comp = 0; comp < 3; comp++)
            for (int i = 0; i < np; i++) {
                int64_t id = IDX(d, comp, i, c);
                double u = d->data[D_V1][id];
                if (d->has_pen) u += d->data[D_PSS][id];
                double src = (comp < 2) ? r * d->src_vec[i] : 0.0;
                d->data[D_S][id] += dt * (u + src) + c3 * d->data[D_S2][id];
            }
    }
}

static void kernel_solupd(or_dg *d, int64_t c, int vel, int in, int pin) {
    int np = d->np, nco = vel ? 2 : 3;
    double x[45], p[45];
    solve_into(d, c, vel, d->data[in], x);
    if (pin >= 0) solve_into(d, c, vel, d->data[pin], p);
    double r = (!vel && c == d->src_cell) ? or_ricker(d->t_half, d->src_f0, d->src_t0, d->src_amp) : 0.0;
    for (int comp = 0; comp < nco; comp++)
        for (int i = 0; i < np; i++) {
            double u = x[comp * np + i] + (pin >= 0 ? p[comp * np + i] : 0.0);
            if (!vel && comp < 2) u += r * d->src_vec[i];
            d->data[vel ? D_V : D_S][IDX(d, comp, i, c)] += d->dt * u;
        }
}

/* run iteration `it` of loop j */
static void run_iteration(or_dg *d, int j, int64_t it) {
    const dg_loop *L = &d->loops[j];
    switch (L->kind) {
    case K_VOL_V: kernel_vol(d, it, 1, L->in, L->out, L->pout); break;
    case K_VOL_S: kernel_vol(d, it, 0, L->in, L->out, L->pout); break;
    case K_INT_V: kernel_int(d, it, 1, L->in, L->out, L->pin, L->pout); break;
    case K_INT_S: kernel_int(d, it, 0, L->in, L->out, L->pin, L->pout); break;
    case K_EXT_V: kernel_ext(d, it, 1, L->in, L->out, L->pin, L->pout); break;
    case K_EXT_S: kernel_ext(d, it, 0, L->in, L->out, L->pin, L->pout); break;
    case K_SOLVE_V: kernel_solve(d, it, 1, L->in, L->out, L->pin, L->pout); break;
    case K_SOLVE_S: kernel_solve(d, it, 0, L->in, L->out, L->pin, L->pout); break;
    case K_UPD_V: kernel_update(d, it, 1); break;
    case K_UPD_S: kernel_update(d, it, 0); break;
    case K_SOLUPD_V: kernel_solupd(d, it, 1, L->in, L->pin); break;
    case K_SOLUPD_S: kernel_solupd(d, it, 0, L->in, L->pin); break;
    }
}

static int64_t loop_size(const or_dg *d, int j) {
    int k = d->loops[j].kind;
    if (k == K_INT_V || k == K_INT_S) return d->nf;
    if (k == K_EXT_V || k == K_EXT_S) return d->nb;
    return d->nc;
}

static void load_state(or_dg *d, const double *v, const double *s) {
    memcpy(d->data[D_V], v, sizeof(double) * 2 * d->np * d->nc);
    memcpy(d->data[D_S], s, sizeof(double) * 3 * d->np * d->nc);
}

static void store_state(const or_dg *d, double *v, double *s) {
    memcpy(v, d->data[D_V], sizeof(double) * 2 * d->np * d->nc);
    memcpy(s, d->data[D_S], sizeof(double) * 3 * d->np * d->nc);
}

int or_dg_step(or_dg *d, double *v, double *s, int64_t nsteps, double t0) {
    load_state(d, v, s);
    for (int64_t n = 0; n < nsteps; n++) {
        d->t_half = t0 + ((double)n + 0.5) * d->dt;
        for (int j = 0; j < d->nloops; j++) {
            int64_t sz = loop_size(d, j);
            for (int64_t it = 0; it < sz; it++) run_iteration(d, j, it);
        }
    }
    store_state(d, v, s);
    return 0;
}

/* Tiled executor support (chain.c): run one iteration with explicit time. */
void or_dg_begin_step(or_dg *d, double t_half) { d->t_half = t_half; }
void or_dg_iteration(or_dg *d, int j, int64_t it) { run_iteration(d, j, it); }
int or_dg_nloops(const or_dg *d) { return d->nloops; }
void or_dg_load(or_dg *d, const double *v, const double *s) { load_state(d, v, s); }
void or_dg_store(const or_dg *d, double *v, double *s) { store_state(d, v, s); }
double or_dg_dt(const or_dg *d) { return d->dt; }

double or_dg_energy(const or_dg *d, const double *v, const double *s_new, const double *s_old) {
    int np = d->np;
    int64_t nc = d->nc;
    double e = 0.0;
    for (int64_t c = 0; c < nc; c++) {
        double l = d->lam[c], mu = d->mu[c], rho = d->rho[c];
        for (int q = 0; q < d->nq; q++) {
            const double *ph = d->qphi + q * np;
            double vv[2] = {0, 0}, a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            for (int j = 0; j < np; j++) {
                for (int comp = 0; comp < 2; comp++) vv[comp] += v[((int64_t)comp * np + j) * nc + c] * ph[j];
                for (int comp = 0; comp < 3; comp++) {
                    a[comp] += s_new[((int64_t)comp * np + j) * nc + c] * ph[j];
                    b[comp] += s_old[((int64_t)comp * np + j) * nc + c] * ph[j];
                }
            }
            double ke = rho * (vv[0] * vv[0] + vv[1] * vv[1]);
            double se = ((l + 2 * mu) * (a[0] * b[0] + a[1] * b[1]) - l * (a[0] * b[1] + a[1] * b[0])) /
                            (4.0 * mu * (l + mu)) + a[2] * b[2] / mu;
            e += 0.5 * d->qw[q] * d->det[c] * (ke + se);
        }
    }
    return e;
}

/* Rate operator for the brute-force time-order test: dv = A s + D_v v,
 * ds = B v + D_s s, using the same loops as the chain (first applications). */
int or_dg_rate(or_dg *d, const double *v, const double *s, double *dv, double *ds) {
    load_state(d, v, s);
    int np = d->np;
    int64_t nc = d->nc;
    for (int64_t c = 0; c < nc; c++) kernel_vol(d, c, 1, D_S, D_BV, -1);
    memset(d->data[D_PV], 0, sizeof(double) * 2 * np * nc);
    for (int64_t f = 0; f < d->nf; f++) kernel_int(d, f, 1, D_S, D_BV, D_V, D_PV);
    for (int64_t b = 0; b < d->nb; b++) kernel_ext(d, b, 1, D_S, D_BV, D_V, D_PV);
    for (int64_t c = 0; c < nc; c++) kernel_solve(d, c, 1, D_BV, D_U1, D_PV, D_PVS);
    for (int64_t c = 0; c < nc; c++) kernel_vol(d, c, 0, D_V, D_BS, -1);
    memset(d->data[D_PS], 0, sizeof(double) * 3 * np * nc);
    for (int64_t f = 0; f < d->nf; f++) kernel_int(d, f, 0, D_V, D_BS, D_S, D_PS);
    for (int64_t b = 0; b < d->nb; b++) kernel_ext(d, b, 0, D_V, D_BS, D_S, D_PS);
    for (int64_t c = 0; c < nc; c++) kernel_solve(d, c, 0, D_BS, D_V1, D_PS, D_PSS);
    for (int64_t i = 0; i < 2 * np * nc; i++) dv[i] = d->data[D_U1][i] + d->data[D_PVS][i];
    for (int64_t i = 0; i < 3 * np * nc; i++) ds[i] = d->data[D_V1][i] + d->data[D_PSS][i];
    return 0;
}

/* The chain as a generic loop chain: sets C=0, F=1, B=2; maps f2c=0, b2c=1.
 * Data-space ids are the D_* indices above. */
int or_dg_chain(const or_dg *d, or_chain **out) { return or_dg_chain_steps(d, 1, out); }

/* The chain of `steps` consecutive time steps: the step's loops repeated (a chain
 * fused over several steps, an extension of the paper's per-step loop chain). */
int or_dg_chain_steps(const or_dg *d, int steps, or_chain **out) {
    if (steps < 1 || steps * d->nloops > 64) return -1;
    or_chain *ch;
    or_chain_create(&ch);
    or_chain_set(ch, d->nc);
    or_chain_set(ch, d->nf);
    or_chain_set(ch, d->nb);
    or_chain_map(ch, 1, 0, 2, d->f2c);
    or_chain_map(ch, 2, 0, 1, d->b2c);
    for (int jj = 0; jj < steps * d->nloops; jj++) {
        const dg_loop *L = &d->loops[jj % d->nloops];
        int32_t maps[8], modes[8], data[8];
        int nd = 0;
#define ADD(m_, mo_, da_) do { maps[nd] = (m_); modes[nd] = (mo_); data[nd] = (da_); nd++; } while (0)
        int set = 0;
        switch (L->kind) {
        case K_VOL_V: case K_VOL_S:
            ADD(-1, OR_R, L->in); ADD(-1, OR_W, L->out);
            if (L->pout >= 0) ADD(-1, OR_W, L->pout);
            break;
        case K_INT_V: case K_INT_S:
            set = 1;
            ADD(0, OR_R, L->in); ADD(0, OR_INC, L->out);
            if (L->pout >= 0) { ADD(0, OR_R, L->pin); ADD(0, OR_INC, L->pout); }
            break;
        case K_EXT_V: case K_EXT_S:
            set = 2;
            ADD(1, OR_R, L->in); ADD(1, OR_INC, L->out);
            if (L->pout >= 0) { ADD(1, OR_R, L->pin); ADD(1, OR_INC, L->pout); }
            break;
        case K_SOLVE_V: case K_SOLVE_S:
            ADD(-1, OR_R, L->in); ADD(-1, OR_W, L->out);
            if (L->pout >= 0) { ADD(-1, OR_R, L->pin); ADD(-1, OR_W, L->pout); }
            break;
        case K_UPD_V:
            ADD(-1, OR_R, D_U1); ADD(-1, OR_R, D_U2);
            if (d->has_pen) ADD(-1, OR_R, D_PVS);
            ADD(-1, OR_R, D_V); ADD(-1, OR_W, D_V); break;
        case K_UPD_S:
            ADD(-1, OR_R, D_V1); ADD(-1, OR_R, D_S2);
            if (d->has_pen) ADD(-1, OR_R, D_PSS);
            ADD(-1, OR_R, D_S); ADD(-1, OR_W, D_S); break;
        case K_SOLUPD_V:
            ADD(-1, OR_R, L->in); if (L->pin >= 0) ADD(-1, OR_R, L->pin);
            ADD(-1, OR_R, D_V); ADD(-1, OR_W, D_V); break;
        case K_SOLUPD_S:
            ADD(-1, OR_R, L->in); if (L->pin >= 0) ADD(-1, OR_R, L->pin);
            ADD(-1, OR_R, D_S); ADD(-1, OR_W, D_S); break;
        }
#undef ADD
        or_chain_loop(ch, set, nd, maps, modes, data);
    }
    *out = ch;
    return 0;
}
