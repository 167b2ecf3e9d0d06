/*
 * mesh.c -- oracle facet maps (test infrastructure only).
 *
 * The loop chain of the DG step iterates over cells, interior facets and
 * exterior facets and reaches cells through maps (Sec. 2: sets, maps of arity
 * a; Sec. 7.3: cell, interior-facet and exterior-facet loops).  Canonical
 * numbering used by both sides of the parity tests (a convention, not the
 * paper's):
 *   - local facet l of a cell joins its vertices l and (l+1) mod 3;
 *   - interior facet list: cells c in ascending id, local facets l = 0,1,2, emit
 *     (c, l, c', l') whenever the neighbour c' across (c, l) has c' > c;
 *   - exterior facet list: cells ascending, l ascending, facets with no neighbour.
 * Periodic meshes pair boundary edges whose midpoints differ by the bounding
 * box period.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_mesh {
    int64_t nv, nc, nf, nb;
    double *xy;
    int32_t *c2v;
    int32_t *nbr;  /* [nc*3] neighbour cell or -1 */
    int8_t *nbrl;  /* [nc*3] neighbour's local facet */
    int32_t *f2c;
    int8_t *f2l;
    int32_t *b2c;
    int8_t *b2l;
    int8_t *bside;
    double bbox[4];
};

typedef struct {
    int32_t a, b, c, l;
} half_edge;

static int cmp_half(const void *x, const void *y) {
    const half_edge *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->c != q->c) return p->c < q->c ? -1 : 1;
    return p->l < q->l ? -1 : (p->l > q->l);
}

int or_mesh_build(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int periodic,
                  or_mesh **out) {
    *out = NULL;
    if (nv < 0 || nc < 0) return -1;
    for (int64_t i = 0; i < 3 * nc; i++)
        if (c2v[i] < 0 || c2v[i] >= nv) return -1;
    for (int64_t c = 0; c < nc; c++) {
        const double *p0 = xy + 2 * c2v[3 * c], *p1 = xy + 2 * c2v[3 * c + 1], *p2 = xy + 2 * c2v[3 * c + 2];
        double det = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]);
        if (!(det > 0)) return -1;
    }
    or_mesh *m = calloc(1, sizeof(*m));
    m->nv = nv;
    m->nc = nc;
    m->xy = malloc(sizeof(double) * 2 * (nv ? nv : 1));
    memcpy(m->xy, xy, sizeof(double) * 2 * nv);
    m->c2v = malloc(sizeof(int32_t) * 3 * (nc ? nc : 1));
    memcpy(m->c2v, c2v, sizeof(int32_t) * 3 * nc);
    m->nbr = malloc(sizeof(int32_t) * 3 * (nc ? nc : 1));
    m->nbrl = malloc(3 * (nc ? nc : 1));
    for (int64_t i = 0; i < 3 * nc; i++) {
        m->nbr[i] = -1;
        m->nbrl[i] = -1;
    }
    m->bbox[0] = m->bbox[2] = INFINITY;
    m->bbox[1] = m->bbox[3] = -INFINITY;
    for (int64_t v = 0; v < nv; v++) {
        if (xy[2 * v] < m->bbox[0]) m->bbox[0] = xy[2 * v];
        if (xy[2 * v] > m->bbox[1]) m->bbox[1] = xy[2 * v];
        if (xy[2 * v + 1] < m->bbox[2]) m->bbox[2] = xy[2 * v + 1];
        if (xy[2 * v + 1] > m->bbox[3]) m->bbox[3] = xy[2 * v + 1];
    }
    /* match half-edges by sorted vertex pair */
    half_edge *he = malloc(sizeof(half_edge) * 3 * (nc ? nc : 1));
    for (int64_t c = 0; c < nc; c++)
        for (int l = 0; l < 3; l++) {
            int32_t a = c2v[3 * c + l], b = c2v[3 * c + (l + 1) % 3];
            he[3 * c + l] = (half_edge){a < b ? a : b, a < b ? b : a, (int32_t)c, l};
        }
    qsort(he, 3 * nc, sizeof(half_edge), cmp_half);
    int bad = 0;
    for (int64_t i = 0; i < 3 * nc;) {
        int64_t j = i;
        while (j < 3 * nc && he[j].a == he[i].a && he[j].b == he[i].b) j++;
        if (j - i > 2) bad = 1;
        if (j - i == 2) {
            m->nbr[3 * he[i].c + he[i].l] = he[i + 1].c;
            m->nbrl[3 * he[i].c + he[i].l] = he[i + 1].l;
            m->nbr[3 * he[i + 1].c + he[i + 1].l] = he[i].c;
            m->nbrl[3 * he[i + 1].c + he[i + 1].l] = he[i].l;
        }
        i = j;
    }
    free(he);
    if (bad) {
        or_mesh_free(m);
        return -1;
    }
    double ext = fmax(m->bbox[1] - m->bbox[0], m->bbox[3] - m->bbox[2]);
    double tol = 1e-9 * (ext > 0 ? ext : 1.0);
    if (periodic) {
        /* plain O(n^2) pairing of unmatched boundary edges by translated midpoints */
        for (int dir = 0; dir < 2; dir++) {
            if (!(periodic & (1 << dir))) continue;
            double lo = m->bbox[2 * dir], hi = m->bbox[2 * dir + 1];
            for (int64_t c = 0; c < nc; c++)
                for (int l = 0; l < 3; l++) {
                    if (m->nbr[3 * c + l] >= 0) continue;
                    const double *pa = xy + 2 * c2v[3 * c + l], *pb = xy + 2 * c2v[3 * c + (l + 1) % 3];
                    if (fabs(pa[dir] - lo) > tol || fabs(pb[dir] - lo) > tol) continue;
                    double mid = 0.5 * (pa[1 - dir] + pb[1 - dir]);
                    for (int64_t c2 = 0; c2 < nc; c2++)
                        for (int l2 = 0; l2 < 3; l2++) {
                            if (m->nbr[3 * c2 + l2] >= 0) continue;
                            const double *qa = xy + 2 * c2v[3 * c2 + l2], *qb = xy + 2 * c2v[3 * c2 + (l2 + 1) % 3];
                            if (fabs(qa[dir] - hi) > tol || fabs(qb[dir] - hi) > tol) continue;
                            if (fabs(0.5 * (qa[1 - dir] + qb[1 - dir]) - mid) > tol) continue;
                            m->nbr[3 * c + l] = (int32_t)c2;
                            m->nbrl[3 * c + l] = (int8_t)l2;
                            m->nbr[3 * c2 + l2] = (int32_t)c;
                            m->nbrl[3 * c2 + l2] = (int8_t)l;
                        }
                }
        }
    }
    /* canonical facet lists */
    int64_t nf = 0, nb = 0;
    for (int64_t c = 0; c < nc; c++)
        for (int l = 0; l < 3; l++) {
            int32_t o = m->nbr[3 * c + l];
            if (o < 0) nb++;
            else if (o > c) nf++;
            else if (o == c) bad = 1;
        }
    if (bad) {
        or_mesh_free(m);
        return -1;
    }
    m->nf = nf;
    m->nb = nb;
    m->f2c = malloc(sizeof(int32_t) * 2 * (nf ? nf : 1));
    m->f2l = malloc(2 * (nf ? nf : 1));
    m->b2c = malloc(sizeof(int32_t) * (nb ? nb : 1));
    m->b2l = malloc(nb ? nb : 1);
    m->bside = malloc(nb ? nb : 1);
    int64_t f = 0, b = 0;
    for (int64_t c = 0; c < nc; c++)
        for (int l = 0; l < 3; l++) {
            int32_t o = m->nbr[3 * c + l];
            if (o < 0) {
                m->b2c[b] = (int32_t)c;
                m->b2l[b] = (int8_t)l;
                const double *pa = xy + 2 * c2v[3 * c + l], *pb = xy + 2 * c2v[3 * c + (l + 1) % 3];
                double mx = 0.5 * (pa[0] + pb[0]), my = 0.5 * (pa[1] + pb[1]);
                int side = -1;
                if (fabs(mx - m->bbox[0]) <= tol) side = 0;
                else if (fabs(mx - m->bbox[1]) <= tol) side = 1;
                else if (fabs(my - m->bbox[2]) <= tol) side = 2;
                else if (fabs(my - m->bbox[3]) <= tol) side = 3;
                m->bside[b] = (int8_t)side;
                b++;
            } else if (o > c) {
                m->f2c[2 * f] = (int32_t)c;
                m->f2l[2 * f] = (int8_t)l;
                m->f2c[2 * f + 1] = o;
                m->f2l[2 * f + 1] = m->nbrl[3 * c + l];
                f++;
            }
        }
    *out = m;
    return 0;
}

void or_mesh_free(or_mesh *m) {
    if (!m) return;
    free(m->xy);
    free(m->c2v);
    free(m->nbr);
    free(m->nbrl);
    free(m->f2c);
    free(m->f2l);
    free(m->b2c);
    free(m->b2l);
    free(m->bside);
    free(m);
}

void or_mesh_counts(const or_mesh *m, int64_t *nc, int64_t *nf, int64_t *nb) {
    if (nc) *nc = m->nc;
    if (nf) *nf = m->nf;
    if (nb) *nb = m->nb;
}

void or_mesh_maps(const or_mesh *m, int32_t *f2c, int8_t *f2l, int32_t *b2c, int8_t *b2l, int8_t *bside) {
    if (f2c) memcpy(f2c, m->f2c, sizeof(int32_t) * 2 * m->nf);
    if (f2l) memcpy(f2l, m->f2l, 2 * m->nf);
    if (b2c) memcpy(b2c, m->b2c, sizeof(int32_t) * m->nb);
    if (b2l) memcpy(b2l, m->b2l, m->nb);
    if (bside) memcpy(bside, m->bside, m->nb);
}

/* accessors for dg.c */
const double *or_mesh_xy(const or_mesh *m) { return m->xy; }
const int32_t *or_mesh_c2v(const or_mesh *m) { return m->c2v; }
const int32_t *or_mesh_f2c(const or_mesh *m) { return m->f2c; }
const int8_t *or_mesh_f2l(const or_mesh *m) { return m->f2l; }
const int32_t *or_mesh_b2c(const or_mesh *m) { return m->b2c; }
const int8_t *or_mesh_b2l(const or_mesh *m) { return m->b2l; }
const int8_t *or_mesh_bside(const or_mesh *m) { return m->bside; }
