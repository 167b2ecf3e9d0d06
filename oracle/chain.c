/*
 * chain.c -- oracle loop chain, sparse-tiling inspector, dependence checker and
 * tiled executor (test infrastructure only).
 *
 * Loop chain (Sec. 2): iteration sets, maps M: S_i -> S_j^a, loops over a set
 * with descriptors <M or direct, mode in {r, w, i}>.  Dependences are tracked
 * per set, not per data space.
 *
 * Inspector (Alg. 1): partition the seed loop into blocks of ts iterations,
 * colour the tiles, then for every later loop project the previous loop's
 * tiling function onto the sets it touches (Alg. 3) and tile the loop from
 * the projections (Alg. 4); repeat with fake connections while two tiles of one
 * colour conflict.  Readings of passages the paper leaves open:
 *   R1 (projection start)  a projection starts from the previous projection of
 *       the same set when one exists and is raised with MAX; it is never reset
 *       to bottom, so a loop touching part of a set keeps the constraints on the
 *       rest.  Every descriptor is projected, whatever its mode.
 *   R2 (tiling start)      sigma_j starts at bottom once; MAX runs over every
 *       descriptor and every arity slot.
 *   R3 (MAX order)         tiles compare by the packed key (colour+1)<<32 | id,
 *       so the maximum is unique; bottom is key 0.  An iteration left at bottom
 *       goes to the first tile of colour 0.
 *   R4 (projections per round)  Phi is emptied at the start of every conflict
 *       round, since colours change between rounds.
 *   R5 (colouring)         deterministic Jones-Plassmann: priority
 *       (fmix32(t), t) with fmix32 the MurmurHash3 finaliser; each round every
 *       uncoloured tile that beats all its uncoloured neighbours takes the
 *       smallest colour unused by its coloured neighbours.
 *   R6 (tile adjacency)    tiles t(x), t(y) of seed iterations x, y are
 *       adjacent when a map from the seed set sends x and y to a common element,
 *       or a map into the seed set sends one element to both; plus fake edges.
 *   R7 (conflicts)         two different tiles of the same colour that touch a
 *       common element of any set, in any loops of the chain, through any
 *       descriptor, conflict; each conflicting pair becomes a fake edge and the
 *       colouring restarts from scratch.
 *   R8 (seed order)        partition 1 sorts seed iterations by the Hilbert
 *       index of their quantised coordinates (2^16 per axis), ties by id.
 *   R9 (lists)             iteration lists and footprints are sorted by id.
 *   R10 (regions, Sec. 3.3 and 5.1.2)  with seed regions (core 0, boundary 1,
 *       non-exec 2) the seeds of each region are taken in seed order and cut into
 *       blocks of ts: core tiles first, then boundary tiles, then one tile T_ne
 *       holding every non-exec seed.  A GPU runs the tiles of one colour in
 *       parallel, so each region is coloured by Jones-Plassmann (R5) on the tile
 *       graph restricted to its own tiles; boundary colours follow all core
 *       colours and T_ne takes the highest colour alone.  T_ne is never
 *       executed; anything touching its data joins it through the MAX of
 *       Alg. 3/4.  The colour-class cap (R5b) is not combined with regions.
 *   R11 (one exchange per chain)  with carry set, the halo is exchanged once
 *       before the first sub-chain only: every later sub-chain treats as
 *       non-exec, besides the given non-exec seeds, every seed element that a
 *       T_ne iteration of an earlier sub-chain wrote (its value is stale).  This
 *       needs every write of the chain to land in the seed set.  Without carry,
 *       every sub-chain starts from the given regions (the paper's case: each
 *       loop chain exchanges its own halo).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXSETS 8
#define MAXMAPS 8
#define MAXLOOPS 64
#define MAXDESC 8

typedef struct {
    int map, mode, data;
} desc_t;

typedef struct {
    int set, ndesc;
    desc_t d[MAXDESC];
} loop_t;

typedef struct {
    int from, to, arity;
    int32_t *values;
} map_t;

struct or_chain {
    int nsets, nmaps, nloops;
    int64_t size[MAXSETS];
    map_t maps[MAXMAPS];
    loop_t loops[MAXLOOPS];
};

typedef struct {
    int first, n;       /* loop range */
    int ntiles, ncolors, rounds;
    int32_t *color;     /* [ntiles] */
    int64_t foot_len[MAXSETS];
    int32_t *foot_off[MAXSETS], *foot[MAXSETS];
    uint32_t *acc[MAXSETS];
    /* regions (Sec. 3.3): core tiles [0, ncore), boundary tiles [ncore,
     * ncore + nbnd), the non-exec tile tne = ncore + nbnd; region[] holds the
     * seed regions this sub-chain was inspected with (NULL: no regions) */
    int32_t ncore, nbnd, tne;
    uint8_t *region;
} sub_t;

struct or_sched {
    int nsub;
    sub_t sub[MAXLOOPS];
    int nloops;
    int32_t *sigma[MAXLOOPS]; /* tile per iteration */
    int64_t loop_size[MAXLOOPS];
    int sub_of[MAXLOOPS];
};

int or_chain_create(or_chain **out) {
    *out = calloc(1, sizeof(or_chain));
    return 0;
}

void or_chain_free(or_chain *c) {
    if (!c) return;
    for (int i = 0; i < c->nmaps; i++) free(c->maps[i].values);
    free(c);
}

int or_chain_set(or_chain *c, int64_t size) {
    if (c->nsets >= MAXSETS || size < 0) return -1;
    c->size[c->nsets] = size;
    return c->nsets++;
}

int or_chain_map(or_chain *c, int from, int to, int arity, const int32_t *values) {
    if (c->nmaps >= MAXMAPS || from < 0 || from >= c->nsets || to < 0 || to >= c->nsets || arity < 1) return -1;
    int64_t n = c->size[from] * arity;
    for (int64_t i = 0; i < n; i++)
        if (values[i] < 0 || values[i] >= c->size[to]) return -1;
    map_t *m = &c->maps[c->nmaps];
    m->from = from;
    m->to = to;
    m->arity = arity;
    m->values = malloc(sizeof(int32_t) * (n ? n : 1));
    memcpy(m->values, values, sizeof(int32_t) * n);
    return c->nmaps++;
}

int or_chain_loop(or_chain *c, int set, int ndesc, const int32_t *maps, const int32_t *modes, const int32_t *data) {
    if (c->nloops >= MAXLOOPS || set < 0 || set >= c->nsets || ndesc < 0 || ndesc > MAXDESC) return -1;
    loop_t *L = &c->loops[c->nloops];
    L->set = set;
    L->ndesc = ndesc;
    for (int i = 0; i < ndesc; i++) {
        if (maps[i] >= c->nmaps || maps[i] < -1) return -1;
        if (maps[i] >= 0 && c->maps[maps[i]].from != set) return -1;
        if (modes[i] < 0 || modes[i] > 2) return -1;
        L->d[i].map = maps[i];
        L->d[i].mode = modes[i];
        L->d[i].data = data ? data[i] : -1;
    }
    return c->nloops++;
}

int or_chain_nloops(const or_chain *c) { return c->nloops; }

int64_t or_chain_set_size(const or_chain *c, int set) { return set < 0 || set >= c->nsets ? -1 : c->size[set]; }

int or_chain_get_loop(const or_chain *c, int j, int32_t *set, int32_t *ndesc, int32_t *maps, int32_t *modes) {
    if (j < 0 || j >= c->nloops) return -1;
    *set = c->loops[j].set;
    *ndesc = c->loops[j].ndesc;
    for (int i = 0; i < c->loops[j].ndesc; i++) {
        maps[i] = c->loops[j].d[i].map;
        modes[i] = c->loops[j].d[i].mode;
    }
    return 0;
}

int or_chain_get_map(const or_chain *c, int m, int32_t *from, int32_t *to, int32_t *arity, int32_t *values) {
    if (m < 0 || m >= c->nmaps) return -1;
    *from = c->maps[m].from;
    *to = c->maps[m].to;
    *arity = c->maps[m].arity;
    if (values) memcpy(values, c->maps[m].values, sizeof(int32_t) * c->size[c->maps[m].from] * c->maps[m].arity);
    return 0;
}

/* target set of a descriptor */
static int dset(const or_chain *c, const loop_t *L, const desc_t *D) {
    return D->map < 0 ? L->set : c->maps[D->map].to;
}

/* ---------------------------------------------------------------- helpers */

static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* Hilbert index of (x, y) on a 2^16 x 2^16 grid (the classic rotate-and-flip
 * construction: at each level pick the quadrant, then rotate/reflect the
 * coordinates inside it). */
static uint64_t hilbert_d(uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        x &= s - 1;
        y &= s - 1;
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y);
}

static uint64_t key_of(const int32_t *color, int32_t t) { return ((uint64_t)(uint32_t)(color[t] + 1) << 32) | (uint32_t)t; }

/* CSR inverse of a map (Fig. 8): for each target element, the source iterations
 * touching it, ascending. */
typedef struct {
    int32_t *off, *val;
} inv_t;

static inv_t invert_map(const or_chain *c, const map_t *m) {
    inv_t r;
    int64_t nt = c->size[m->to], ns = c->size[m->from];
    r.off = calloc(nt + 1, sizeof(int32_t));
    r.val = malloc(sizeof(int32_t) * (ns * m->arity + 1));
    for (int64_t i = 0; i < ns * m->arity; i++) r.off[m->values[i] + 1]++;
    for (int64_t e = 0; e < nt; e++) r.off[e + 1] += r.off[e];
    int32_t *pos = malloc(sizeof(int32_t) * (nt + 1));
    memcpy(pos, r.off, sizeof(int32_t) * (nt + 1));
    for (int64_t i = 0; i < ns; i++)
        for (int k = 0; k < m->arity; k++) r.val[pos[m->values[i * m->arity + k]]++] = (int32_t)i;
    free(pos);
    return r;
}

/* --------------------------------------------------------------- colouring */

typedef struct {
    int64_t n;
    uint64_t *e; /* sorted unique (a<<32|b), a<b */
} edges_t;

static void edges_add_sorted_unique(edges_t *E) {
    if (E->n == 0) return;
    qsort(E->e, E->n, sizeof(uint64_t), cmp_u64);
    int64_t w = 1;
    for (int64_t i = 1; i < E->n; i++)
        if (E->e[i] != E->e[w - 1]) E->e[w++] = E->e[i];
    E->n = w;
}

/* Colour-class cap (R5b, used when cap > 0): one pass over the tiles in
 * ascending id; a tile whose colour class holds more than cap tiles moves to the
 * smallest colour that holds fewer than cap tiles and that no neighbour has, or
 * to a new colour.  Afterwards every class holds at most cap tiles and the
 * colouring is still proper.  Returns the new number of colours, or -1 past 64. */
static int cap_colour_classes(int ntiles, const int32_t *deg, const int32_t *adj, int32_t *color, int ncol,
                              int cap) {
    int32_t size[64] = {0};
    for (int t = 0; t < ntiles; t++) size[color[t]]++;
    for (int t = 0; t < ntiles; t++) {
        int c = color[t];
        if (size[c] <= cap) continue;
        uint64_t used = 0;
        for (int32_t k = deg[t]; k < deg[t + 1]; k++) used |= 1ull << color[adj[k]];
        int c2 = 0;
        while (c2 < ncol && (c2 == c || size[c2] >= cap || ((used >> c2) & 1))) c2++;
        if (c2 == ncol) {
            if (ncol >= 64) return -1;
            ncol++;
        }
        color[t] = c2;
        size[c]--;
        size[c2]++;
    }
    return ncol;
}

/* Jones-Plassmann colouring (R5), then the class cap (R5b); returns ncolors or -1 */
static int colour_tiles(int ntiles, const edges_t *E, int32_t *color, int cap) {
    /* symmetric adjacency CSR */
    int32_t *deg = calloc(ntiles + 1, sizeof(int32_t));
    for (int64_t i = 0; i < E->n; i++) {
        deg[(int32_t)(E->e[i] >> 32) + 1]++;
        deg[(int32_t)(E->e[i] & 0xffffffffu) + 1]++;
    }
    for (int t = 0; t < ntiles; t++) deg[t + 1] += deg[t];
    int32_t *adj = malloc(sizeof(int32_t) * (2 * E->n + 1));
    int32_t *pos = malloc(sizeof(int32_t) * (ntiles + 1));
    memcpy(pos, deg, sizeof(int32_t) * (ntiles + 1));
    for (int64_t i = 0; i < E->n; i++) {
        int32_t a = (int32_t)(E->e[i] >> 32), b = (int32_t)(E->e[i] & 0xffffffffu);
        adj[pos[a]++] = b;
        adj[pos[b]++] = a;
    }
    free(pos);
    for (int t = 0; t < ntiles; t++) color[t] = -1;
    char *mark = malloc(ntiles + 1);
    int remaining = ntiles, ncol = 0;
    while (remaining > 0) {
        for (int t = 0; t < ntiles; t++) {
            mark[t] = 0;
            if (color[t] >= 0) continue;
            uint64_t pt = ((uint64_t)fmix32((uint32_t)t) << 32) | (uint32_t)t;
            int best = 1;
            for (int32_t k = deg[t]; k < deg[t + 1]; k++) {
                int32_t u = adj[k];
                if (color[u] >= 0) continue;
                uint64_t pu = ((uint64_t)fmix32((uint32_t)u) << 32) | (uint32_t)u;
                if (pu > pt) { best = 0; break; }
            }
            mark[t] = (char)best;
        }
        for (int t = 0; t < ntiles; t++) {
            if (!mark[t]) continue;
            uint64_t used = 0;
            for (int32_t k = deg[t]; k < deg[t + 1]; k++) {
                int32_t u = adj[k];
                if (color[u] >= 0 && !mark[u]) {
                    if (color[u] >= 64) { free(deg); free(adj); free(mark); return -1; }
                    used |= 1ull << color[u];
                }
            }
            int col = 0;
            while (col < 64 && (used >> col) & 1) col++;
            if (col >= 64) { free(deg); free(adj); free(mark); return -1; }
            color[t] = col;
            if (col + 1 > ncol) ncol = col + 1;
            remaining--;
        }
    }
    if (cap > 0) ncol = cap_colour_classes(ntiles, deg, adj, color, ncol, cap);
    free(deg);
    free(adj);
    free(mark);
    return ncol;
}

/* ---------------------------------------------------------------- inspector */

static int seed_ranks(int64_t n, int partition, const double *xy, int32_t *rank) {
    if (partition == 0 || n == 0) {
        for (int64_t i = 0; i < n; i++) rank[i] = (int32_t)i;
        return 0;
    }
    if (!xy) return -1;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 2; a++) {
            if (xy[2 * i + a] < lo[a]) lo[a] = xy[2 * i + a];
            if (xy[2 * i + a] > hi[a]) hi[a] = xy[2 * i + a];
        }
    uint64_t *key = malloc(sizeof(uint64_t) * n);
    for (int64_t i = 0; i < n; i++) {
        uint32_t q[2];
        for (int a = 0; a < 2; a++) {
            double ext = hi[a] - lo[a];
            double v = ext > 0.0 ? floor((xy[2 * i + a] - lo[a]) / ext * 65536.0) : 0.0;
            q[a] = v >= 65535.0 ? 65535u : (uint32_t)v;
        }
        key[i] = (hilbert_d(q[0], q[1]) << 32) | (uint64_t)i;
    }
    qsort(key, n, sizeof(uint64_t), cmp_u64);
    for (int64_t p = 0; p < n; p++) rank[key[p] & 0xffffffffu] = (int32_t)p;
    free(key);
    return 0;
}

/* tile adjacency through the maps touching the seed set (R6) */
static void seed_adjacency(const or_chain *c, int first, int nl, const int32_t *tile0, edges_t *E) {
    int seed = c->loops[first].set;
    int used[MAXMAPS] = {0};
    for (int j = first; j < first + nl; j++)
        for (int i = 0; i < c->loops[j].ndesc; i++)
            if (c->loops[j].d[i].map >= 0) used[c->loops[j].d[i].map] = 1;
    int64_t cap = 16, n = 0;
    uint64_t *e = malloc(sizeof(uint64_t) * cap);
#define PUSH(a_, b_) do { int32_t A_ = (a_), B_ = (b_); if (A_ != B_) { if (A_ > B_) { int32_t T_ = A_; A_ = B_; B_ = T_; } \
        if (n == cap) { cap *= 2; e = realloc(e, sizeof(uint64_t) * cap); } e[n++] = ((uint64_t)A_ << 32) | (uint32_t)B_; } } while (0)
    for (int mi = 0; mi < c->nmaps; mi++) {
        if (!used[mi]) continue;
        const map_t *m = &c->maps[mi];
        if (m->from == seed) {
            inv_t inv = invert_map(c, m);
            for (int64_t x = 0; x < c->size[m->to]; x++)
                for (int32_t a = inv.off[x]; a < inv.off[x + 1]; a++)
                    for (int32_t b = a + 1; b < inv.off[x + 1]; b++) PUSH(tile0[inv.val[a]], tile0[inv.val[b]]);
            free(inv.off);
            free(inv.val);
        }
        if (m->to == seed) {
            for (int64_t s = 0; s < c->size[m->from]; s++)
                for (int a = 0; a < m->arity; a++)
                    for (int b = a + 1; b < m->arity; b++)
                        PUSH(tile0[m->values[s * m->arity + a]], tile0[m->values[s * m->arity + b]]);
        }
    }
#undef PUSH
    E->e = e;
    E->n = n;
    edges_add_sorted_unique(E);
}

/* (element, tile) pairs of one set for the sub-chain, with loop bits */
typedef struct {
    uint64_t key; /* element<<32 | tile */
    uint32_t bits;
} touch_t;

static int cmp_touch(const void *a, const void *b) {
    const touch_t *x = a, *y = b;
    return x->key < y->key ? -1 : (x->key > y->key);
}

static int64_t collect_touches(const or_chain *c, const or_sched *s, int first, int nl, int set, touch_t **out) {
    int64_t n = 0;
    for (int j = first; j < first + nl; j++) {
        const loop_t *L = &c->loops[j];
        for (int i = 0; i < L->ndesc; i++)
            if (dset(c, L, &L->d[i]) == set)
                n += c->size[L->set] * (L->d[i].map < 0 ? 1 : c->maps[L->d[i].map].arity);
    }
    touch_t *t = malloc(sizeof(touch_t) * (n ? n : 1));
    int64_t w = 0;
    for (int j = first; j < first + nl; j++) {
        const loop_t *L = &c->loops[j];
        for (int i = 0; i < L->ndesc; i++) {
            const desc_t *D = &L->d[i];
            if (dset(c, L, D) != set) continue;
            for (int64_t it = 0; it < c->size[L->set]; it++) {
                uint32_t tile = (uint32_t)s->sigma[j][it];
                if (D->map < 0) {
                    t[w].key = ((uint64_t)it << 32) | tile;
                    t[w++].bits = 1u << (j - first);
                } else {
                    const map_t *m = &c->maps[D->map];
                    for (int k = 0; k < m->arity; k++) {
                        t[w].key = ((uint64_t)(uint32_t)m->values[it * m->arity + k] << 32) | tile;
                        t[w++].bits = 1u << (j - first);
                    }
                }
            }
        }
    }
    qsort(t, w, sizeof(touch_t), cmp_touch);
    /* merge equal keys, OR-ing loop bits */
    int64_t u = 0;
    for (int64_t i = 0; i < w; i++) {
        if (u > 0 && t[u - 1].key == t[i].key) t[u - 1].bits |= t[i].bits;
        else t[u++] = t[i];
    }
    *out = t;
    return u;
}

/* When set (negative tests only), Alg. 3 is read literally: every indirect
 * projection restarts from bottom instead of from the previous projection. */
static int g_literal_projection = 0;
void or_set_literal_projection(int on) { g_literal_projection = on; }

/* Alg. 3 (projection of loop j) with reading R1 */
static void project(const or_chain *c, int j, const int32_t *sigma, const int32_t *color, uint64_t **Phi) {
    const loop_t *L = &c->loops[j];
    for (int i = 0; i < L->ndesc; i++) {
        const desc_t *D = &L->d[i];
        int S = dset(c, L, D);
        int64_t nS = c->size[S];
        uint64_t *phi = malloc(sizeof(uint64_t) * (nS ? nS : 1));
        int restart = g_literal_projection && D->map >= 0;
        for (int64_t e = 0; e < nS; e++) phi[e] = (Phi[S] && !restart) ? Phi[S][e] : 0;
        if (D->map < 0) {
            for (int64_t e = 0; e < nS; e++) {
                uint64_t k = key_of(color, sigma[e]);
                if (k > phi[e]) phi[e] = k;
            }
        } else {
            inv_t inv = invert_map(c, &c->maps[D->map]);
            for (int64_t e = 0; e < nS; e++)
                for (int32_t a = inv.off[e]; a < inv.off[e + 1]; a++) {
                    uint64_t k = key_of(color, sigma[inv.val[a]]);
                    if (k > phi[e]) phi[e] = k;
                }
            free(inv.off);
            free(inv.val);
        }
        free(Phi[S]);
        Phi[S] = phi;
    }
}

/* Alg. 4 (tiling function of loop j) with readings R2, R3 */
static void tile_loop(const or_chain *c, int j, uint64_t **Phi, const int32_t *color, int ntiles, int32_t *sigma) {
    const loop_t *L = &c->loops[j];
    int64_t n = c->size[L->set];
    /* default tile for unconstrained iterations: first tile of colour 0 */
    int32_t deft = 0;
    for (int t = 0; t < ntiles; t++)
        if (color[t] == 0) { deft = t; break; }
    for (int64_t e = 0; e < n; e++) {
        uint64_t best = 0;
        for (int i = 0; i < L->ndesc; i++) {
            const desc_t *D = &L->d[i];
            int S = dset(c, L, D);
            if (!Phi[S]) continue;
            if (D->map < 0) {
                if (Phi[S][e] > best) best = Phi[S][e];
            } else {
                const map_t *m = &c->maps[D->map];
                for (int k = 0; k < m->arity; k++) {
                    uint64_t v = Phi[S][m->values[e * m->arity + k]];
                    if (v > best) best = v;
                }
            }
        }
        sigma[e] = best ? (int32_t)(best & 0xffffffffu) : deft;
    }
}

/* conflicts (R7): same-colour different tiles touching one element */
static int64_t find_conflicts(const or_chain *c, const or_sched *s, int first, int nl, const int32_t *color,
                              edges_t *out) {
    int64_t cap = 16, n = 0;
    uint64_t *e = malloc(sizeof(uint64_t) * cap);
    for (int S = 0; S < c->nsets; S++) {
        touch_t *t;
        int64_t m = collect_touches(c, s, first, nl, S, &t);
        for (int64_t a = 0; a < m;) {
            int64_t b = a;
            while (b < m && (t[b].key >> 32) == (t[a].key >> 32)) b++;
            for (int64_t x = a; x < b; x++)
                for (int64_t y = x + 1; y < b; y++) {
                    int32_t tx = (int32_t)(t[x].key & 0xffffffffu), ty = (int32_t)(t[y].key & 0xffffffffu);
                    if (tx != ty && color[tx] == color[ty]) {
                        if (n == cap) { cap *= 2; e = realloc(e, sizeof(uint64_t) * cap); }
                        e[n++] = ((uint64_t)(tx < ty ? tx : ty) << 32) | (uint32_t)(tx < ty ? ty : tx);
                    }
                }
            a = b;
        }
        free(t);
    }
    out->e = e;
    out->n = n;
    edges_add_sorted_unique(out);
    return out->n;
}

/* One pass of the inner loop of Alg. 1 with a given seed tiling and given tile
 * colours (no colouring, no conflict handling): sigma[j] for every loop. */
int or_tile_with_colors(const or_chain *c, const int32_t *tile0, int ntiles, const int32_t *color,
                        int32_t **sigma) {
    uint64_t *Phi[MAXSETS] = {0};
    memcpy(sigma[0], tile0, sizeof(int32_t) * c->size[c->loops[0].set]);
    for (int j = 1; j < c->nloops; j++) {
        project(c, j - 1, sigma[j - 1], color, Phi);
        tile_loop(c, j, Phi, color, ntiles, sigma[j]);
    }
    for (int S = 0; S < MAXSETS; S++) free(Phi[S]);
    return 0;
}

/* Projection of one set after the first `upto` loops (for the worked example). */
int or_projection_after(const or_chain *c, const int32_t *tile0, int ntiles, const int32_t *color, int upto,
                        int set, int32_t *phi_tile) {
    uint64_t *Phi[MAXSETS] = {0};
    int32_t *sig[MAXLOOPS] = {0};
    for (int j = 0; j < c->nloops; j++) sig[j] = malloc(sizeof(int32_t) * (c->size[c->loops[j].set] + 1));
    memcpy(sig[0], tile0, sizeof(int32_t) * c->size[c->loops[0].set]);
    for (int j = 1; j <= upto && j <= c->nloops; j++) {
        project(c, j - 1, sig[j - 1], color, Phi);
        if (j < c->nloops) tile_loop(c, j, Phi, color, ntiles, sig[j]);
    }
    for (int64_t e = 0; e < c->size[set]; e++)
        phi_tile[e] = (Phi[set] && Phi[set][e]) ? (int32_t)(Phi[set][e] & 0xffffffffu) : -1;
    for (int S = 0; S < MAXSETS; S++) free(Phi[S]);
    for (int j = 0; j < c->nloops; j++) free(sig[j]);
    return 0;
}

/* Region-aware colouring (R10): Jones-Plassmann on the edges joining tiles of
 * one region, then boundary colours shifted past the core ones and T_ne alone
 * in the highest colour.  Returns the number of colours or -1. */
static int colour_regions(int ntiles, const edges_t *E, const uint8_t *treg, int32_t *color) {
    edges_t F;
    F.e = malloc(sizeof(uint64_t) * (E->n + 1));
    F.n = 0;
    for (int64_t i = 0; i < E->n; i++) {
        int32_t a = (int32_t)(E->e[i] >> 32), b = (int32_t)(E->e[i] & 0xffffffffu);
        if (treg[a] == treg[b]) F.e[F.n++] = E->e[i];
    }
    int ncol = colour_tiles(ntiles, &F, color, 0);
    free(F.e);
    if (ncol < 0) return -1;
    int ccore = 0, cbnd = 0; /* colours used by core and by boundary tiles */
    for (int t = 0; t < ntiles; t++) {
        if (treg[t] == 0 && color[t] + 1 > ccore) ccore = color[t] + 1;
        if (treg[t] == 1 && color[t] + 1 > cbnd) cbnd = color[t] + 1;
    }
    for (int t = 0; t < ntiles; t++) {
        if (treg[t] == 1) color[t] += ccore;
        if (treg[t] == 2) color[t] = ccore + cbnd;
    }
    return ccore + cbnd + 1 > 64 ? -1 : ccore + cbnd + 1;
}

static int inspect_sub(const or_chain *c, or_sched *s, sub_t *sb, int64_t ts, int partition, const double *seed_xy,
                       int max_rounds,
                       int cap, const uint8_t *region) {
    int first = sb->first, nl = sb->n;
    int seedset = c->loops[first].set;
    int64_t n0 = c->size[seedset];
    int ntiles = (int)((n0 + ts - 1) / ts);
    if (ntiles == 0) ntiles = 1; /* empty seed set: one (empty) tile */
    int32_t *rank = malloc(sizeof(int32_t) * (n0 ? n0 : 1));
    if (seed_ranks(n0, partition, seed_xy, rank)) { free(rank); return -1; }
    int32_t *tile0 = malloc(sizeof(int32_t) * (n0 ? n0 : 1));
    uint8_t *treg = NULL;
    if (!region) {
        for (int64_t i = 0; i < n0; i++) tile0[i] = (int32_t)(rank[i] / ts);
    } else {
        /* R10: blocks of ts seeds per region in seed order, then T_ne */
        int64_t cnt[3] = {0, 0, 0};
        for (int64_t i = 0; i < n0; i++) cnt[region[i]]++;
        int32_t ncore = (int32_t)((cnt[0] + ts - 1) / ts), nbnd = (int32_t)((cnt[1] + ts - 1) / ts);
        ntiles = ncore + nbnd + 1;
        int32_t *order = malloc(sizeof(int32_t) * (n0 ? n0 : 1));
        for (int64_t i = 0; i < n0; i++) order[rank[i]] = (int32_t)i;
        int64_t q[2] = {0, 0};
        for (int64_t p = 0; p < n0; p++) {
            int32_t i = order[p];
            int r = region[i];
            if (r == 2) tile0[i] = ncore + nbnd;
            else tile0[i] = (r == 0 ? 0 : ncore) + (int32_t)(q[r]++ / ts);
        }
        free(order);
        treg = malloc((size_t)ntiles);
        for (int t = 0; t < ntiles; t++) treg[t] = t < ncore ? 0 : (t < ncore + nbnd ? 1 : 2);
        sb->ncore = ncore;
        sb->nbnd = nbnd;
        sb->tne = ncore + nbnd;
        sb->region = malloc((size_t)(n0 ? n0 : 1));
        memcpy(sb->region, region, (size_t)n0);
    }
    free(rank);
    edges_t adj;
    seed_adjacency(c, first, nl, tile0, &adj);
    int32_t *color = malloc(sizeof(int32_t) * ntiles);
    int round, ncol = 0;
    for (round = 0; round < max_rounds; round++) {
        ncol = treg ? colour_regions(ntiles, &adj, treg, color) : colour_tiles(ntiles, &adj, color, cap);
        if (ncol < 0) { free(tile0); free(color); free(adj.e); free(treg); return -3; }
        uint64_t *Phi[MAXSETS] = {0};
        memcpy(s->sigma[first], tile0, sizeof(int32_t) * n0);
        for (int j = first + 1; j < first + nl; j++) {
            project(c, j - 1, s->sigma[j - 1], color, Phi);
            tile_loop(c, j, Phi, color, ntiles, s->sigma[j]);
        }
        for (int S = 0; S < MAXSETS; S++) free(Phi[S]);
        edges_t conf;
        int64_t nconf = find_conflicts(c, s, first, nl, color, &conf);
        if (nconf == 0) { free(conf.e); break; }
        /* add fake connections and start over */
        adj.e = realloc(adj.e, sizeof(uint64_t) * (adj.n + conf.n + 1));
        memcpy(adj.e + adj.n, conf.e, sizeof(uint64_t) * conf.n);
        adj.n += conf.n;
        edges_add_sorted_unique(&adj);
        free(conf.e);
    }
    free(tile0);
    free(adj.e);
    free(treg);
    if (round == max_rounds) { free(color); return -4; }
    sb->ntiles = ntiles;
    sb->ncolors = ncol;
    sb->rounds = round + 1;
    sb->color = color;
    /* footprints per set (local maps on the executor side derive from these) */
    for (int S = 0; S < c->nsets; S++) {
        touch_t *t;
        int64_t m = collect_touches(c, s, first, nl, S, &t);
        /* single-tile flag per element */
        for (int64_t a = 0; a < m;) {
            int64_t b = a;
            while (b < m && (t[b].key >> 32) == (t[a].key >> 32)) b++;
            if (b - a == 1) t[a].bits |= 1u << 31;
            a = b;
        }
        /* re-key by (tile, element) */
        for (int64_t i = 0; i < m; i++) {
            uint64_t el = t[i].key >> 32, tl = t[i].key & 0xffffffffu;
            t[i].key = (tl << 32) | el;
        }
        qsort(t, m, sizeof(touch_t), cmp_touch);
        sb->foot_len[S] = m;
        sb->foot_off[S] = calloc(ntiles + 1, sizeof(int32_t));
        sb->foot[S] = malloc(sizeof(int32_t) * (m ? m : 1));
        sb->acc[S] = malloc(sizeof(uint32_t) * (m ? m : 1));
        for (int64_t i = 0; i < m; i++) {
            sb->foot_off[S][(t[i].key >> 32) + 1]++;
            sb->foot[S][i] = (int32_t)(t[i].key & 0xffffffffu);
            sb->acc[S][i] = t[i].bits;
        }
        for (int tt = 0; tt < ntiles; tt++) sb->foot_off[S][tt + 1] += sb->foot_off[S][tt];
        free(t);
    }
    return 0;
}

/* R11: seeds written by a T_ne iteration of sub-chain sb become non-exec */
static void carry_stale(const or_chain *c, const or_sched *s, const sub_t *sb, uint8_t *region) {
    for (int j = sb->first; j < sb->first + sb->n; j++) {
        const loop_t *L = &c->loops[j];
        for (int64_t it = 0; it < c->size[L->set]; it++) {
            if (s->sigma[j][it] != sb->tne) continue;
            for (int i = 0; i < L->ndesc; i++) {
                const desc_t *D = &L->d[i];
                if (D->mode == OR_R) continue;
                if (D->map < 0) region[it] = 2;
                else
                    for (int k = 0; k < c->maps[D->map].arity; k++)
                        region[c->maps[D->map].values[it * c->maps[D->map].arity + k]] = 2;
            }
        }
    }
}

int or_inspect(const or_chain *c, int64_t ts, int partition, const double *seed_xy, int max_rounds,
               int max_colour_tiles, const int32_t *splits, int nsplits, const int32_t *sub_ts, or_sched **out) {
    return or_inspect_regions(c, ts, partition, seed_xy, max_rounds, max_colour_tiles, splits, nsplits, sub_ts, NULL,
                              0, out);
}

int or_inspect_regions(const or_chain *c, int64_t ts, int partition, const double *seed_xy, int max_rounds,
                       int max_colour_tiles, const int32_t *splits, int nsplits, const int32_t *sub_ts,
                       const uint8_t *seed_region, int carry, or_sched **out) {
    *out = NULL;
    if (ts < 1 || c->nloops == 0 || max_rounds < 1 || max_colour_tiles < 0) return -1;
    if (sub_ts)
        for (int i = 0; i <= nsplits; i++)
            if (sub_ts[i] < 1) return -1;
    uint8_t *region = NULL;
    if (seed_region) {
        /* every sub-chain seeds on the region set; no cap; carry needs all writes there */
        int rset = c->loops[0].set;
        if (max_colour_tiles != 0) return -1;
        for (int i = 0; i < nsplits; i++)
            if (splits[i] < 0 || splits[i] >= c->nloops || c->loops[splits[i]].set != rset) return -1;
        for (int64_t e = 0; e < c->size[rset]; e++)
            if (seed_region[e] > 2) return -1;
        if (carry)
            for (int j = 0; j < c->nloops; j++)
                for (int i = 0; i < c->loops[j].ndesc; i++)
                    if (c->loops[j].d[i].mode != OR_R && dset(c, &c->loops[j], &c->loops[j].d[i]) != rset) return -1;
        region = malloc((size_t)(c->size[rset] ? c->size[rset] : 1));
        memcpy(region, seed_region, (size_t)c->size[rset]);
    }
    or_sched *s = calloc(1, sizeof(*s));
    s->nloops = c->nloops;
    for (int j = 0; j < c->nloops; j++) {
        s->loop_size[j] = c->size[c->loops[j].set];
        s->sigma[j] = malloc(sizeof(int32_t) * (s->loop_size[j] + 1));
    }
    int start = 0;
    for (int i = 0; i <= nsplits; i++) {
        int end = (i < nsplits) ? splits[i] : c->nloops;
        if (end <= start || end > c->nloops || end - start > 31) { or_sched_free(s); free(region); return -1; }
        sub_t *sb = &s->sub[s->nsub++];
        sb->first = start;
        sb->n = end - start;
        for (int j = start; j < end; j++) s->sub_of[j] = s->nsub - 1;
        /* a fusion scheme gives each sub-chain its own seed tile size (Sec. 7.2) */
        int rc = inspect_sub(c, s, sb, sub_ts ? sub_ts[i] : ts, partition, seed_xy, max_rounds, max_colour_tiles,
                             region);
        if (rc) { or_sched_free(s); free(region); return rc; }
        if (region && carry) carry_stale(c, s, sb, region);
        start = end;
    }
    free(region);
    *out = s;
    return 0;
}

int or_sched_regions(const or_sched *s, int sub, int32_t *info, uint8_t *region) {
    if (sub < 0 || sub >= s->nsub || !s->sub[sub].region) return -1;
    const sub_t *b = &s->sub[sub];
    if (info) {
        info[0] = b->ncore;
        info[1] = b->nbnd;
        info[2] = b->tne;
        info[3] = b->color[b->tne];
    }
    if (region) memcpy(region, b->region, (size_t)s->loop_size[b->first]);
    return 0;
}

void or_sched_free(or_sched *s) {
    if (!s) return;
    for (int j = 0; j < s->nloops; j++) free(s->sigma[j]);
    for (int i = 0; i < s->nsub; i++) {
        free(s->sub[i].color);
        free(s->sub[i].region);
        for (int S = 0; S < MAXSETS; S++) {
            free(s->sub[i].foot_off[S]);
            free(s->sub[i].foot[S]);
            free(s->sub[i].acc[S]);
        }
    }
    free(s);
}

int or_sched_nsub(const or_sched *s) { return s->nsub; }

int or_sched_sub_info(const or_sched *s, int sub, int32_t *first_loop, int32_t *nloops, int32_t *ntiles,
                      int32_t *ncolors, int32_t *rounds) {
    if (sub < 0 || sub >= s->nsub) return -1;
    const sub_t *b = &s->sub[sub];
    if (first_loop) *first_loop = b->first;
    if (nloops) *nloops = b->n;
    if (ntiles) *ntiles = b->ntiles;
    if (ncolors) *ncolors = b->ncolors;
    if (rounds) *rounds = b->rounds;
    return 0;
}

int or_sched_tile_color(const or_sched *s, int sub, int32_t *color) {
    if (sub < 0 || sub >= s->nsub) return -1;
    memcpy(color, s->sub[sub].color, sizeof(int32_t) * s->sub[sub].ntiles);
    return 0;
}

int or_sched_sigma(const or_sched *s, int loop, int32_t *sigma) {
    if (loop < 0 || loop >= s->nloops) return -1;
    memcpy(sigma, s->sigma[loop], sizeof(int32_t) * s->loop_size[loop]);
    return 0;
}

int or_sched_tiles_by_color(const or_sched *s, int sub, int32_t *color_off, int32_t *tiles) {
    if (sub < 0 || sub >= s->nsub) return -1;
    const sub_t *b = &s->sub[sub];
    for (int k = 0; k <= b->ncolors; k++) color_off[k] = 0;
    for (int t = 0; t < b->ntiles; t++) color_off[b->color[t] + 1]++;
    for (int k = 0; k < b->ncolors; k++) color_off[k + 1] += color_off[k];
    int32_t *pos = malloc(sizeof(int32_t) * (b->ncolors + 1));
    memcpy(pos, color_off, sizeof(int32_t) * (b->ncolors + 1));
    for (int t = 0; t < b->ntiles; t++) tiles[pos[b->color[t]]++] = t;
    free(pos);
    return 0;
}

int64_t or_sched_footprint(const or_sched *s, int sub, int set, int32_t *off, int32_t *elem, uint32_t *acc) {
    if (sub < 0 || sub >= s->nsub || set < 0 || set >= MAXSETS) return -1;
    const sub_t *b = &s->sub[sub];
    if (!b->foot_off[set]) return 0;
    int64_t m = b->foot_len[set];
    if (off) memcpy(off, b->foot_off[set], sizeof(int32_t) * (b->ntiles + 1));
    if (elem) memcpy(elem, b->foot[set], sizeof(int32_t) * m);
    if (acc) memcpy(acc, b->acc[set], sizeof(uint32_t) * m);
    return m;
}

int or_sched_set_color(or_sched *s, int sub, int tile, int color) {
    if (sub < 0 || sub >= s->nsub || tile < 0 || tile >= s->sub[sub].ntiles) return -1;
    s->sub[sub].color[tile] = color;
    if (color + 1 > s->sub[sub].ncolors) s->sub[sub].ncolors = color + 1;
    return 0;
}

int or_sched_set_sigma(or_sched *s, int loop, int64_t it, int tile) {
    if (loop < 0 || loop >= s->nloops) return -1;
    s->sigma[loop][it] = tile;
    return 0;
}

int or_sched_iters(const or_sched *s, int loop, int32_t *tile_off, int32_t *iters) {
    if (loop < 0 || loop >= s->nloops) return -1;
    const sub_t *b = &s->sub[s->sub_of[loop]];
    int64_t n = s->loop_size[loop];
    for (int t = 0; t <= b->ntiles; t++) tile_off[t] = 0;
    for (int64_t e = 0; e < n; e++) tile_off[s->sigma[loop][e] + 1]++;
    for (int t = 0; t < b->ntiles; t++) tile_off[t + 1] += tile_off[t];
    int32_t *pos = malloc(sizeof(int32_t) * (b->ntiles + 1));
    memcpy(pos, tile_off, sizeof(int32_t) * (b->ntiles + 1));
    for (int64_t e = 0; e < n; e++) iters[pos[s->sigma[loop][e]]++] = (int32_t)e;
    free(pos);
    return 0;
}

/* ------------------------------------------------------------------ checker */

typedef struct {
    int32_t j, it, mode, tile;
} access_t;

static int cmp_access(const void *a, const void *b) {
    const access_t *x = a, *y = b;
    if (x->j != y->j) return x->j - y->j;
    if (x->it != y->it) return x->it < y->it ? -1 : 1;
    return x->mode - y->mode;
}

/* C20: every ordered pair of accesses to one element, at least one a write. */
int64_t or_check(const or_chain *c, const or_sched *s) {
    int64_t viol = 0;
    for (int si = 0; si < s->nsub; si++) {
        const sub_t *b = &s->sub[si];
        /* every iteration assigned to one valid tile */
        for (int j = b->first; j < b->first + b->n; j++)
            for (int64_t it = 0; it < c->size[c->loops[j].set]; it++)
                if (s->sigma[j][it] < 0 || s->sigma[j][it] >= b->ntiles) viol++;
        if (viol) return viol;
        for (int S = 0; S < c->nsets; S++) {
            /* bucket accesses per element */
            int64_t nS = c->size[S];
            int32_t *cnt = calloc(nS + 1, sizeof(int32_t));
            for (int j = b->first; j < b->first + b->n; j++) {
                const loop_t *L = &c->loops[j];
                for (int i = 0; i < L->ndesc; i++) {
                    const desc_t *D = &L->d[i];
                    if (dset(c, L, D) != S) continue;
                    for (int64_t it = 0; it < c->size[L->set]; it++) {
                        if (D->map < 0) cnt[it + 1]++;
                        else {
                            const map_t *m = &c->maps[D->map];
                            for (int k = 0; k < m->arity; k++) cnt[m->values[it * m->arity + k] + 1]++;
                        }
                    }
                }
            }
            for (int64_t e = 0; e < nS; e++) cnt[e + 1] += cnt[e];
            access_t *acc = malloc(sizeof(access_t) * (cnt[nS] + 1));
            int32_t *pos = malloc(sizeof(int32_t) * (nS + 1));
            memcpy(pos, cnt, sizeof(int32_t) * (nS + 1));
            for (int j = b->first; j < b->first + b->n; j++) {
                const loop_t *L = &c->loops[j];
                for (int i = 0; i < L->ndesc; i++) {
                    const desc_t *D = &L->d[i];
                    if (dset(c, L, D) != S) continue;
                    for (int64_t it = 0; it < c->size[L->set]; it++) {
                        access_t a = {j, (int32_t)it, D->mode, s->sigma[j][it]};
                        if (D->map < 0) acc[pos[it]++] = a;
                        else {
                            const map_t *m = &c->maps[D->map];
                            for (int k = 0; k < m->arity; k++) acc[pos[m->values[it * m->arity + k]]++] = a;
                        }
                    }
                }
            }
            for (int64_t e = 0; e < nS; e++) {
                access_t *A = acc + cnt[e];
                int64_t na = cnt[e + 1] - cnt[e];
                qsort(A, na, sizeof(access_t), cmp_access); /* untiled order */
                for (int64_t p = 0; p < na; p++)
                    for (int64_t q = p + 1; q < na; q++) {
                        const access_t *x = &A[p], *y = &A[q];
                        if (x->mode == OR_R && y->mode == OR_R) continue;
                        int cx = b->color[x->tile], cy = b->color[y->tile];
                        if (x->j == y->j) {
                            /* intra-loop: only concurrent writes/increments race */
                            if (x->mode != OR_R && y->mode != OR_R && x->tile != y->tile && cx == cy) viol++;
                            continue;
                        }
                        if (x->tile == y->tile) continue; /* loops run in chain order inside a tile */
                        if (cx == cy) { viol++; continue; }
                        if (cx > cy) viol++;
                    }
            }
            free(acc);
            free(pos);
            free(cnt);
        }
    }
    return viol;
}

/* -------------------------------------------------------- instrumented chain */

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void instr_iteration(const or_chain *c, int j, int64_t it, uint64_t **data, const int *dsetof) {
    const loop_t *L = &c->loops[j];
    uint64_t h = mix64(((uint64_t)j << 40) ^ (uint64_t)it);
    for (int i = 0; i < L->ndesc; i++) {
        const desc_t *D = &L->d[i];
        if (D->mode != OR_R || D->data < 0) continue;
        int ar = D->map < 0 ? 1 : c->maps[D->map].arity;
        for (int k = 0; k < ar; k++) {
            int64_t x = D->map < 0 ? it : c->maps[D->map].values[it * ar + k];
            h = mix64(h ^ data[D->data][x]);
        }
    }
    for (int i = 0; i < L->ndesc; i++) {
        const desc_t *D = &L->d[i];
        if (D->mode == OR_R || D->data < 0) continue;
        int ar = D->map < 0 ? 1 : c->maps[D->map].arity;
        for (int k = 0; k < ar; k++) {
            int64_t x = D->map < 0 ? it : c->maps[D->map].values[it * ar + k];
            if (D->mode == OR_W) data[D->data][x] = h ^ (uint64_t)k;
            else data[D->data][x] += (h ^ (uint64_t)k) % 524288u; /* commutative increment */
        }
    }
    (void)dsetof;
}

int or_instrumented_run(const or_chain *c, const or_sched *s, int nrep, uint64_t *hash_out) {
    /* data spaces: ids used by descriptors; size = target set size */
    int maxd = -1;
    int64_t dsize[64] = {0};
    for (int j = 0; j < c->nloops; j++)
        for (int i = 0; i < c->loops[j].ndesc; i++) {
            const desc_t *D = &c->loops[j].d[i];
            if (D->data < 0) continue;
            if (D->data >= 64) return -1;
            if (D->data > maxd) maxd = D->data;
            dsize[D->data] = c->size[dset(c, &c->loops[j], D)];
        }
    uint64_t *data[64] = {0};
    for (int d = 0; d <= maxd; d++) {
        data[d] = malloc(sizeof(uint64_t) * (dsize[d] + 1));
        for (int64_t x = 0; x < dsize[d]; x++) data[d][x] = mix64(((uint64_t)d << 48) ^ (uint64_t)x);
    }
    for (int r = 0; r < nrep; r++) {
        if (!s) {
            for (int j = 0; j < c->nloops; j++)
                for (int64_t it = 0; it < c->size[c->loops[j].set]; it++) instr_iteration(c, j, it, data, NULL);
        } else {
            for (int si = 0; si < s->nsub; si++) {
                const sub_t *b = &s->sub[si];
                int32_t *coff = malloc(sizeof(int32_t) * (b->ncolors + 1));
                int32_t *tl = malloc(sizeof(int32_t) * (b->ntiles + 1));
                or_sched_tiles_by_color(s, si, coff, tl);
                for (int p = 0; p < b->ntiles; p++) {
                    int t = tl[p];
                    if (b->region && t == b->tne) continue; /* T_ne is never executed */
                    for (int j = b->first; j < b->first + b->n; j++)
                        for (int64_t it = 0; it < c->size[c->loops[j].set]; it++)
                            if (s->sigma[j][it] == t) instr_iteration(c, j, it, data, NULL);
                }
                free(coff);
                free(tl);
            }
        }
    }
    uint64_t h = 0;
    for (int d = 0; d <= maxd; d++)
        for (int64_t x = 0; x < dsize[d]; x++) h = mix64(h ^ data[d][x] ^ ((uint64_t)d << 56));
    for (int d = 0; d <= maxd; d++) free(data[d]);
    *hash_out = h;
    return 0;
}

/* -------------------------------------------------------- tiled DG executor */

void or_dg_begin_step(or_dg *d, double t_half);
void or_dg_iteration(or_dg *d, int j, int64_t it);
int or_dg_nloops(const or_dg *d);
void or_dg_load(or_dg *d, const double *v, const double *s);
void or_dg_store(const or_dg *d, double *v, double *s);
double or_dg_dt(const or_dg *d);

/* Alg. 2 on one shared-memory node: colour by colour, tile by tile, and
 * inside a tile every loop's iterations in chain order.  A schedule of a chain
 * fused over F steps (F times the step's loops) runs F steps per pass; loop j
 * belongs to step j / (loops per step) of the pass and takes that step's time. */
int or_dg_step_tiled(or_dg *d, const or_sched *sch, double *v, double *s, int64_t nsteps, double t0) {
    int lps = or_dg_nloops(d);
    if (sch->nloops % lps) return -1;
    int fuse = sch->nloops / lps;
    if (nsteps % fuse) return -1;
    or_chain *c;
    if (or_dg_chain_steps(d, fuse, &c)) return -1;
    if (sch->nloops != c->nloops) { or_chain_free(c); return -1; }
    /* per loop, per tile iteration lists */
    int32_t *toff[MAXLOOPS], *its[MAXLOOPS];
    for (int j = 0; j < c->nloops; j++) {
        const sub_t *b = &sch->sub[sch->sub_of[j]];
        toff[j] = malloc(sizeof(int32_t) * (b->ntiles + 1));
        its[j] = malloc(sizeof(int32_t) * (c->size[c->loops[j].set] + 1));
        or_sched_iters(sch, j, toff[j], its[j]);
    }
    or_dg_load(d, v, s);
    double dt = or_dg_dt(d);
    for (int64_t n = 0; n < nsteps; n += fuse) {
        for (int si = 0; si < sch->nsub; si++) {
            const sub_t *b = &sch->sub[si];
            int32_t *coff = malloc(sizeof(int32_t) * (b->ncolors + 1));
            int32_t *tl = malloc(sizeof(int32_t) * (b->ntiles + 1));
            or_sched_tiles_by_color(sch, si, coff, tl);
            for (int p = 0; p < b->ntiles; p++) {
                int t = tl[p];
                if (b->region && t == b->tne) continue; /* T_ne is never executed (Alg. 2) */
                for (int j = b->first; j < b->first + b->n; j++) {
                    or_dg_begin_step(d, t0 + ((double)(n + j / lps) + 0.5) * dt);
                    for (int32_t q = toff[j][t]; q < toff[j][t + 1]; q++) or_dg_iteration(d, j % lps, its[j][q]);
                }
            }
            free(coff);
            free(tl);
        }
    }
    or_dg_store(d, v, s);
    for (int j = 0; j < c->nloops; j++) {
        free(toff[j]);
        free(its[j]);
    }
    or_chain_free(c);
    return 0;
}
