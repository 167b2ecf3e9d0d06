/*
 * oracle.h -- plain, slow, FP64 CPU oracle for the sparse-tiled DG elastic
 * loop chain.  TEST INFRASTRUCTURE ONLY: the product path (libdgtile and its
 * Python binding) never links, loads or calls anything declared here; only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * Contents (each function cites the passage of Luporini et al., "Automated
 * Tiling of Unstructured Mesh Computations with Application to Seismological
 * Modelling", that it follows; where the paper is silent the reading used is
 * stated in the .c file):
 *   refelem.c  nodal P_k reference triangle (mass, derivatives, facet mass)
 *   mesh.c     facet maps from cell-to-vertex connectivity
 *   dg.c       the untiled velocity-stress DG loop chain, energy, source
 *   chain.c    loop-chain model, inspector (Alg. 1, 3, 4), dependence checker,
 *              tiled executor (Alg. 2) and an integer-instrumented chain
 *
 * Every function returns 0 on success and a negative value on error.
 */
#ifndef DGTILE_ORACLE_H
#define DGTILE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- reference element ---------------- */
int or_np(int k);
/* Fills (any pointer may be NULL): nodes[Np*2], M[Np*Np], Minv[Np*Np], Dr[Np*Np]
 * (Dr[i*Np+j] = d phi_j / dr at node i), Ds, M1[(k+1)^2] (facet mass on [0,1]),
 * fnodes[3*(k+1)] (cell node index of facet node m of local facet f). */
int or_refelem(int k, double *nodes, double *M, double *Minv, double *Dr, double *Ds,
               double *M1, int32_t *fnodes);
/* Triangle quadrature of the oracle (collapsed Gauss-Legendre): returns count. */
int or_tri_quad(int n, double *pts /*[n*n*2]*/, double *w /*[n*n]*/);
/* Lagrange basis of degree k at (r,s): phi[Np]. */
int or_basis(int k, double r, double s, double *phi);

/* ---------------- mesh ---------------- */
typedef struct or_mesh or_mesh;
/* periodic: bit0 x, bit1 y.  Returns <0 for invalid meshes. */
int or_mesh_build(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int periodic,
                  or_mesh **out);
void or_mesh_free(or_mesh *m);
void or_mesh_counts(const or_mesh *m, int64_t *nc, int64_t *nf, int64_t *nb);
/* f2c[nf*2], f2l[nf*2] (local facet ids), b2c[nb], b2l[nb], bside[nb] (0..3 bbox side or -1) */
void or_mesh_maps(const or_mesh *m, int32_t *f2c, int8_t *f2l, int32_t *b2c, int8_t *b2l,
                  int8_t *bside);

/* ---------------- DG loop chain ---------------- */
typedef struct or_dg or_dg;
int or_dg_create(const or_mesh *m, int k, const double *lam, const double *mu, const double *rho,
                 int flux /*0 central, 1 upwind*/, int order /*2|4*/, double dt,
                 int free_sides /*bbox sides with free surface; others absorbing*/, or_dg **out);
void or_dg_free(or_dg *d);
int or_dg_set_source(or_dg *d, double x, double y, double f0, double t0, double amp);
int or_dg_source_cell(const or_dg *d);
/* Untiled chain, loops in chain order and iterations in ascending id.
 * v[2*Np*nc], s[3*Np*nc] in [comp][node][cell] layout, updated in place. */
int or_dg_step(or_dg *d, double *v, double *s, int64_t nsteps, double t0);
double or_dg_energy(const or_dg *d, const double *v, const double *s_new, const double *s_old);
double or_cfl_dt(const or_mesh *m, int k, const double *lam, const double *mu, const double *rho,
                 double cfl);
double or_ricker(double t, double f0, double t0, double amp);
/* Semi-discrete rate operator u' = L u (no source, no lagging): applies the
 * velocity operator (incl. penalty) and the stress operator to (v, s). */
int or_dg_rate(or_dg *d, const double *v, const double *s, double *dv, double *ds);
/* The chain as a generic loop chain (sets C, F, B; maps f2c, b2c). */
struct or_chain;
int or_dg_chain(const or_dg *d, struct or_chain **out);
/* The chain of `steps` consecutive steps (the step's loops repeated; at most 64). */
int or_dg_chain_steps(const or_dg *d, int steps, struct or_chain **out);

/* ---------------- loop chain + inspector ---------------- */
typedef struct or_chain or_chain;
typedef struct or_sched or_sched;
enum { OR_R = 0, OR_W = 1, OR_INC = 2 };
int or_chain_create(or_chain **out);
void or_chain_free(or_chain *c);
int or_chain_set(or_chain *c, int64_t size);
int or_chain_map(or_chain *c, int from, int to, int arity, const int32_t *values);
/* maps[i] = map id or -1 (direct), modes[i] in OR_R/W/INC, data[i] = data space id */
int or_chain_loop(or_chain *c, int set, int ndesc, const int32_t *maps, const int32_t *modes,
                  const int32_t *data);
int or_chain_nloops(const or_chain *c);
/* read-back of the chain (tests): set sizes, loops (maps[ndesc], modes[ndesc], at
 * most 8), maps (values[size(from)*arity] or NULL) */
int64_t or_chain_set_size(const or_chain *c, int set);
int or_chain_get_loop(const or_chain *c, int j, int32_t *set, int32_t *ndesc, int32_t *maps, int32_t *modes);
int or_chain_get_map(const or_chain *c, int m, int32_t *from, int32_t *to, int32_t *arity, int32_t *values);

/* Alg. 1 with readings C10-C17; splits = loop indices starting new sub-chains;
 * max_colour_tiles > 0 caps every colour class after each colouring (R5b in chain.c). */
int or_inspect(const or_chain *c, int64_t ts, int partition, const double *seed_xy,
               int max_rounds, int max_colour_tiles, const int32_t *splits, int nsplits,
               const int32_t *sub_ts, or_sched **out);
/* Alg. 1 with regions (Sec. 3.3, 5.1.2; readings R10, R11 in chain.c):
 * seed_region[size(seed set)] in {0 core, 1 boundary, 2 non-exec}; every
 * sub-chain must start on the seed set of loop 0; max_colour_tiles must be 0.
 * carry = 1: one halo exchange for the whole chain (later sub-chains treat seeds
 * written by an earlier T_ne as non-exec; every write must land in the seed
 * set); carry = 0: each sub-chain starts from seed_region. */
int or_inspect_regions(const or_chain *c, int64_t ts, int partition, const double *seed_xy,
                       int max_rounds, int max_colour_tiles, const int32_t *splits, int nsplits,
                       const int32_t *sub_ts, const uint8_t *seed_region, int carry, or_sched **out);
/* info[4] = {core tiles, boundary tiles, T_ne id, T_ne colour}; region[size(seed
 * set)] = the seed regions the sub-chain was inspected with.  -1 without regions. */
int or_sched_regions(const or_sched *s, int sub, int32_t *info, uint8_t *region);
void or_sched_free(or_sched *s);
int or_sched_nsub(const or_sched *s);
/* per sub-chain: loop range, ntiles, ncolors, rounds used */
int or_sched_sub_info(const or_sched *s, int sub, int32_t *first_loop, int32_t *nloops,
                      int32_t *ntiles, int32_t *ncolors, int32_t *rounds);
int or_sched_tile_color(const or_sched *s, int sub, int32_t *color /*[ntiles]*/);
/* tiling function of loop j (global loop index): tile per iteration */
int or_sched_sigma(const or_sched *s, int loop, int32_t *sigma /*[size(S_j)]*/);
/* iteration lists of loop j: tile_off[ntiles+1], iters[size(S_j)] */
int or_sched_iters(const or_sched *s, int loop, int32_t *tile_off, int32_t *iters);
/* footprint of sub-chain `sub` on set `set`: returns total length; fills
 * off[ntiles+1], elem[len], acc[len] (bit i = loop first+i touches it in that
 * tile; bit 31 = element touched by one tile only).  Pointers may be NULL. */
int64_t or_sched_footprint(const or_sched *s, int sub, int set, int32_t *off, int32_t *elem,
                           uint32_t *acc);
/* tiles in execution order (colour, id) */
int or_sched_tiles_by_color(const or_sched *s, int sub, int32_t *color_off, int32_t *tiles);
/* overwrite a tile colour (negative tests of the checker) */
int or_sched_set_color(or_sched *s, int sub, int tile, int color);
/* overwrite sigma of one iteration (negative tests) */
int or_sched_set_sigma(or_sched *s, int loop, int64_t it, int tile);

/* C20: brute-force dependence-validity checker; returns the number of violations
 * (0 = legal), or <0 on error.  Also checks every iteration has exactly one tile. */
int64_t or_check(const or_chain *c, const or_sched *s);

/* Integer-instrumented chain: one uint64 array per data space, sized by its set.
 * Runs untiled (s == NULL) or in schedule order; returns a hash of all data. */
int or_instrumented_run(const or_chain *c, const or_sched *s, int nrep, uint64_t *hash_out);

/* Test hooks: one pass of tiling with given colours (sigma[j] preallocated per
 * loop); projection of `set` after projecting loops 0..upto-1 (tile or -1);
 * literal reading of Alg. 3 (indirect projections restart from bottom). */
int or_tile_with_colors(const or_chain *c, const int32_t *tile0, int ntiles, const int32_t *color,
                        int32_t **sigma);
int or_projection_after(const or_chain *c, const int32_t *tile0, int ntiles, const int32_t *color, int upto,
                        int set, int32_t *phi_tile);
void or_set_literal_projection(int on);

/* Tiled DG step: the same per-iteration kernels as or_dg_step run in
 * schedule order (Alg. 2: colour by colour, tile by tile, loop by loop).  A
 * schedule of the chain of F steps (or_dg_chain_steps) runs F steps per pass;
 * nsteps must be a multiple of F. */
int or_dg_step_tiled(or_dg *d, const or_sched *sch, double *v, double *s, int64_t nsteps, double t0);

#ifdef __cplusplus
}
#endif
#endif
