/*
 * dgtile.h -- C ABI of libdgtile: sparse-tiled, fused execution of the loop
 * chain of a discontinuous-Galerkin velocity-stress elastic time step on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Luporini, Lange, Jacobs, Gorman, Ramanujam, Kelly, "Automated Tiling
 * of Unstructured Mesh Computations with Application to Seismological
 * Modelling" (ACM TOMS; arXiv 1708.03183).
 *   - loop chain abstraction (sets, maps, loops with descriptors): Sec. 2;
 *   - inspector (seed partition, colouring, projection, tiling, conflicts,
 *     local maps): Sec. 5.1, Alg. 1, Alg. 3, Alg. 4;
 *   - executor (colour by colour, one tile at a time, loops in chain order
 *     inside a tile): Sec. 5.2, Alg. 2;
 *   - the DG elastic application (cell, interior-facet and exterior-facet
 *     loops plus block-diagonal inverse-mass solves, 4th-order leapfrog):
 *     Sec. 7.1-7.3.
 *
 * Conventions
 *   - Every function returns a dgt_status; DGT_OK is 0.  No C++ exception
 *     crosses this boundary.  dgt_last_error() returns a thread-local message
 *     describing the last non-OK status of the calling thread.
 *   - "host" pointers are read (and copied) during the call; "device" pointers
 *     are HIP device addresses on the solver's device.
 *   - Objects are not thread-safe; distinct objects may be used from distinct
 *     threads.
 *   - Work is enqueued on the HIP stream given at creation; functions that
 *     synchronise say so.
 *   - Cell-based device arrays use the layout [component][node][cell] with the
 *     cell index fastest (a "field" of ncomp components and Np nodes).
 */
#ifndef DGTILE_H
#define DGTILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DGT_OK = 0,
    DGT_EINVAL = 1,        /* invalid argument or mesh */
    DGT_ENOMEM = 2,        /* device or host allocation failed */
    DGT_EHIP = 3,          /* a HIP runtime call failed */
    DGT_ESTATE = 4,        /* call not valid in the object's state, or the
                              inspector exceeded max_conflict_rounds */
    DGT_EUNSUPPORTED = 5   /* valid request this build cannot run (e.g. a tile
                              footprint beyond 16,383 cells) */
} dgt_status;

/* Message for the calling thread's last failing call (never NULL). */
const char *dgt_last_error(void);
/* ABI version of this header (major*100 + minor). */
int dgt_version(void);

/* =====================================================================
 * Tier 1: generic loop chain and GPU inspector (Sec. 2, Sec. 5.1)
 * ===================================================================== */

typedef struct dgt_chain dgt_chain;
typedef struct dgt_schedule dgt_schedule;

/* Access modes of a descriptor (Sec. 2): read, write, increment. */
typedef enum { DGT_R = 0, DGT_W = 1, DGT_INC = 2 } dgt_mode;

/* Descriptor <M, mode> (Sec. 2).  map = map id or -1 for a direct access.
 * data = id of the data space accessed (>= 0) or -1; the inspector analyses
 * dependences per set (Sec. 2) and ignores it, the checker tools use it. */
typedef struct {
    int32_t map;
    int32_t mode;
    int32_t data;
} dgt_desc;

/* Create an empty chain.  *out owned by the caller (dgt_chain_destroy). */
dgt_status dgt_chain_create(dgt_chain **out);
/* Add an iteration set of `size` >= 0 elements; *set_id receives its id
 * (0, 1, ...).  At most 8 sets. */
dgt_status dgt_chain_set(dgt_chain *c, int64_t size, int32_t *set_id);
/* Add a map M: from -> to^arity (Sec. 2).  values: host, [size(from)*arity],
 * each in [0, size(to)); copied.  EINVAL on out-of-range values.  At most 8. */
dgt_status dgt_chain_map(dgt_chain *c, int32_t from, int32_t to, int32_t arity, const int32_t *values,
                         int32_t *map_id);
/* Append loop L_j over `set` with ndesc (<= 8) descriptors (host, copied).
 * Every indirect descriptor's map must start at `set`.  At most 64 loops. */
dgt_status dgt_chain_loop(dgt_chain *c, int32_t set, int32_t ndesc, const dgt_desc *desc, int32_t *loop_id);
void dgt_chain_destroy(dgt_chain *c);

/* Inspector parameters (Alg. 1). */
typedef struct {
    int64_t tile_size;            /* seed iterations per tile, >= 1 (Sec. 5.1.2) */
    int32_t partition;            /* 0: blocks of the given numbering (the paper's
                                     choice); 1: blocks of the Hilbert order of
                                     seed_xy (quantised to 2^16 per axis) */
    const double *seed_xy;        /* host [size(seed)*2] points of the seed set;
                                     required when partition == 1 */
    int32_t max_conflict_rounds;  /* colouring rounds before DGT_ESTATE, >= 1 */
    const int32_t *splits;        /* host [nsplits] ascending loop indices where a
                                     new sub-chain (fusion scheme, Sec. 7.4)
                                     starts; each sub-chain has <= 31 loops and
                                     is inspected independently */
    int32_t nsplits;
    int32_t max_colour_tiles;     /* 0: colour classes as Jones-Plassmann leaves them;
                                     > 0: after each colouring, a deterministic
                                     greedy pass (tiles in ascending id) moves tiles
                                     out of classes larger than this into the
                                     smallest colour with room that no neighbour
                                     has, or into a new colour, so that no colour
                                     launch needs more than one round of resident
                                     workgroups.  -1 (dgt_solver_inspect only): the
                                     solver picks the number of tile workgroups the
                                     GPU holds at once when a class exceeds it. */
    const int32_t *sub_tile_sizes; /* host [nsplits+1]: the seed tile size of each
                                     sub-chain (a fusion scheme fixes one per
                                     sub-chain, Sec. 7.2), each >= 1; NULL:
                                     tile_size for all */
    const uint8_t *seed_region;   /* host [size(seed set)] or NULL.  The region of
                                     each seed iteration on one process's part of a
                                     distributed mesh (Sec. 3.3): 0 core, 1 boundary
                                     (owned iterations next to the halo, and exec
                                     halo), 2 non-exec halo.  Seeds of each region
                                     are cut into blocks of tile_size in seed order:
                                     core tiles 0.., then boundary tiles, then one
                                     tile T_ne with every non-exec seed (Sec.
                                     5.1.2).  Each region's tiles are coloured apart
                                     (Jones-Plassmann on the edges inside the
                                     region); boundary colours follow the core ones
                                     and T_ne alone takes the highest colour; it is
                                     never executed (Alg. 2).  Every sub-chain must
                                     start on the seed set of loop 0, and
                                     max_colour_tiles must be 0 (else DGT_EINVAL). */
    int32_t region_carry;         /* with seed_region: 0, every sub-chain starts from
                                     seed_region (one halo exchange before each
                                     sub-chain, as in the paper); 1, one exchange
                                     before the first sub-chain only: a later
                                     sub-chain also treats as non-exec every seed
                                     element that T_ne of an earlier sub-chain
                                     writes (its value is stale), which needs every
                                     write of the chain to land in the seed set
                                     (else DGT_EINVAL). */
} dgt_inspect_params;

/* Run the inspector on the GPU (Alg. 1 with Alg. 3 projections and Alg. 4
 * tiling functions, colouring and conflict rounds).  The result is a pure
 * function of the chain and the parameters (bit-identical run to run).
 * stream: hipStream_t or NULL (default stream).  Synchronises the stream.
 * *out owned by the caller (dgt_schedule_destroy). */
dgt_status dgt_inspect(const dgt_chain *c, const dgt_inspect_params *p, void *stream, dgt_schedule **out);

/* Read-back of a schedule (host copies; each call synchronises). */
dgt_status dgt_schedule_nsub(const dgt_schedule *s, int32_t *nsub);
dgt_status dgt_schedule_sub_info(const dgt_schedule *s, int32_t sub, int32_t *first_loop, int32_t *nloops,
                                 int32_t *ntiles, int32_t *ncolors, int32_t *rounds);
/* tile colours of sub-chain `sub`: host [ntiles] */
dgt_status dgt_schedule_colors(const dgt_schedule *s, int32_t sub, int32_t *color);
/* tiling function sigma_j of loop j: host [size(S_j)] tile per iteration */
dgt_status dgt_schedule_sigma(const dgt_schedule *s, int32_t loop, int32_t *sigma);
/* iteration lists [T_i]_j of loop j (ascending id in each tile):
 * host tile_off[ntiles+1], iters[size(S_j)] */
dgt_status dgt_schedule_iters(const dgt_schedule *s, int32_t loop, int32_t *tile_off, int32_t *iters);
/* footprint of sub-chain `sub` on `set`: elements touched by each tile through
 * any descriptor, ascending per tile, with acc bit i set when loop
 * (first_loop + i) touches the element in that tile, and bit 31 set when one
 * tile alone touches it.  *len receives the total; arrays may be NULL to query
 * the length: host off[ntiles+1], elem[len], acc[len]. */
dgt_status dgt_schedule_footprint(const dgt_schedule *s, int32_t sub, int32_t set, int64_t *len, int32_t *off,
                                  int32_t *elem, uint32_t *acc);
/* tiles in execution order (colour ascending, then id): host color_off[ncolors+1], tiles[ntiles] */
dgt_status dgt_schedule_tiles_by_color(const dgt_schedule *s, int32_t sub, int32_t *color_off, int32_t *tiles);
/* Regions of sub-chain `sub` of a region-aware schedule: info[4] = {core tiles,
 * boundary tiles, id of T_ne, colour of T_ne}; region (host [size(seed set)] or
 * NULL) = the seed regions the sub-chain was inspected with (after carrying
 * stale seeds).  DGT_EINVAL for a schedule without regions. */
dgt_status dgt_schedule_regions(const dgt_schedule *s, int32_t sub, int32_t *info, uint8_t *region);
/* JSON inspection summary (tiles, colours, rounds, footprint sizes, GPU time
 * of the inspector in ms); writes at most len bytes including the NUL. */
dgt_status dgt_schedule_summary_json(const dgt_schedule *s, char *buf, size_t len);
void dgt_schedule_destroy(dgt_schedule *s);

/* =====================================================================
 * Tier 2: the DG elastic solver built on tier 1 (Sec. 7.1-7.3)
 * ===================================================================== */

typedef struct dgt_mesh dgt_mesh;
typedef struct dgt_solver dgt_solver;

/* Triangle mesh from vertex coordinates (host [nv*2], double) and counter-
 * clockwise cell-to-vertex connectivity (host [nc*3]); copied.  periodic: bit 0
 * pairs the x = xmin / xmax boundary edges, bit 1 the y ones.  Derives the
 * interior-facet map f2c (cells ascending, local facets 0..2, emitted from the
 * lower cell id; local facet l joins local vertices l and l+1 mod 3), the
 * exterior-facet map b2c, and each exterior facet's bounding-box side.
 * EINVAL for a clockwise or degenerate cell, an edge shared by > 2 cells, or a
 * vertex id out of range.  *out owned by the caller (dgt_mesh_destroy). */
dgt_status dgt_mesh_create(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int32_t periodic,
                           dgt_mesh **out);
dgt_status dgt_mesh_counts(const dgt_mesh *m, int64_t *nc, int64_t *nf, int64_t *nb);
/* host copies: f2c[nf*2], f2l[nf*2], b2c[nb], b2l[nb], bside[nb] (0: x=xmin,
 * 1: x=xmax, 2: y=ymin, 3: y=ymax, -1: none).  Any pointer may be NULL. */
dgt_status dgt_mesh_maps(const dgt_mesh *m, int32_t *f2c, int8_t *f2l, int32_t *b2c, int8_t *b2l, int8_t *bside);
void dgt_mesh_destroy(dgt_mesh *m);

typedef struct {
    int32_t degree;      /* polynomial degree k in 1..4 (Sec. 7.4: q = 1..4) */
    int32_t flux;        /* 0 central, 1 upwind (exact isotropic Riemann state) */
    int32_t time_order;  /* 4: Taylor leapfrog (Sec. 7.1, 26 loops); 2: 8 loops */
    int32_t precision;   /* 0 FP64, 1 FP32 (state, arithmetic and accumulation) */
    int32_t free_sides;  /* bounding-box sides with a free surface (bits as
                            bside); the other exterior facets are absorbing */
    double dt;           /* time step > 0 */
} dgt_solver_params;

/* Build the solver: per-cell material lam, mu, rho (host [nc] doubles, > 0),
 * reference-element operators, device copies of mesh maps and geometry, and
 * the DG loop chain (tier 1).  stream: hipStream_t or NULL.  The mesh must
 * outlive the solver. */
dgt_status dgt_solver_create(const dgt_mesh *m, const double *lam, const double *mu, const double *rho,
                             const dgt_solver_params *p, void *stream, dgt_solver **out);
/* Inspect the solver's chain on the GPU (dgt_inspect; seed_xy is ignored and
 * the cell centroids are used) and build the executor plan: cells renumbered
 * by seed tile, within a tile the cells that other tiles' footprints gather last,
 * grouped by the neighbouring tile (the environment variable DGT_EXEC_ORDER=seed,
 * read here, keeps the plain seed order; results are identical), per-tile
 * footprints in LDS slots and local maps.  A tile whose
 * working set exceeds the LDS runs on the generic tile kernel with that working set
 * in a global scratch region per workgroup (it stays in L2 and the MALL while the
 * tile runs; sized for the largest colour launch, allocated at the first tiled
 * step).  A footprint beyond 16,383 cells cannot be addressed: the schedule is still
 * built and returned, and dgt_step in tiled mode then fails with DGT_EUNSUPPORTED
 * (smaller tile_size or more splits needed).  Synchronises the stream. */
dgt_status dgt_solver_inspect(dgt_solver *s, const dgt_inspect_params *p);
/* Multi-step fusion (an extension of the paper's fusion schemes, which stay within
 * one time step): the loop chain handed to the inspector spans `steps`
 * consecutive time steps (26 loops per step at order 4, 8 at order 2; at most 64
 * loops, each sub-chain at most 31), so a sub-chain may run the loops of two or
 * more steps in one tile pass; splits index the fused chain.  Drops the current
 * inspection (call dgt_solver_inspect again).  Tiled dgt_step then needs nsteps to
 * be a multiple of `steps` (DGT_EINVAL otherwise); the untiled chain is unchanged.
 * The chain kernel runs two whole second-order steps and the stress half of a
 * fourth-order step fused with the next velocity half; other fused sub-chains run
 * on the generic or matrix-core kernels.  Batches and the tiled FWI refuse fused
 * solvers.  DGT_EINVAL for steps < 1 or more than 64 loops. */
dgt_status dgt_solver_fuse_steps(dgt_solver *s, int32_t steps);
/* Autotuner: picks the seed tile size (from tile_sizes) and the executor
 * schedule (0 or 1, see dgt_solver_set_schedule) by timing trial steps, and
 * leaves the solver inspected and scheduled with the fastest pair.  Each
 * candidate is inspected; those the tiled executor cannot run are skipped, and
 * so are those with tiles beyond the LDS (run from global scratch) when any
 * candidate fits the LDS.  A footprint model orders the rest: the cells every tile gathers, summed over
 * tiles and sub-chains and divided by the mesh's cells (the data a step moves
 * per cell, larger for smaller tiles, in the spirit of the paper's estimates of
 * tile footprints and reuse); with prune > 0 a candidate whose model cost
 * exceeds prune times the lowest is dropped untimed.  Every remaining candidate
 * runs one step and then trial_steps timed steps (HIP events) with each
 * schedule its kernels support, from a zero state with the solver's sources
 * and shots.  The caller's state is kept (restored afterwards); without an
 * uploaded state the fields are zero afterwards.  A solver last inspected with
 * seed regions keeps them (one halo exchange per step) for every candidate.
 * Synchronises the stream.
 * EINVAL for bad parameters, EUNSUPPORTED when no candidate fits. */
typedef struct {
    const int32_t *tile_sizes;  /* host [ntile_sizes] candidate seed tile sizes, >= 1 */
    int32_t ntile_sizes;        /* 1..64 */
    const int32_t *splits;      /* fusion scheme, as in dgt_inspect_params */
    int32_t nsplits;
    int32_t partition;          /* 0 or 1, as in dgt_inspect_params */
    int32_t trial_steps;        /* timed steps per candidate and schedule, 1..1000 */
    double prune;               /* model cost cut-off (multiple of the lowest); 0: time all */
} dgt_autotune_params;
typedef struct {
    int32_t tile_size;  /* chosen seed tile size */
    int32_t schedule;   /* chosen schedule */
    double ms_per_step; /* its trial time */
    int32_t timed;      /* (tile size, schedule) pairs timed */
    int32_t skipped;    /* tile sizes not timed (not runnable, beyond the LDS, or the model) */
} dgt_autotune_result;
dgt_status dgt_solver_autotune(dgt_solver *s, const dgt_autotune_params *p, dgt_autotune_result *out);
/* The schedule of the last dgt_solver_inspect (borrowed; NULL before). */
dgt_status dgt_solver_schedule(const dgt_solver *s, const dgt_schedule **out);
/* Ricker point source on sxx and syy: r(t) = amp (1 - 2 a) exp(-a),
 * a = (pi f0 (t - t0))^2, placed in the lowest-id cell containing (x, y); with
 * several shots, every shot gets this source. */
dgt_status dgt_set_source(dgt_solver *s, double x, double y, double f0, double t0, double amp);
/* Shots: nshots (1..65536) independent states advanced together on this mesh
 * (the batched forward run; one shot is the default).  Each shot has its own
 * Ricker point source at (xy[2q], xy[2q+1]) (host, [nshots*2]) with the common
 * wavelet f0, t0, amp, placed as by dgt_set_source; xy NULL: no sources.  The
 * state of every shot is reset to zero and must be uploaded again; the schedule
 * and plan stay (shots share the mesh, its tiles and geometry).  A tiled step
 * runs every (tile, shot) pair as one work item, with the shots of a tile next
 * to each other in the launch order; dgt_step mode 0 runs the shots one after
 * another.  Results of a shot do not depend on the other shots.  EINVAL for a
 * bad count, a non-finite position or one outside the mesh (the solver then has
 * no sources).  Synchronises the stream. */
dgt_status dgt_solver_set_shots(dgt_solver *s, int32_t nshots, const double *xy, double f0, double t0,
                                double amp);
/* Copy the state into / out of the solver (device pointers, caller layout
 * v[nshots][2][Np][nc], s[nshots][3][Np][nc] in the solver precision; enqueued on
 * the stream). */
dgt_status dgt_state_upload(dgt_solver *s, const void *v, const void *sig);
dgt_status dgt_state_download(dgt_solver *s, void *v, void *sig);
/* Halo exchange of a distributed step (Sec. 4, Alg. 2): before a step, each GPU's
 * part receives the state of its exec and non-exec halo cells from the GPUs that
 * own them.  A cell list names cells of one solver's mesh (host ids in the mesh's
 * numbering, each in [0, nc), copied to the device; DGT_EINVAL otherwise);
 * dgt_state_pack copies their state into packed device buffers
 * v[nshots][2][Np][n], sig[nshots][3][Np][n] (solver precision), and
 * dgt_state_unpack copies such buffers into them.  Between GPUs the packed buffers
 * travel by RCCL point-to-point; on one GPU, packing from a solver of the whole
 * mesh and unpacking into the part's halo is the device-to-device fill.  The list
 * must belong to a solver of the same mesh size and device; both calls need an
 * uploaded state and are enqueued on the solver's stream.  An empty list copies
 * nothing (its buffers may be NULL). */
typedef struct dgt_cell_list dgt_cell_list;
dgt_status dgt_cell_list_create(const dgt_solver *s, int64_t n, const int32_t *cells, dgt_cell_list **out);
void dgt_cell_list_destroy(dgt_cell_list *l);
dgt_status dgt_state_pack(dgt_solver *s, const dgt_cell_list *l, void *v, void *sig);
dgt_status dgt_state_unpack(dgt_solver *s, const dgt_cell_list *l, const void *v, const void *sig);
/* Advance nsteps time steps starting at time t0 (sigma at t0, v at t0 - dt/2).
 * mode 0: untiled chain (one kernel per loop); mode 1: sparse-tiled fused
 * executor (requires dgt_solver_inspect).  Enqueued on the stream. */
dgt_status dgt_step(dgt_solver *s, int64_t nsteps, int32_t mode, double t0);
/* Discrete energy 1/2 v'M_rho v + 1/2 sum_K int sig_new : C^-1 sig_old, reduced
 * in FP64 on the GPU.  v, sig_new, sig_old: device, caller layout of one shot,
 * solver precision.  Synchronises the stream. */
dgt_status dgt_energy(dgt_solver *s, const void *v, const void *sig_new, const void *sig_old, double *out);
/* dgt_energy without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and summation order, hence the same value
 * bit for bit.  Its partial sums live in a fixed per-GPU array inside the
 * library, whose address is looked up once per device
 * when the first solver on that device is created; nothing is allocated per
 * call.  Limit: the solver's mesh may have at most 4,194,304 (2^22) cells
 * (the array holds 16,385 doubles, 128 KiB); beyond that DGT_EINVAL with a
 * message.  Every call on one GPU shares that array: calls that overlap on a
 * GPU (several streams or host threads) race and must be serialised by the
 * caller.  Arguments as for dgt_energy; synchronises the stream. */
dgt_status dgt_energy_noalloc(dgt_solver *s, const void *v, const void *sig_new, const void *sig_old, double *out);
/* Full-waveform inversion (an extension beyond the paper's forward chain).
 * Receivers are velocity sensors: receiver r reads sum_i phi_i(x_r) v_i of the
 * lowest-id cell containing x_r, after every time step.  Both calls start from
 * rest at t = 0 with the solver's shots and sources (dgt_solver_set_shots /
 * dgt_set_source), run nsteps steps with the untiled chain (mode 0) or the tiled
 * executor (mode 1, after dgt_solver_inspect, with the solver's schedule), and
 * overwrite the solver's state.  Enqueued on the stream; synchronise on return. */
typedef struct {
    int32_t nrec;           /* receivers, >= 1 */
    const double *rec_xy;   /* host [nrec*2] receiver positions inside the mesh */
    int64_t nsteps;         /* time steps, >= 1 */
    int32_t nsnap;          /* checkpoints of the reversal (dgt_fwi_gradient), >= 1 */
    int32_t mode;           /* 0 untiled, 1 tiled */
} dgt_fwi_params;
/* Receiver traces of the forward run: traces device [nshots][nsteps][nrec][2]
 * FP64 (vx, vy), caller-owned.  EINVAL for bad parameters or a receiver outside
 * the mesh, ESTATE for mode 1 without a usable inspection. */
dgt_status dgt_fwi_forward(dgt_solver *s, const dgt_fwi_params *p, double *traces);
/* Misfit J = 1/2 sum_shots sum_steps sum_receivers |r - d|^2 against observed
 * (device, layout of dgt_fwi_forward) and its gradient with respect to each
 * cell's lambda, mu, rho: g_lam, g_mu, g_rho device [nc] FP64 in the mesh's cell
 * numbering, caller-owned, summed over the shots.  Discrete adjoint of the
 * time-stepped chain; forward states are recomputed from nsnap checkpoints by a
 * binomial reversal schedule; the per-cell terms are accumulated in FP64.  With
 * the central flux and free or periodic boundaries the
 * transposed step is the reversed chain (-dt) on a second solver (same inspection
 * and schedule); with the upwind
 * flux or absorbing sides it is the closed form of the transposed step in the energy
 * inner product (operator parts skew, penalties self-adjoint: the operators run with
 * -dt and the penalties with +dt, each penalty in the other half step), built from
 * untiled operator applications (one cell-centric launch each over all shots), and
 * the gradient adds the derivatives of the flux weights with respect to the
 * impedances of both cells of every facet.  *misfit host.  Environment, read per
 * call: DGT_FWI_CLOSED_FORM takes the closed form also where the reversed chain
 * applies (the two agree); DGT_FWI_UNTILED_INTERMEDIATES computes the reversed
 * chain's intermediates by untiled operator applications instead of recording them
 * from tiled steps. */
dgt_status dgt_fwi_gradient(dgt_solver *s, const dgt_fwi_params *p, const double *observed, double *misfit,
                            double *g_lam, double *g_mu, double *g_rho);
/* Schedule of the tiled executor (default 0).  0: one kernel launch per colour
 * of every sub-chain (Alg. 2's colour loop).  1: sub-chains that run on the
 * chain kernel (whole operator applications) launch once; workgroups take tiles
 * in colour order from a ticket counter and a tile starts when every tile of a
 * lower colour whose footprint meets its own has finished (device-scope
 * counters; field data that can cross tiles is read and written with
 * device-coherent accesses, and each workgroup waits for its stores to
 * complete before it counts its successors), so no colour waits for a whole
 * earlier colour.
 * Every wait is bounded: if one gives up, the next dgt_state_download (which
 * waits for the stream) returns DGT_ESTATE and the counters are reset; a later
 * dgt_step or dgt_state_pack reports it as well once the flags of the failed call
 * have reached the host (they are copied behind each call; neither waits for
 * them).  mode: 0 or 1, else DGT_EINVAL. */
dgt_status dgt_solver_set_schedule(dgt_solver *s, int32_t mode);
/* Polls of a dependence wait (schedule 1) before it gives up, 1..2^32-1; default
 * 2^20 (about a second).  A tiny value makes waits time out on purpose, which
 * exercises the error path (the kernels still exit normally).  DGT_EINVAL
 * outside the range. */
dgt_status dgt_solver_set_wait_limit(dgt_solver *s, int64_t polls);
/* Per-launch timing switch (default off).  When on, the tiled executor of
 * dgt_step records a HIP event pair on the solver stream around every tile
 * kernel launch, so that dgt_last_step_timing reports the time spent inside
 * tile kernels apart from launch gaps.  The events cost a little host time per
 * launch: time throughput with it off.  on: 0 or 1, else DGT_EINVAL. */
dgt_status dgt_solver_profile(dgt_solver *s, int32_t on);
/* Timing of the last dgt_step (HIP events on the solver stream; synchronises
 * with its end event): total_ms from the first to the last kernel of the call;
 * kernel_ms the sum of the tile kernels' durations when per-launch timing was
 * on for a tiled call, else equal to total_ms; launches: kernels launched. */
dgt_status dgt_last_step_timing(const dgt_solver *s, double *total_ms, double *kernel_ms, int64_t *launches);
/* Per-step algorithmic HBM bytes of the fused step (the state of every shot
 * read and written once, cell invariants read once) and the LDS bytes per tile
 * slot. */
dgt_status dgt_solver_info(const dgt_solver *s, int64_t *np, int64_t *bytes_per_step, int64_t *lds_bytes);
void dgt_solver_destroy(dgt_solver *s);

/* ---- Several meshes in one launch (batched forward runs; an extension beyond
 * the paper, which runs one mesh at a time) ---- */
typedef struct dgt_batch dgt_batch;
/* A batch of solvers advanced together by shared launches: one work queue over
 * the (tile, shot) items of all members, ordered by colour and then member, each
 * member's tiles in its own execution order.  Schedule 0 (default): one launch
 * per colour of a sub-chain for all members (Alg. 2's colour loop across meshes),
 * one item per workgroup.  Schedule 1: one launch per sub-chain, workgroups take
 * items from a ticket counter and a tile starts once its lower-colour neighbours
 * of the same member have finished (dgt_solver_set_schedule mode 1, with the
 * batch's own counters).  Members: host [n], 1 <= n <= 4096, distinct, each
 * inspected with a usable plan whose sub-chains all run on the register-resident
 * chain kernel (degrees 1 and 2), sharing degree, precision, flux, time order and
 * fusion scheme (half steps, or the whole order-2 step); they keep their own mesh,
 * material, dt, shots, sources and state and must outlive the batch.  Each item
 * runs the arithmetic of a member's own tiled step, so results equal stepping
 * each member alone to rounding (the batched kernel is compiled on its own;
 * multiply-adds may be contracted differently).  stream: hipStream_t or NULL; the
 * batch also owns a stream for graph replays, joined to it with events.  EINVAL
 * for mismatched members, ESTATE for an uninspected one, EUNSUPPORTED at degrees
 * 3-4.  Synchronises the stream. *out owned by the caller (dgt_batch_destroy). */
dgt_status dgt_batch_create(dgt_solver *const *solvers, int32_t n, void *stream, dgt_batch **out);
/* Schedule of the batch's launches (default 0), as described above; mode 0 or 1,
 * else EINVAL.  A change drops a captured graph. */
dgt_status dgt_batch_set_schedule(dgt_batch *b, int32_t mode);
/* Graph mode: steps_per_graph = G > 0 captures G steps (kernel nodes only, no
 * memory nodes) into a HIP graph at the next dgt_batch_step and replays it
 * floor(nsteps / G) times per call, the remaining steps launched directly; before
 * each replay the batch sets the replay's step offset into the call's source
 * amplitudes and, under schedule 1, clears its counters (outside the graph).
 * 0 (default): direct launches.  0 <= G <= 4096, else EINVAL. */
dgt_status dgt_batch_set_graph(dgt_batch *b, int32_t steps_per_graph);
/* Advance every member nsteps steps, member i from its time t0[i] (host [n]),
 * like dgt_step(member, nsteps, 1, t0[i]).  Enqueued on the stream (the source
 * amplitudes of the call are computed on the host and uploaded first).  ESTATE if
 * a member was inspected again, got new shots, has no state, or an earlier wait
 * timed out (the counters are then reset). */
dgt_status dgt_batch_step(dgt_batch *b, int64_t nsteps, const double *t0);
/* Timing of the last dgt_batch_step (synchronises with its end): ms between HIP
 * events on the stream around the call, kernel launches it made (graph nodes
 * included) and graph replays among them.  Any pointer may be NULL. */
dgt_status dgt_batch_timing(dgt_batch *b, double *ms, int64_t *launches, int64_t *graph_launches);
void dgt_batch_destroy(dgt_batch *b);

/* Tile kernel of each sub-chain of the current plan (after a successful
 * dgt_solver_inspect; *nsub = 0 before): 0 the generic in-LDS executor, 1 the
 * register-resident chain kernel (whole operator applications, one thread per
 * footprint cell), 2 the matrix-core kernel (whole operator applications at
 * degrees 3 and 4, per-cell contractions as 16x16x4 MFMA products), 3 the generic
 * executor with its working set in global memory (tiles beyond the LDS).  kinds:
 * host [*nsub] or NULL.  The environment variable DGT_TILE_OP read at inspection
 * selects 0 (generic everywhere) or 1 (the chain kernel where it is built) instead
 * of the default. */
dgt_status dgt_solver_kernels(const dgt_solver *s, int32_t *nsub, int32_t *kinds);
/* Host copies of the reference-element tables the kernels of degree `degree`
 * (1..4) use (Sec. 7.1: nodal Lagrange P_k on the equispaced nodes of the
 * reference triangle, exact integration; the tables are the exact rationals
 * rounded to double once).  dr, ds: [Np*Np], D[i*Np+j] = d phi_j / dr (ds) at
 * node i; minv: [Np*Np] inverse reference mass; lift: [3][Np][k+1], the inverse
 * mass times facet f's mass matrix.  Any pointer may be NULL.  No device work;
 * EINVAL for a degree outside 1..4. */
dgt_status dgt_refelem(int32_t degree, double *dr, double *ds, double *minv, double *lift);

#ifdef __cplusplus
}
#endif
#endif /* DGTILE_H */
