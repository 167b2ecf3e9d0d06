// DG elastic solver object of libdgtile (tier 2 of the C ABI): set-up, the DG
// loop chain handed to the GPU inspector, the executor plan, and the step,
// state and energy entry points.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>

#include "dg_device.h"
#include "tile_chain.h"
#include "tile_exec.h"

namespace dgt {

struct GLoop {
    int8_t kind, in, out, pen;
    double scale, pscale;
    int set;   // 0 cells, 1 interior facets, 2 exterior facets
    int step;  // time step of the loop in a chain fused over several steps
};

struct SubPlan {
    int first = 0, n = 0, ntiles = 0, ncolors = 0;
    // a region-aware schedule never runs its last tile T_ne (the only tile of the
    // last colour): colours [0, nexec_colors) hold the nexec tiles that run
    int tne = -1, nexec = 0, nexec_colors = 0;
    int step0 = 0;  // step of the first loop within a chain fused over steps
    int64_t gmem_bytes = 0;  // working set per workgroup in global scratch (0: in LDS)
    DBuf<char> gmem;         // the scratch of the largest colour launch
    DBuf<int32_t> efoot;
    DBuf<uint32_t> eacc;
    DBuf<uint32_t> lmap[31];
    DBuf<uint32_t> tnb;
    DBuf<int32_t> tnb_off;
    DBuf<int32_t> tmeta;  // [ntiles][4] in colour order: tile, first slot, footprint length, table offset
    std::vector<int32_t> color_off;
    TileArgs args{};
    size_t lds_bytes = 0;
    int max_foot = 0;
    int threads = 256;
    TileKernel kind = TK_GENERIC;  // chain kernel for sub-chains of whole operator applications
    int o0 = 0, nops = 0;  // chain kernel: operators of the sub-chain
    // dependence-driven schedule (built on first use)
    bool graph = false;
    DBuf<int32_t> err;
    DBuf<uint32_t> cnt, head;
    uint32_t epoch = 0;
    int slots = 0;  // workgroups of the tile kernel the whole GPU holds at once
};

}  // namespace dgt

struct dgt_solver {
    const dgt::Mesh *mesh = nullptr;
    const dgt_mesh *mesh_handle = nullptr;
    dgt_solver_params p{};
    hipStream_t st = nullptr;
    int dev = 0;  // device current at creation (the stream's device)
    dgt::RefElem E;
    int K = 1, fp32 = 0, upw = 0, haspen = 0;
    int64_t nc = 0, nf = 0, nb = 0;
    size_t esz = 8;
    // input-order mesh and material on the device
    dgt::DBuf<double> xy, lam, mu, rho;
    dgt::DBuf<int32_t> c2v, f2c, b2c;
    dgt::DBuf<int8_t> f2l, b2l;
    dgt::DBuf<uint8_t> bfree;
    // exec order
    std::vector<int32_t> rank_h;
    dgt::DBuf<int32_t> rank;
    dgt::DBuf<char> geo, fld[dgt::F_COUNT], G, Gx, tmp;
    dgt::DBuf<int32_t> ef2c, eb2c, c2f;
    dgt::DBuf<uint8_t> ef2l, eb2l;
    bool state_valid = false;
    int sched_mode = 0;  // tiled executor: 0 one launch per colour, 1 dependence-driven
    uint32_t wait_limit = 1u << 20;  // polls before a dependence wait gives up
    // shots: independent states on this mesh, each with its own point source (one
    // Ricker wavelet for all) or none
    int32_t nshots = 1;
    bool has_src = false;
    std::vector<int64_t> src_in;       // [nshots] mesh cell holding each source
    std::vector<int32_t> src_exec_h;   // [nshots] its exec id
    double sf0 = 0, st0 = 0, samp = 0;
    dgt::DBuf<char> src_vec;           // [nshots][Np] inverse mass times the basis at the source
    dgt::DBuf<int32_t> src_cells;      // [nshots] exec ids, -1 without sources
    int64_t fshot(int f) const { return (int64_t)dgt::field_ncomp(f) * E.np * nc; }
    // chain, schedule, plan
    std::vector<dgt::GLoop> loops;
    int fuse = 1;  // time steps in the chain handed to the inspector
    dgt_chain chain;
    dgt_schedule *sched = nullptr;
    std::vector<dgt::SubPlan> plan;
    dgt_status plan_status = DGT_ESTATE;  // why the tiled executor cannot run (DGT_OK when it can)
    // parameters of the last inspection (the FWI adjoint solver repeats it)
    bool inspected = false;
    uint64_t gen = 0;  // counts inspections and field reallocations (batches built on this solver check it)
    dgt_inspect_params last_ip{};
    std::vector<int32_t> last_splits, last_sub_ts;
    std::vector<uint8_t> last_region;  // seed regions of the last inspection (empty: none)
    int last_cap = 0;
    std::string plan_error = "tiled mode needs dgt_solver_inspect";
    // error flags of the dependence-driven launches, copied to pinned memory after each
    // tiled call and read once the copy has landed (no wait on the next call)
    int32_t *err_host = nullptr;  // [kMaxLoops]
    hipEvent_t err_ev = nullptr;
    bool err_pending = false;
    // timing of the last step
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0;
    int64_t last_launches = 0;
    // per-launch timing of the tile kernels (event pairs of the last tiled call)
    bool prof = false;
    std::vector<hipEvent_t> pev;
    size_t npev = 0;
    void mark() {
        if (!prof) return;
        if (npev == pev.size()) {
            hipEvent_t e;
            DGT_HIP(hipEventCreate(&e));
            pev.push_back(e);
        }
        DGT_HIP(hipEventRecord(pev[npev++], st));
    }
    ~dgt_solver() {
        for (auto e : pev) (void)hipEventDestroy(e);
        delete sched;
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (err_ev) (void)hipEventDestroy(err_ev);
        if (err_host) (void)hipHostFree(err_host);
    }
};

namespace dgt {

// ------------------------------------------------------------ dispatch helpers

template <class F>
static void dispatch(const dgt_solver *s, F &&f) {
    switch (s->K * 2 + s->fp32) {
    case 2: f.template operator()<1, double>(); break;
    case 3: f.template operator()<1, float>(); break;
    case 4: f.template operator()<2, double>(); break;
    case 5: f.template operator()<2, float>(); break;
    case 6: f.template operator()<3, double>(); break;
    case 7: f.template operator()<3, float>(); break;
    case 8: f.template operator()<4, double>(); break;
    case 9: f.template operator()<4, float>(); break;
    default: throw Error{DGT_EINVAL, "unsupported degree"};
    }
}

static double ricker(double t, double f0, double t0, double amp) {
    const double a = M_PI * M_PI * f0 * f0 * (t - t0) * (t - t0);
    return amp * (1.0 - 2.0 * a) * std::exp(-a);
}

// ------------------------------------------------------------ chain of the DG step

static void build_loops(dgt_solver *s) {
    auto &L = s->loops;
    L.clear();
    const double dt = s->p.dt, c3 = dt * dt * dt / 24.0;
    auto app = [&](bool vel, int in, int out, double sc, int pen, double ps) {
        L.push_back({(int8_t)(vel ? KV_VOL_V : KV_VOL_S), (int8_t)in, (int8_t)out, -1, sc, 0.0, 0});
        L.push_back({(int8_t)(vel ? KV_INT_V : KV_INT_S), (int8_t)in, (int8_t)out, (int8_t)pen, sc, ps, 1});
        L.push_back({(int8_t)(vel ? KV_EXT_V : KV_EXT_S), (int8_t)in, (int8_t)out, (int8_t)pen, sc, ps, 2});
    };
    auto solve = [&](int f) { L.push_back({KV_SOLVE, (int8_t)f, (int8_t)f, -1, 0.0, 0.0, 0}); };
    const int penv = s->haspen ? F_V : -1, pens = s->haspen ? F_S : -1;
    if (s->p.time_order == 4) {
        // velocity half step: U = A s; X = B U; Z = dt^3/24 A X + dt D_v v; v += dt U + Z
        app(true, F_S, F_U, 1.0, -1, 0.0);
        solve(F_U);
        app(false, F_U, F_X, 1.0, -1, 0.0);
        solve(F_X);
        app(true, F_X, F_Z, c3, penv, dt);
        solve(F_Z);
        L.push_back({KV_UPD_V, -1, F_V, -1, dt, 0.0, 0});
        // stress half step: X = B v; U = A X; Z = dt^3/24 B U + dt D_s s; s += dt X + Z + source
        app(false, F_V, F_X, 1.0, -1, 0.0);
        solve(F_X);
        app(true, F_X, F_U, 1.0, -1, 0.0);
        solve(F_U);
        app(false, F_U, F_Z, c3, pens, dt);
        solve(F_Z);
        L.push_back({KV_UPD_S, -1, F_S, -1, dt, 0.0, 0});
    } else {
        app(true, F_S, F_Z, dt, penv, dt);
        L.push_back({KV_UPD2_V, -1, F_V, -1, dt, 0.0, 0});
        app(false, F_V, F_Z, dt, pens, dt);
        L.push_back({KV_UPD2_S, -1, F_S, -1, dt, 0.0, 0});
    }
    // a chain fused over several time steps repeats the step's loops
    const size_t per = L.size();
    for (int r = 1; r < s->fuse; ++r)
        for (size_t j = 0; j < per; ++j) {
            GLoop g = L[j];
            g.step = r;
            L.push_back(g);
        }
    // the loop chain seen by the inspector: sets C, F, B; maps f2c, b2c
    dgt::ChainDesc &c = s->chain.c;
    c = dgt::ChainDesc();
    c.nsets = 3;
    c.size[0] = s->nc;
    c.size[1] = s->nf;
    c.size[2] = s->nb;
    c.nmaps = 2;
    c.maps[0].from = 1;
    c.maps[0].to = 0;
    c.maps[0].arity = 2;
    c.maps[0].values = s->mesh->f2c;
    c.maps[1].from = 2;
    c.maps[1].to = 0;
    c.maps[1].arity = 1;
    c.maps[1].values = s->mesh->b2c;
    c.nloops = (int)L.size();
    for (size_t j = 0; j < L.size(); ++j) {
        ChainLoop &cl = c.loops[j];
        const GLoop &g = L[j];
        cl.set = g.set;
        const int mp = g.set == 0 ? -1 : g.set - 1;
        int nd = 0;
        auto add = [&](int m, int mode, int data) { cl.d[nd++] = dgt_desc{m, mode, data}; };
        switch (g.kind) {
        case KV_VOL_V: case KV_VOL_S: case KV_SOLVE:
            add(-1, DGT_R, g.in);
            add(-1, DGT_W, g.out);
            break;
        case KV_INT_V: case KV_INT_S: case KV_EXT_V: case KV_EXT_S:
            add(mp, DGT_R, g.in);
            add(mp, DGT_INC, g.out);
            if (g.pen >= 0) add(mp, DGT_R, g.pen);
            break;
        default: {  // updates
            const bool vel = g.kind == KV_UPD_V || g.kind == KV_UPD2_V;
            add(-1, DGT_R, F_Z);
            if (g.kind == KV_UPD_V) add(-1, DGT_R, F_U);
            if (g.kind == KV_UPD_S) add(-1, DGT_R, F_X);
            add(-1, DGT_R, vel ? F_V : F_S);
            add(-1, DGT_W, vel ? F_V : F_S);
        }
        }
        cl.ndesc = nd;
    }
}

// ------------------------------------------------------------ exec order

// caller layout v[nshots][2][Np][nc], sg[nshots][3][Np][nc] in the mesh's numbering
static void to_caller(dgt_solver *s, void *v, void *sg) {
    dispatch(s, [&]<int K, typename T>() {
        constexpr int NP = np_of(K);
        const int64_t nv = 2 * NP * s->nc, ns = 3 * NP * s->nc;
        for (int q = 0; q < s->nshots; ++q) {
            k_permute_rows<T><<<blocks_for(nv, 256), 256, 0, s->st>>>(
                (const T *)s->fld[F_V].p + q * nv, (T *)v + q * nv, s->rank.p, 2 * NP, s->nc, 0);
            k_permute_rows<T><<<blocks_for(ns, 256), 256, 0, s->st>>>(
                (const T *)s->fld[F_S].p + q * ns, (T *)sg + q * ns, s->rank.p, 3 * NP, s->nc, 0);
        }
    });
}

static void from_caller(dgt_solver *s, const void *v, const void *sg) {
    dispatch(s, [&]<int K, typename T>() {
        constexpr int NP = np_of(K);
        const int64_t nv = 2 * NP * s->nc, ns = 3 * NP * s->nc;
        for (int q = 0; q < s->nshots; ++q) {
            k_permute_rows<T><<<blocks_for(nv, 256), 256, 0, s->st>>>(
                (const T *)v + q * nv, (T *)s->fld[F_V].p + q * nv, s->rank.p, 2 * NP, s->nc, 1);
            k_permute_rows<T><<<blocks_for(ns, 256), 256, 0, s->st>>>(
                (const T *)sg + q * ns, (T *)s->fld[F_S].p + q * ns, s->rank.p, 3 * NP, s->nc, 1);
        }
    });
}

// exec ids of the source cells (the executors compare a cell's exec id with them)
static void set_source_exec(dgt_solver *s) {
    s->src_exec_h.assign(s->nshots, -1);
    if (s->has_src)
        for (int q = 0; q < s->nshots; ++q) s->src_exec_h[q] = s->rank_h[s->src_in[q]];
    s->src_cells.upload(s->src_exec_h, s->st);
    DGT_HIP(hipStreamSynchronize(s->st));
}

// fields for every shot, zeroed
static void alloc_fields(dgt_solver *s) {
    ++s->gen;
    for (int f = 0; f < F_COUNT; ++f) {
        s->fld[f].alloc((size_t)s->fshot(f) * s->nshots * s->esz);
        DGT_HIP(hipMemsetAsync(s->fld[f].p, 0, s->fld[f].n, s->st));
    }
}

static void set_exec_order(dgt_solver *s, const std::vector<int32_t> &rank) {
    hipStream_t st = s->st;
    const int64_t nc = s->nc, nf = s->nf, nb = s->nb;
    const int np = s->E.np;
    // keep any state across the renumbering
    DBuf<char> keep;
    if (s->state_valid) {
        keep.alloc(5 * np * nc * s->esz * s->nshots);
        to_caller(s, keep.p, keep.p + 2 * np * nc * s->esz * s->nshots);
    }
    s->rank_h = rank;
    s->rank.upload(rank, st);
    dispatch(s, [&]<int K, typename T>() {
        k_geometry<T><<<blocks_for(nc, 256), 256, 0, st>>>(s->xy.p, s->c2v.p, s->lam.p, s->mu.p, s->rho.p,
                                                          s->rank.p, nc, (T *)s->geo.p);
    });
    // untiled maps in exec numbering; facets ordered by their lower exec cell
    const auto &M = *s->mesh;
    // (counting sorts by exec cell, stable in the mesh's facet order)
    auto counting_order = [nc](int64_t n, auto key) {
        std::vector<int64_t> start(nc + 1, 0), ord(n);
        for (int64_t i = 0; i < n; ++i) start[key(i) + 1]++;
        for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
        for (int64_t i = 0; i < n; ++i) ord[start[key(i)]++] = i;
        return ord;
    };
    const std::vector<int64_t> ford = counting_order(
        nf, [&](int64_t f) { return std::min(rank[M.f2c[2 * f]], rank[M.f2c[2 * f + 1]]); });
    std::vector<int32_t> ef2c(2 * std::max<int64_t>(nf, 1)), c2f(3 * std::max<int64_t>(nc, 1), INT32_MIN);
    std::vector<uint8_t> ef2l(std::max<int64_t>(nf, 1));
    for (int64_t e = 0; e < nf; ++e) {
        const int64_t f = ford[e];
        const int32_t x0 = rank[M.f2c[2 * f]], x1 = rank[M.f2c[2 * f + 1]];
        ef2c[2 * e] = x0;
        ef2c[2 * e + 1] = x1;
        ef2l[e] = (uint8_t)(M.f2l[2 * f] | (M.f2l[2 * f + 1] << 2));
        c2f[(int64_t)M.f2l[2 * f] * nc + x0] = (int32_t)(2 * e);
        c2f[(int64_t)M.f2l[2 * f + 1] * nc + x1] = (int32_t)(2 * e + 1);
    }
    const std::vector<int64_t> bord = counting_order(nb, [&](int64_t b) { return rank[M.b2c[b]]; });
    std::vector<int32_t> eb2c(std::max<int64_t>(nb, 1));
    std::vector<uint8_t> eb2l(std::max<int64_t>(nb, 1));
    for (int64_t e = 0; e < nb; ++e) {
        const int64_t b = bord[e];
        const int32_t x = rank[M.b2c[b]];
        const bool fr = M.bside[b] >= 0 && ((s->p.free_sides >> M.bside[b]) & 1);
        eb2c[e] = x;
        eb2l[e] = (uint8_t)(M.b2l[b] | (fr ? 4 : 0));
        c2f[(int64_t)M.b2l[b] * nc + x] = (int32_t)(-(e + 1));
    }
    for (int64_t i = 0; i < 3 * nc; ++i)
        DGT_REQUIRE(c2f[i] != INT32_MIN, DGT_EINVAL, "a cell facet is neither interior nor exterior");
    s->ef2c.upload(ef2c, st);
    s->ef2l.upload(ef2l, st);
    s->eb2c.upload(eb2c, st);
    s->eb2l.upload(eb2l, st);
    s->c2f.upload(c2f, st);
    DGT_HIP(hipStreamSynchronize(st));
    set_source_exec(s);
    if (s->state_valid) from_caller(s, keep.p, keep.p + 2 * np * nc * s->esz * s->nshots);
    DGT_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------------ executor plan (local maps, LDS plan)

static void build_plan(dgt_solver *s) {
    hipStream_t st = s->st;
    const dgt::Schedule &S = *s->sched->s;
    s->plan.clear();
    s->plan.resize(S.sub.size());
    int dev = 0;
    DGT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    DGT_HIP(hipGetDeviceProperties(&prop, dev));
    const size_t budget = std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024) - 256;  // room for static LDS
    const int np = s->E.np;
    // fields touched by each sub-chain, for persistence across sub-chains
    std::vector<int> used(S.sub.size(), 0);
    auto fields_of = [&](const GLoop &g) {
        int m = 0;
        if (g.kind == KV_SOLVE) return 0;
        if (g.in >= 0) m |= 1 << g.in;
        if (g.out >= 0) m |= 1 << g.out;
        if (g.pen >= 0) m |= 1 << g.pen;
        if (g.kind == KV_UPD_V) m |= (1 << F_V) | (1 << F_U) | (1 << F_Z);
        if (g.kind == KV_UPD2_V) m |= (1 << F_V) | (1 << F_Z);
        if (g.kind == KV_UPD_S) m |= (1 << F_S) | (1 << F_X) | (1 << F_Z);
        if (g.kind == KV_UPD2_S) m |= (1 << F_S) | (1 << F_Z);
        return m;
    };
    for (size_t b = 0; b < S.sub.size(); ++b)
        for (int j = S.sub[b].first; j < S.sub[b].first + S.sub[b].n; ++j) used[b] |= fields_of(s->loops[j]);
    for (size_t b = 0; b < S.sub.size(); ++b) {
        const SubSched &sb = S.sub[b];
        SubPlan &P = s->plan[b];
        P.first = sb.first;
        P.n = sb.n;
        P.ntiles = sb.ntiles;
        P.ncolors = sb.ncolors;
        P.color_off = sb.color_off.download(st, sb.ncolors + 1);
        P.tne = sb.tne;
        P.nexec_colors = sb.tne >= 0 ? sb.ncolors - 1 : sb.ncolors;
        P.nexec = P.color_off[P.nexec_colors];
        // footprints renumbered into exec order, sorted per tile
        const int64_t len = sb.foot_len[0];
        DGT_REQUIRE(len > 0 || s->nc == 0, DGT_ESTATE, "empty cell footprint");
        {
            DBuf<uint64_t> keys(std::max<int64_t>(len, 1));
            DBuf<uint32_t> vals(std::max<int64_t>(len, 1));
            if (len) {
                k_rank_keys<<<blocks_for(len, 256), 256, 0, st>>>(sb.foot_off[0].p, sb.foot[0].p, s->rank.p,
                                                                  sb.ntiles, len, keys.p);
                DGT_HIP(hipMemcpyAsync(vals.p, sb.acc[0].p, sizeof(uint32_t) * len, hipMemcpyDeviceToDevice, st));
                sort_pairs(keys, vals, len, st);
            }
            P.efoot.alloc(std::max<int64_t>(len, 1));
            if (len) k_split_keys<<<blocks_for(len, 256), 256, 0, st>>>(keys.p, len, P.efoot.p);
            P.eacc = std::move(vals);
        }
        auto foff = sb.foot_off[0].download(st, sb.ntiles + 1);
        for (int t = 0; t < sb.ntiles; ++t)
            if (t != sb.tne) P.max_foot = std::max(P.max_foot, foff[t + 1] - foff[t]);
        DGT_REQUIRE(P.max_foot <= 0x3fff, DGT_EUNSUPPORTED, "tile footprint exceeds 16383 cells");
        // local maps of the facet loops (cell loops take their iterations from the footprint's loop bits)
        DBuf<int32_t> err(1);
        DGT_HIP(hipMemsetAsync(err.p, 0, 4, st));
        for (int j = sb.first; j < sb.first + sb.n; ++j) {
            const int64_t n = S.loop_size[j];
            const int kind = s->loops[j].set;
            if (kind == 0) continue;
            auto &lm = P.lmap[j - sb.first];
            lm.alloc(std::max<int64_t>(n, 1));
            if (n)
                k_lmap<<<blocks_for(n, 256), 256, 0, st>>>(kind, S.it_off[j].p, S.iters[j].p, sb.ntiles, sb.tne, n,
                                                           sb.foot_off[0].p, P.efoot.p, s->rank.p, s->f2c.p,
                                                           s->f2l.p, s->b2c.p, s->b2l.p, s->bfree.p, lm.p, err.p);
        }
        DGT_REQUIRE(err.download(st)[0] == 0, DGT_ESTATE, "local map construction failed");
        // per-field access table of this sub-chain
        TileArgs &A = P.args;
        std::memset(&A, 0, sizeof(A));
        A.nloops = sb.n;
        for (int f = 0; f < F_COUNT; ++f) A.lds_row[f] = -1;
        int rows = 0;
        for (int f = 0; f < F_COUNT; ++f)
            if ((used[b] >> f) & 1) {
                A.lds_row[f] = rows;
                rows += field_ncomp(f) * np;
            }
        A.nrow = rows + G_NROWS;
        if (!(A.nrow & 1)) ++A.nrow;  // odd slot stride: consecutive slots fall in different LDS banks
        // a field written here is kept (written back for every cell) unless the next sub-chain
        // that uses it, cyclically over steps, starts by overwriting it in a volume loop
        A.persistent_mask = (1 << F_V) | (1 << F_S);
        for (int f = 0; f < F_COUNT; ++f) {
            if (!((used[b] >> f) & 1)) continue;
            bool live = true;
            for (size_t d = 1; d <= S.sub.size(); ++d) {
                const SubSched &nx = S.sub[(b + d) % S.sub.size()];
                if (!((used[(b + d) % S.sub.size()] >> f) & 1)) continue;
                for (int j = nx.first; j < nx.first + nx.n; ++j) {
                    const int m = fields_of(s->loops[j]);
                    if (!((m >> f) & 1)) continue;
                    const GLoop &g = s->loops[j];
                    live = !((g.kind == KV_VOL_V || g.kind == KV_VOL_S) && g.out == f);
                    break;
                }
                break;
            }
            if (live) A.persistent_mask |= 1 << f;
        }
        // facet loops with their neighbour tables: an interior loop and the exterior loop that
        // follows it with the same operands share one table and run in one pass
        std::vector<std::vector<int>> groups;
        for (int i = 0; i < sb.n; ++i) {
            const GLoop &g = s->loops[sb.first + i];
            TLoop &t = A.loops[i];
            t.kind = g.kind;
            t.in = g.in;
            t.out = g.out;
            t.step = (int8_t)(g.step - s->loops[sb.first].step);
            t.pen = g.pen;
            t.partner = -1;
            t.grp = -1;
            if (g.set != 0 && !(i > 0 && A.loops[i - 1].partner == i)) {
                t.grp = (int8_t)groups.size();
                groups.push_back({i});
                if ((g.kind == KV_INT_V || g.kind == KV_INT_S) && i + 1 < sb.n) {
                    const GLoop &h = s->loops[sb.first + i + 1];
                    if (h.set == 2 && h.in == g.in && h.out == g.out && h.pen == g.pen) {
                        t.partner = (int8_t)(i + 1);
                        groups.back().push_back(i + 1);
                    }
                }
            }
            t.scale_d = g.scale;
            t.pscale_d = g.pscale;
            t.scale_f = (float)g.scale;
            t.pscale_f = (float)g.pscale;
            const uint32_t bit = 1u << i;
            auto acc = [&](int f, int mode) {  // mode 1 R, 2 W, 3 RW
                if (f < 0) return;
                A.loops_mask[f] |= bit;
                if (mode & 1) A.rfirst_mask[f] |= bit;
                if (mode & 2) A.writes_mask[f] |= bit;
            };
            switch (g.kind) {
            case KV_VOL_V: case KV_VOL_S: acc(g.in, 1); acc(g.out, 2); break;
            case KV_INT_V: case KV_INT_S: case KV_EXT_V: case KV_EXT_S: acc(g.in, 1); acc(g.out, 3); acc(g.pen, 1); break;
            case KV_UPD_V: acc(F_V, 3); acc(F_U, 1); acc(F_Z, 1); break;
            case KV_UPD2_V: acc(F_V, 3); acc(F_Z, 1); break;
            case KV_UPD_S: acc(F_S, 3); acc(F_X, 1); acc(F_Z, 1); break;
            case KV_UPD2_S: acc(F_S, 3); acc(F_Z, 1); break;
            default: break;
            }
        }
        A.nfl = (int32_t)groups.size();
        A.foot_off = sb.foot_off[0].p;
        A.foot = P.efoot.p;
        A.facc = P.eacc.p;
        A.tiles = sb.tiles_by_color.p;
        for (int f = 0; f < F_COUNT; ++f) A.F[f] = s->fld[f].p;
        A.geo = s->geo.p;
        A.nc = s->nc;
        A.stride = std::max(P.max_foot, 1);
        A.src_vec = s->src_vec.p;
        A.src_cells = s->src_cells.p;
        A.nshots = s->nshots;
        for (int f = 0; f < F_COUNT; ++f) A.fshot[f] = s->fshot(f);
        // neighbour tables: for each tile, facet group, local facet and footprint slot, the
        // neighbour's slot and local facet (interior) or the boundary kind (exterior)
        {
            std::vector<std::vector<int32_t>> offs(sb.n);
            std::vector<std::vector<uint32_t>> maps(sb.n);
            for (auto &gr : groups)
                for (int i : gr) {
                    const int j = sb.first + i;
                    offs[i] = S.it_off[j].download(st, sb.ntiles + 1);
                    maps[i] = P.lmap[i].download(st, S.loop_size[j]);
                }
            std::vector<int32_t> toff(sb.ntiles + 1, 0);
            for (int t = 0; t < sb.ntiles; ++t) {
                const int64_t len = t == sb.tne ? 0 : (int64_t)A.nfl * 3 * (foff[t + 1] - foff[t]);
                DGT_REQUIRE(toff[t] + len < INT32_MAX, DGT_EUNSUPPORTED, "neighbour tables exceed 2^31 entries");
                toff[t + 1] = (int32_t)(toff[t] + len);
            }
            std::vector<uint32_t> tab(std::max<int32_t>(toff[sb.ntiles], 1), 0u);
            bool dup = false;
            for (int t = 0; t < sb.ntiles; ++t) {
                if (t == sb.tne) continue;  // never executed: no neighbour tables
                const int nfoot = foff[t + 1] - foff[t];
                for (int gi = 0; gi < A.nfl; ++gi) {
                    uint32_t *T3 = tab.data() + toff[t] + (size_t)gi * 3 * nfoot;
                    auto put = [&](int l, int sl, uint32_t code) {
                        uint32_t &e = T3[(size_t)l * nfoot + sl];
                        dup |= (e != 0u);
                        e = code;
                    };
                    for (int i : groups[gi]) {
                        const bool interior = s->loops[sb.first + i].set == 1;
                        for (int q = offs[i][t]; q < offs[i][t + 1]; ++q) {
                            const uint32_t c = maps[i][q];
                            if (interior) {
                                const int s0 = c & 0x3fff, s1 = (c >> 14) & 0x3fff, l0 = (c >> 28) & 3, l1 = (c >> 30) & 3;
                                put(l0, s0, NB_VALID | (uint32_t)s1 | ((uint32_t)l1 << 14));
                                put(l1, s1, NB_VALID | (uint32_t)s0 | ((uint32_t)l0 << 14));
                            } else {
                                const int s0 = c & 0x3fff, l = (c >> 28) & 3;
                                put(l, s0, NB_VALID | NB_BND | (((c >> 30) & 1) ? NB_FREE : 0u) | (uint32_t)s0);
                            }
                        }
                    }
                }
            }
            DGT_REQUIRE(!dup, DGT_ESTATE, "a cell facet appears twice in one facet loop of a tile");
            P.tnb.upload(tab, st);
            P.tnb_off.upload(toff, st);
            {
                const std::vector<int32_t> byc = sb.tiles_by_color.download(st, sb.ntiles);
                std::vector<int32_t> meta(4 * std::max<int32_t>(sb.ntiles, 1), 0);
                for (int i = 0; i < sb.ntiles; ++i) {
                    const int t = byc[i];
                    meta[4 * i] = t;
                    meta[4 * i + 1] = foff[t];
                    meta[4 * i + 2] = foff[t + 1] - foff[t];
                    meta[4 * i + 3] = toff[t];
                }
                P.tmeta.upload(meta, st);
                A.tmeta = P.tmeta.p;
            }
            A.tnb = P.tnb.p;
            A.tnb_off = P.tnb_off.p;
            for (int i = 0; i < sb.n; ++i) P.lmap[i].release();
        }
        P.lds_bytes = (size_t)A.nrow * A.stride * s->esz + (size_t)A.stride * (4 + 4 + 2) +
                      (size_t)A.nfl * 3 * A.stride * 4 + 16;
        // a sub-chain of whole consecutive operator applications (each with its update, the
        // last one's optional) runs on the chain kernel
        {
            // operators are numbered on across the steps of a fused chain
            const int order = s->p.time_order, nop = ops_per_step(order) * s->fuse;
            int o = 0;
            while (o < nop && op_first_loop(order, o) != sb.first) ++o;
            const int first_op = o;
            P.step0 = s->loops[sb.first].step;  // also for sub-chains that start inside an operator
            int j = sb.first;
            const int end = sb.first + sb.n;
            bool ok = o < nop;
            while (ok && j < end && o < nop) {
                const OpDesc D = op_desc(order, o);
                const GLoop *g = &s->loops[j];
                ok = j + 3 <= end && g[0].kind == (D.vel ? KV_VOL_V : KV_VOL_S) && g[0].in == D.in &&
                     g[0].out == D.out && g[1].kind == (D.vel ? KV_INT_V : KV_INT_S) &&
                     g[2].kind == (D.vel ? KV_EXT_V : KV_EXT_S) && A.loops[j - sb.first + 1].partner == j - sb.first + 2;
                if (!ok) break;
                j += 3;
                if (order == 4) {
                    ok = j < end && s->loops[j].kind == KV_SOLVE;
                    ++j;
                }
                if (ok && D.upd && j < end) {
                    const int k = s->loops[j].kind;
                    ok = D.vel ? (k == KV_UPD_V || k == KV_UPD2_V) : (k == KV_UPD_S || k == KV_UPD2_S);
                    ++j;
                }
                ++o;
            }
            const int nops = o - first_op;
            bool known = false;
            for (const auto &c : TILE_CHAINS)
                known |= c[0] == order && c[1] == first_op % ops_per_step(order) && c[2] == nops;
            const bool whole = ok && j == end && known && A.nfl == nops;
            const int cap = s->K == 4 && s->esz == 8 ? TILE_NT[1] : TILE_NT[2];
            // DGT_TILE_OP: 0 forces the generic kernel, 1 the register-resident chain kernel
            // where it is built (at P3/P4 the matrix-core kernel is the default)
            const char *env = std::getenv("DGT_TILE_OP");
            const int force = env ? std::atoi(env) : -1;
            // at P1/P2 with the upwind flux the chain kernel also holds the reference
            // element in static LDS
            const size_t refb = s->K <= 2 && s->upw
                                    ? (size_t)(3 * np * np + 3 * np * (s->K + 1)) * s->esz + 3 * (s->K + 1) * 4 + 16
                                    : 0;
            if (whole && force != 0 && force != 1 && mfma_built(s->K, order, nops)) {
                // matrix-core kernel: LDS regions [component][node][slot] for the fields an
                // operator reads through a facet (operand, active penalty), a region reused
                // once its field is dead; then the geometry rows and the per-slot words
                int S16 = (std::max(P.max_foot, 1) + 15) & ~15;
                if (S16 % 64 == 0) S16 += 16;  // consecutive node rows start in different banks
                int first[F_COUNT], last[F_COUNT];
                bool res[F_COUNT] = {};
                for (int f = 0; f < F_COUNT; ++f) first[f] = -1, last[f] = -1;
                for (int q = first_op; q < first_op + nops; ++q) {
                    const OpDesc D = op_desc(order, q);
                    const bool pn = D.pen >= 0 && s->loops[op_first_loop(order, q) + 1].pen >= 0;
                    res[D.in] = true;
                    if (pn) res[D.pen] = true;
                    // fields the operator and its update touch (the penalty only when active)
                    uint32_t m = (1u << D.in) | (1u << D.out);
                    if (pn) m |= 1u << D.pen;
                    if (D.upd) m |= 1u << (D.vel ? F_V : F_S);
                    if (D.part >= 0) m |= 1u << D.part;
                    for (int f = 0; f < F_COUNT; ++f) {
                        if (!((m >> f) & 1)) continue;
                        if (first[f] < 0) first[f] = q;
                        last[f] = q;
                    }
                }
                std::vector<std::array<int, 3>> regions;  // row offset, rows, free after op
                int rows = 0;
                // laid out apart from the generic layout, which stays in force when this one
                // does not fit
                int mrow[F_COUNT];
                for (int f = 0; f < F_COUNT; ++f) mrow[f] = -1;
                for (int q = first_op; q < first_op + nops; ++q)
                    for (int f = 0; f < F_COUNT; ++f) {
                        if (!res[f] || first[f] != q) continue;
                        const int need = field_ncomp(f) * np;
                        int pick = -1;
                        for (size_t r = 0; r < regions.size(); ++r)
                            if (regions[r][1] >= need && regions[r][2] < q) { pick = (int)r; break; }
                        if (pick < 0) {
                            regions.push_back({rows, need, last[f]});
                            rows += need;
                            pick = (int)regions.size() - 1;
                        }
                        regions[pick][2] = last[f];
                        mrow[f] = regions[pick][0] * S16;
                    }
                // fields, geometry and facet normals, loop bits, cell ids, flags, neighbour tables
                const size_t bytes = (size_t)(rows + G_NROWS + 9) * S16 * s->esz + (size_t)S16 * (4 + 4 + 2) +
                                     (size_t)nops * 3 * S16 * 4 + 16;
                // the kernel addresses a field's component-node rows with 32-bit offsets
                const bool fits32 = (uint64_t)s->nc * 3 * np < (uint64_t)UINT32_MAX;
                if (bytes <= budget && fits32) {
                    for (int f = 0; f < F_COUNT; ++f) A.lds_row[f] = mrow[f];
                    A.stride = S16;
                    A.nrow = rows * S16;  // geometry rows start here
                    P.kind = TK_MFMA;
                    P.o0 = first_op % ops_per_step(order);
                    P.nops = nops;
                    P.lds_bytes = bytes;
                }
            }
            if (P.kind == TK_GENERIC && whole && chain_built(s->K, nops) && P.max_foot <= cap && force != 0) {
                int w = 0;
                for (int q = first_op; q < first_op + nops; ++q) {
                    const OpDesc D = op_desc(order, q);
                    const bool pn = D.pen >= 0 && s->loops[op_first_loop(order, q) + 1].pen >= 0;
                    w = std::max(w, np * (D.vel ? 3 : 2) + (pn ? np * (D.vel ? 2 : 3) : 0));
                }
                const int nrow = (2 + w) | 1;
                if ((size_t)nrow * A.stride * s->esz + refb <= budget) {
                    A.nrow = nrow;
                    P.kind = TK_CHAIN;
                    P.o0 = first_op % ops_per_step(order);
                    P.nops = nops;
                    P.lds_bytes = (size_t)A.nrow * A.stride * s->esz;
                }
            }
        }
        // a tile whose working set exceeds the LDS runs on the generic kernel with the same
        // working set in a global scratch region per workgroup (L2 / MALL resident)
        P.gmem_bytes = 0;
        if (P.lds_bytes > budget) {
            DGT_REQUIRE(P.kind == TK_GENERIC, DGT_ESTATE, "a specialised tile kernel exceeds the LDS budget");
            P.gmem_bytes = (int64_t)((P.lds_bytes + 255) / 256 * 256);
            P.lds_bytes = 0;
            A.scratch_bytes = P.gmem_bytes;
        }
        // one work item per footprint slot (and node group of the generic kernel)
        const int ng = P.kind == TK_CHAIN || s->K <= 2 ? 1 : (s->K == 3 ? 2 : 3);
        const int items = A.stride * ng;
        P.threads = items <= TILE_NT[0] ? TILE_NT[0] : (items <= TILE_NT[1] ? TILE_NT[1] : TILE_NT[2]);
        if (P.gmem_bytes) P.threads = TILE_NT[2];
        if (P.kind == TK_MFMA) P.threads = MFMA_NT;
        if (const char *e = std::getenv("DGT_TILE_THREADS"); e && P.kind == TK_GENERIC) P.threads = std::atoi(e);
    }
    DGT_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------------ steps

// One operator application of the untiled chain (volume, facet and lift kernels)
// for `shots` fields at once (strides ish, osh, psh between them):
// fout = scale * op(fin) (+ the upwind penalty of fpen scaled by pscale).
template <int K, typename T>
static void apply_op(dgt_solver *s, bool vel, const T *fin, T *fout, double scale, const T *fpen, double pscale,
                     int64_t &launches, int shots = 1, int64_t ish = 0, int64_t osh = 0, int64_t psh = 0) {
    hipStream_t st = s->st;
    const int64_t nc = s->nc, nf = s->nf, nb = s->nb;
    constexpr int NP = np_of(K), NFP = K + 1;
    // facet buffers: one copy per shot
    const int64_t gsh = (int64_t)2 * 3 * NFP * std::max<int64_t>(nf, 1), gxsh = (int64_t)3 * NFP * std::max<int64_t>(nb, 1);
    if (s->G.n < (size_t)(gsh * shots) * sizeof(T)) s->G.alloc((size_t)(gsh * shots) * sizeof(T));
    if (s->Gx.n < (size_t)(gxsh * shots) * sizeof(T)) s->Gx.alloc((size_t)(gxsh * shots) * sizeof(T));
    const T *geo = (const T *)s->geo.p;
    T *G = (T *)s->G.p, *Gx = (T *)s->Gx.p;
    const T sc = (T)scale, ps = (T)pscale;
    const dim3 gc(blocks_for(nc * NP, 256), shots), gf(blocks_for(nf * NFP, 256), shots),
        gb(blocks_for(nb * NFP, 256), shots);
    if (vel) k_vol<K, T, true><<<gc, 256, 0, st>>>(fin, fout, geo, nc, sc, ish, osh);
    else k_vol<K, T, false><<<gc, 256, 0, st>>>(fin, fout, geo, nc, sc, ish, osh);
    ++launches;
    auto fi = [&]<bool VEL, bool UPW, bool PEN>() {
        if (nf) {
            k_flux_int<K, T, VEL, UPW, PEN><<<gf, 256, 0, st>>>(fin, fpen, s->ef2c.p, s->ef2l.p, geo, nc, nf, sc, ps,
                                                                G, ish, psh, gsh);
            ++launches;
        }
        if (nb) {
            k_flux_ext<K, T, VEL, UPW, PEN><<<gb, 256, 0, st>>>(fin, fpen, s->eb2c.p, s->eb2l.p, geo, nc, nb, sc, ps,
                                                                Gx, ish, psh, gxsh);
            ++launches;
        }
    };
    const bool pn = fpen != nullptr;
    if (vel) {
        if (s->upw) { if (pn) fi.template operator()<true, true, true>(); else fi.template operator()<true, true, false>(); }
        else { if (pn) fi.template operator()<true, false, true>(); else fi.template operator()<true, false, false>(); }
        k_lift<K, T, true><<<gc, 256, 0, st>>>(fout, s->c2f.p, G, Gx, nc, nf, nb, osh, gsh, gxsh);
    } else {
        if (s->upw) { if (pn) fi.template operator()<false, true, true>(); else fi.template operator()<false, true, false>(); }
        else { if (pn) fi.template operator()<false, false, true>(); else fi.template operator()<false, false, false>(); }
        k_lift<K, T, false><<<gc, 256, 0, st>>>(fout, s->c2f.p, G, Gx, nc, nf, nb, osh, gsh, gxsh);
    }
    ++launches;
}

// The same operator application in one cell-centric launch (k_op_cell): no facet
// buffers, each cell's facet terms lifted in registers.  The untiled chain keeps the
// per-loop kernels above; this form serves callers that apply single operators to
// arbitrary fields (the FWI reversal).
template <int K, typename T>
static void apply_op_cell(dgt_solver *s, bool vel, const T *fin, T *fout, double scale, const T *fpen,
                          double pscale, int64_t &launches, int shots = 1, int64_t ish = 0, int64_t osh = 0,
                          int64_t psh = 0) {
    const int64_t nc = s->nc;
    if (nc == 0) return;
    const T sc = (T)scale, ps = (T)pscale;
    const dim3 g(blocks_for(nc, 256), shots);
    // exterior-facet kinds come from eb2l, interior neighbours from ef2c / ef2l; a mesh
    // without facets of one kind never reads its (placeholder) table
    auto go = [&]<bool VEL, bool UPW, bool PEN>() {
        k_op_cell<K, T, VEL, UPW, PEN><<<g, 256, 0, s->st>>>(fin, fpen, fout, s->c2f.p, s->ef2c.p, s->ef2l.p,
                                                            s->eb2l.p, (const T *)s->geo.p, nc, sc, ps, ish, osh,
                                                            psh);
    };
    const bool pn = fpen != nullptr;
    if (vel) {
        if (s->upw) { if (pn) go.template operator()<true, true, true>(); else go.template operator()<true, true, false>(); }
        else { if (pn) go.template operator()<true, false, true>(); else go.template operator()<true, false, false>(); }
    } else {
        if (s->upw) { if (pn) go.template operator()<false, true, true>(); else go.template operator()<false, true, false>(); }
        else { if (pn) go.template operator()<false, false, true>(); else go.template operator()<false, false, false>(); }
    }
    ++launches;
}

template <int K, typename T>
static void apply_untiled(dgt_solver *s, int shot, bool vel, int in, int out, double scale, int pen, double pscale,
                          int64_t &launches) {
    apply_op<K, T>(s, vel, (const T *)s->fld[in].p + shot * s->fshot(in), (T *)s->fld[out].p + shot * s->fshot(out),
                   scale, pen >= 0 ? (const T *)s->fld[pen].p + shot * s->fshot(pen) : nullptr, pscale, launches);
}

template <int K, typename T>
static void step_untiled(dgt_solver *s, int64_t nsteps, double t0, int64_t &launches) {
    hipStream_t st = s->st;
    constexpr int NP = np_of(K);
    const int64_t nc = s->nc;
    const double dt = s->p.dt, c3 = dt * dt * dt / 24.0;
    const int penv = s->haspen ? F_V : -1, pens = s->haspen ? F_S : -1;
    for (int q = 0; q < s->nshots; ++q) {  // shots one after another
    T *V = (T *)s->fld[F_V].p + q * s->fshot(F_V), *Sg = (T *)s->fld[F_S].p + q * s->fshot(F_S),
      *U = (T *)s->fld[F_U].p + q * s->fshot(F_U), *X = (T *)s->fld[F_X].p + q * s->fshot(F_X),
      *Z = (T *)s->fld[F_Z].p + q * s->fshot(F_Z);
    const T *sv = (const T *)s->src_vec.p + q * NP;
    for (int64_t n = 0; n < nsteps; ++n) {
        const double th = t0 + ((double)n + 0.5) * dt;
        const double amp = s->has_src ? dt * ricker(th, s->sf0, s->st0, s->samp) : 0.0;
        const int64_t src = s->src_exec_h[q];
        if (s->p.time_order == 4) {
            apply_untiled<K, T>(s, q, true, F_S, F_U, 1.0, -1, 0.0, launches);
            apply_untiled<K, T>(s, q, false, F_U, F_X, 1.0, -1, 0.0, launches);
            apply_untiled<K, T>(s, q, true, F_X, F_Z, c3, penv, dt, launches);
            k_upd_v<T><<<blocks_for(2 * NP * nc, 256), 256, 0, st>>>(V, U, Z, 2 * NP * nc, (T)dt);
            apply_untiled<K, T>(s, q, false, F_V, F_X, 1.0, -1, 0.0, launches);
            apply_untiled<K, T>(s, q, true, F_X, F_U, 1.0, -1, 0.0, launches);
            apply_untiled<K, T>(s, q, false, F_U, F_Z, c3, pens, dt, launches);
            k_upd_s<K, T><<<blocks_for(3 * NP * nc, 256), 256, 0, st>>>(Sg, X, Z, nc, (T)dt, src, (T)amp, sv);
        } else {
            apply_untiled<K, T>(s, q, true, F_S, F_Z, dt, penv, dt, launches);
            k_upd_v<T><<<blocks_for(2 * NP * nc, 256), 256, 0, st>>>(V, nullptr, Z, 2 * NP * nc, (T)dt);
            apply_untiled<K, T>(s, q, false, F_V, F_Z, dt, pens, dt, launches);
            k_upd_s<K, T><<<blocks_for(3 * NP * nc, 256), 256, 0, st>>>(Sg, nullptr, Z, nc, (T)dt, src, (T)amp, sv);
        }
        launches += 2;
    }
    }
}

// Counters of the dependence-driven schedule of one sub-chain (the dependence graph
// itself comes with the inspector's schedule); they start at zero.
static void build_graph(dgt_solver *s, int b, SubPlan &P) {
    hipStream_t st = s->st;
    const SubSched &sb = s->sched->s->sub[b];
    P.cnt.alloc((size_t)sb.ntiles * s->nshots);
    P.head.alloc(1);
    P.err.alloc(1);
    DGT_HIP(hipMemsetAsync(P.cnt.p, 0, sizeof(uint32_t) * sb.ntiles * s->nshots, st));
    DGT_HIP(hipMemsetAsync(P.head.p, 0, sizeof(uint32_t), st));
    DGT_HIP(hipMemsetAsync(P.err.p, 0, sizeof(int32_t), st));
    P.epoch = 0;
    P.graph = true;
}

static void reset_graph(dgt_solver *s, SubPlan &P) {
    DGT_HIP(hipMemsetAsync(P.cnt.p, 0, sizeof(uint32_t) * P.ntiles * s->nshots, s->st));
    DGT_HIP(hipMemsetAsync(P.head.p, 0, sizeof(uint32_t), s->st));
    DGT_HIP(hipMemsetAsync(P.err.p, 0, sizeof(int32_t), s->st));
    P.epoch = 0;
}

// Raises DGT_ESTATE (and resets the counters) when a dependence wait timed out.
// blocking: read the flags now (synchronises the stream).  Otherwise read the copy
// that the last tiled call enqueued, if it has landed; a flag raised later is seen
// by a later call (every wait is bounded, so launches in between end too, with
// invalid results that the error then covers).
static void check_graphs(dgt_solver *s, bool blocking = true) {
    bool bad = false;
    if (blocking) {
        for (auto &P : s->plan) {
            if (!P.graph) continue;
            if (P.err.download(s->st)[0] != 0) {
                bad = true;
                reset_graph(s, P);
            }
        }
        s->err_pending = false;
    } else {
        if (!s->err_pending) return;
        const hipError_t q = hipEventQuery(s->err_ev);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();  // not an error: the copy is still in flight
            return;
        }
        DGT_HIP(q);
        s->err_pending = false;
        for (size_t b = 0; b < s->plan.size() && b < (size_t)kMaxLoops; ++b)
            if (s->plan[b].graph && s->err_host[b] != 0) {
                bad = true;
                reset_graph(s, s->plan[b]);
            }
    }
    if (bad && s->err_host)
        for (int b = 0; b < kMaxLoops; ++b) s->err_host[b] = 0;
    DGT_REQUIRE(!bad, DGT_ESTATE, "a dependence wait of the tiled executor timed out; its results are invalid");
}

// after a dependence-driven call: copy the error flags to pinned memory behind it
static void post_graph_flags(dgt_solver *s) {
    if (s->sched_mode != 1) return;
    if (!s->err_host) {
        DGT_HIP(hipHostMalloc((void **)&s->err_host, sizeof(int32_t) * kMaxLoops, hipHostMallocDefault));
        for (int b = 0; b < kMaxLoops; ++b) s->err_host[b] = 0;
        DGT_HIP(hipEventCreateWithFlags(&s->err_ev, hipEventDisableTiming));
    }
    bool any = false;
    for (size_t b = 0; b < s->plan.size() && b < (size_t)kMaxLoops; ++b) {
        if (!s->plan[b].graph) continue;
        DGT_HIP(hipMemcpyAsync(s->err_host + b, s->plan[b].err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
        any = true;
    }
    if (!any) return;
    DGT_HIP(hipEventRecord(s->err_ev, s->st));
    s->err_pending = true;
}

// extra_persist: fields written back for every cell that writes them (the FWI
// reversal keeps the intermediates U, X, Z this way); after: called once a
// sub-chain's launches are enqueued, with its plan index
template <int K, typename T>
static void step_tiled(dgt_solver *s, int64_t nsteps, double t0, int64_t &launches, int32_t extra_persist = 0,
                       const std::function<void(size_t)> *after = nullptr) {
    hipStream_t st = s->st;
    const double dt = s->p.dt;
    for (auto &P : s->plan)
        tile_launch<K, T>(P.kind, P.threads, s->upw, s->haspen, s->p.time_order, P.o0, P.nops, 0, P.lds_bytes,
                          st, P.args, TA_ATTR);
    // a chain fused over F steps runs F steps per pass (callers pass multiples of F)
    for (int64_t n = 0; n + s->fuse <= nsteps; n += s->fuse) {
        for (size_t b = 0; b < s->plan.size(); ++b) {
            SubPlan &P = s->plan[b];
            TileArgs A = P.args;
            for (int f = 0; f < F_COUNT; ++f) {
                A.F[f] = s->fld[f].p;
                A.fshot[f] = s->fshot(f);
            }
            A.nshots = s->nshots;
            A.src_cells = s->src_cells.p;
            A.src_vec = s->src_vec.p;
            A.persistent_mask |= extra_persist;
            A.dt = dt;
            // source amplitudes of the sub-chain's steps (a sub-chain spans at most four)
            for (int q = 0; q < 4; ++q) {
                const double th = t0 + ((double)(n + P.step0 + q) + 0.5) * dt;
                A.src_amps[q] = s->has_src ? dt * ricker(th, s->sf0, s->st0, s->samp) : 0.0;
            }
            A.src_amp = A.src_amps[0];
            if (s->sched_mode == 1 && P.kind != TK_GENERIC) {  // one launch for all colours
                A.persist = 1;
                A.ntiles = P.ntiles;
                A.nexec = P.nexec;
                A.tile_base = 0;
                const SubSched &sb = s->sched->s->sub[b];
                A.need = sb.dep_need.p;
                A.succ_off = sb.dep_off.p;
                A.succ = sb.dep_succ.p;
                A.cnt = P.cnt.p;
                A.head = P.head.p;
                A.err = P.err.p;
                A.head_base = P.epoch * (uint32_t)(P.nexec * s->nshots + P.slots);
                A.epoch = ++P.epoch;
                A.spin_limit = s->wait_limit;
                s->mark();
                tile_launch<K, T>(P.kind, P.threads, s->upw, s->haspen, s->p.time_order, P.o0, P.nops, P.slots,
                                  P.lds_bytes, st, A, TA_LAUNCH);
                s->mark();
                ++launches;
                if (after) (*after)(b);
                continue;
            }
            if (P.gmem_bytes) {  // one working set per workgroup of the largest colour launch
                int most = 0;
                for (int c = 0; c < P.nexec_colors; ++c) most = std::max(most, P.color_off[c + 1] - P.color_off[c]);
                const size_t need = (size_t)most * s->nshots * (size_t)P.gmem_bytes;
                if (P.gmem.n < need) P.gmem.alloc(need);
                A.scratch = P.gmem.p;
            }
            for (int c = 0; c < P.nexec_colors; ++c) {
                const int ntiles = P.color_off[c + 1] - P.color_off[c];
                if (ntiles == 0) continue;
                A.tile_base = P.color_off[c];
                s->mark();
                tile_launch<K, T>(P.kind, P.threads, s->upw, s->haspen, s->p.time_order, P.o0, P.nops,
                                  ntiles * s->nshots, P.lds_bytes, st, A, TA_LAUNCH);
                s->mark();
                ++launches;
            }
            if (after) (*after)(b);
        }
    }
}

}  // namespace dgt

using namespace dgt;

extern "C" {

dgt_status dgt_mesh_create(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int32_t periodic,
                           dgt_mesh **out) {
    return guard([&] {
        DGT_REQUIRE(out, DGT_EINVAL, "out is NULL");
        *out = nullptr;
        auto m = std::make_unique<dgt_mesh>();
        m->m = build_mesh(nv, xy, nc, c2v, periodic);
        *out = m.release();
    });
}

dgt_status dgt_mesh_counts(const dgt_mesh *m, int64_t *nc, int64_t *nf, int64_t *nb) {
    return guard([&] {
        DGT_REQUIRE(m, DGT_EINVAL, "mesh is NULL");
        if (nc) *nc = m->m.nc;
        if (nf) *nf = m->m.nf;
        if (nb) *nb = m->m.nb;
    });
}

dgt_status dgt_mesh_maps(const dgt_mesh *m, int32_t *f2c, int8_t *f2l, int32_t *b2c, int8_t *b2l, int8_t *bside) {
    return guard([&] {
        DGT_REQUIRE(m, DGT_EINVAL, "mesh is NULL");
        const Mesh &M = m->m;
        if (f2c) std::copy(M.f2c.begin(), M.f2c.end(), f2c);
        if (f2l) std::copy(M.f2l.begin(), M.f2l.end(), f2l);
        if (b2c) std::copy(M.b2c.begin(), M.b2c.end(), b2c);
        if (b2l) std::copy(M.b2l.begin(), M.b2l.end(), b2l);
        if (bside) std::copy(M.bside.begin(), M.bside.end(), bside);
    });
}

void dgt_mesh_destroy(dgt_mesh *m) { delete m; }

}  // extern "C"

namespace dgt {

// Scratch of the allocation-free energy reduction: the per-workgroup partial
// energies of k_energy and their sum, in a file-scope device array (one copy per
// GPU, held until the process ends).  Host code never passes the array's name to
// a kernel: each device's address is looked up once, with that device current,
// when the first solver on it is created.
constexpr int64_t ENERGY_NOALLOC_MAX_CELLS = int64_t(1) << 22;
constexpr int64_t ENERGY_NOALLOC_BLOCKS = ENERGY_NOALLOC_MAX_CELLS / 256;
static __device__ __align__(256) double scratch[ENERGY_NOALLOC_BLOCKS + 1];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// with device `dev` current
static void energy_scratch_init(int dev) {
    DGT_REQUIRE(dev >= 0 && dev < SCRATCH_MAX_DEVICES, DGT_EUNSUPPORTED, "device id beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void *p = nullptr;
    DGT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DGT_REQUIRE(p != nullptr, DGT_EHIP, "hipGetSymbolAddress returned NULL for the energy scratch");
    g_scratch_ptr[dev] = static_cast<double *>(p);
}

static double *energy_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    double *p = dev >= 0 && dev < SCRATCH_MAX_DEVICES ? g_scratch_ptr[dev] : nullptr;
    DGT_REQUIRE(p, DGT_ESTATE, "energy scratch of the solver's device was not set up");
    return p;
}

// The solver without the sign check of dt: the FWI adjoint runs the chain backward
// in time (dt < 0) on a solver of its own.
static std::unique_ptr<dgt_solver> new_solver(const dgt_mesh *m, const double *lam, const double *mu,
                                          const double *rho, const dgt_solver_params *p, void *stream) {
    DGT_REQUIRE(p->degree >= 1 && p->degree <= 4, DGT_EINVAL, "degree must be 1..4");
    DGT_REQUIRE(p->flux == 0 || p->flux == 1, DGT_EINVAL, "flux must be 0 or 1");
    DGT_REQUIRE(p->time_order == 2 || p->time_order == 4, DGT_EINVAL, "time_order must be 2 or 4");
    DGT_REQUIRE(p->precision == 0 || p->precision == 1, DGT_EINVAL, "precision must be 0 or 1");
    DGT_REQUIRE(p->dt != 0 && std::isfinite(p->dt), DGT_EINVAL, "dt must be finite and nonzero");
    const Mesh &M = m->m;
    DGT_REQUIRE(M.nc > 0, DGT_EINVAL, "empty mesh");
    DGT_REQUIRE(lam && mu && rho, DGT_EINVAL, "material is NULL");
    for (int64_t c = 0; c < M.nc; ++c)
        DGT_REQUIRE(lam[c] > 0 && mu[c] > 0 && rho[c] > 0, DGT_EINVAL, "material must be positive");
    auto s = std::make_unique<dgt_solver>();
    DGT_HIP(hipGetDevice(&s->dev));
    energy_scratch_init(s->dev);
    s->mesh = &M;
    s->mesh_handle = m;
    s->p = *p;
    s->st = (hipStream_t)stream;
    s->K = p->degree;
    s->fp32 = p->precision;
    s->esz = p->precision ? 4 : 8;
    s->upw = p->flux == 1;
    s->nc = M.nc;
    s->nf = M.nf;
    s->nb = M.nb;
    s->haspen = s->upw;
    for (int64_t b = 0; b < M.nb; ++b)
        if (!(M.bside[b] >= 0 && ((p->free_sides >> M.bside[b]) & 1))) s->haspen = 1;
    s->E = make_refelem(p->degree);
    hipStream_t st = s->st;
    dispatch(s.get(), [&]<int K, typename T>() {
        upload_ref<K, T>(s->E, st);
        tile_upload_ref<K, T>(s->E, st);
    });
    s->xy.upload(M.xy, st);
    s->c2v.upload(M.c2v, st);
    s->f2c.upload(M.f2c.empty() ? std::vector<int32_t>{0, 0} : M.f2c, st);
    s->f2l.upload(M.f2l.empty() ? std::vector<int8_t>{0, 0} : M.f2l, st);
    s->b2c.upload(M.b2c.empty() ? std::vector<int32_t>{0} : M.b2c, st);
    s->b2l.upload(M.b2l.empty() ? std::vector<int8_t>{0} : M.b2l, st);
    std::vector<uint8_t> bfree(std::max<int64_t>(M.nb, 1), 0);
    for (int64_t b = 0; b < M.nb; ++b) bfree[b] = M.bside[b] >= 0 && ((p->free_sides >> M.bside[b]) & 1);
    s->bfree.upload(bfree, st);
    s->lam.upload(lam, M.nc, st);
    s->mu.upload(mu, M.nc, st);
    s->rho.upload(rho, M.nc, st);
    const int np = s->E.np, nfp = s->E.nfp;
    s->geo.alloc((size_t)(G_NROWS + 1) * M.nc * s->esz);
    alloc_fields(s.get());
    s->G.alloc((size_t)2 * 3 * nfp * std::max<int64_t>(M.nf, 1) * s->esz);
    s->Gx.alloc((size_t)3 * nfp * std::max<int64_t>(M.nb, 1) * s->esz);
    s->src_vec.alloc((size_t)np * s->esz);
    DGT_HIP(hipMemsetAsync(s->src_vec.p, 0, s->src_vec.n, st));
    s->src_in.assign(1, -1);
    std::vector<int32_t> id(M.nc);
    std::iota(id.begin(), id.end(), 0);
    set_exec_order(s.get(), id);
    build_loops(s.get());
    DGT_HIP(hipEventCreate(&s->ev0));
    DGT_HIP(hipEventCreate(&s->ev1));
    return s;
}

}  // namespace dgt

extern "C" {

dgt_status dgt_solver_create(const dgt_mesh *m, const double *lam, const double *mu, const double *rho,
                             const dgt_solver_params *p, void *stream, dgt_solver **out) {
    return guard([&] {
        DGT_REQUIRE(m && p && out, DGT_EINVAL, "NULL argument");
        *out = nullptr;
        DGT_REQUIRE(p->dt > 0 && std::isfinite(p->dt), DGT_EINVAL, "dt must be positive");
        *out = new_solver(m, lam, mu, rho, p, stream).release();
    });
}

// The lowest-id cell containing (x, y) (with a 1e-12 tolerance in reference
// coordinates) and the point's reference coordinates; -1 when none does.
static int64_t locate_point(const dgt_solver *s, double x, double y, double &rs, double &ss) {
    const Mesh &M = *s->mesh;
    for (int64_t c = 0; c < M.nc; ++c) {
        const double *p0 = &M.xy[2 * M.c2v[3 * c]], *p1 = &M.xy[2 * M.c2v[3 * c + 1]],
                     *p2 = &M.xy[2 * M.c2v[3 * c + 2]];
        const double xr = p1[0] - p0[0], xs = p2[0] - p0[0], yr = p1[1] - p0[1], ys = p2[1] - p0[1];
        const double det = xr * ys - xs * yr;
        const double r = (ys * (x - p0[0]) - xs * (y - p0[1])) / det;
        const double sv = (-yr * (x - p0[0]) + xr * (y - p0[1])) / det;
        if (r >= -1e-12 && sv >= -1e-12 && 1.0 - r - sv >= -1e-12) {
            rs = r;
            ss = sv;
            return c;
        }
    }
    return -1;
}

// Point sources of every shot: the lowest-id cell containing (x, y) and the vector
// inverse reference mass times the basis at the point, divided by |det J| (the
// projection of a point force onto the cell's polynomial space).
static void set_sources(dgt_solver *s, const double *xy, double f0, double t0, double amp) {
    const Mesh &M = *s->mesh;
    const int np = s->E.np;
    std::vector<int64_t> cells(s->nshots, -1);
    std::vector<double> svs((size_t)s->nshots * np);
    for (int q = 0; q < s->nshots; ++q) {
        const double x = xy[2 * q], y = xy[2 * q + 1];
        DGT_REQUIRE(std::isfinite(x) && std::isfinite(y), DGT_EINVAL, "source position is not finite");
        double rs = 0, ss = 0;
        const int64_t cell = locate_point(s, x, y, rs, ss);
        DGT_REQUIRE(cell >= 0, DGT_EINVAL, "source outside the mesh");
        std::vector<double> phi(np);
        s->E.phi(rs, ss, phi.data());
        const double *p0 = &M.xy[2 * M.c2v[3 * cell]], *p1 = &M.xy[2 * M.c2v[3 * cell + 1]],
                     *p2 = &M.xy[2 * M.c2v[3 * cell + 2]];
        const double det = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]);
        for (int i = 0; i < np; ++i) {
            double a = 0;
            for (int j = 0; j < np; ++j) a += s->E.Minv[i * np + j] * phi[j];
            svs[(size_t)q * np + i] = a / det;
        }
        cells[q] = cell;
    }
    s->src_vec.alloc(svs.size() * s->esz);
    if (s->fp32) {
        std::vector<float> f(svs.begin(), svs.end());
        DGT_HIP(hipMemcpyAsync(s->src_vec.p, f.data(), 4 * f.size(), hipMemcpyHostToDevice, s->st));
    } else {
        DGT_HIP(hipMemcpyAsync(s->src_vec.p, svs.data(), 8 * svs.size(), hipMemcpyHostToDevice, s->st));
    }
    DGT_HIP(hipStreamSynchronize(s->st));
    s->has_src = true;
    s->src_in = cells;
    s->sf0 = f0;
    s->st0 = t0;
    s->samp = amp;
    set_source_exec(s);
}

// workgroups of a sub-chain's tile kernel that the whole GPU holds at once
static int plan_slots(dgt_solver *s, const SubPlan &P) {
    int occ = 0, dev = 0;
    dispatch(s, [&]<int K, typename T>() {
        tile_launch<K, T>(P.kind, P.threads, s->upw, s->haspen, s->p.time_order, P.o0, P.nops, 0, P.lds_bytes,
                          s->st, P.args, TA_ATTR);
        tile_launch<K, T>(P.kind, P.threads, s->upw, s->haspen, s->p.time_order, P.o0, P.nops, 0, P.lds_bytes,
                          s->st, P.args, TA_OCCUPANCY, &occ);
    });
    DGT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    DGT_HIP(hipGetDeviceProperties(&prop, dev));
    return occ * prop.multiProcessorCount;
}

// Counters and workgroup counts of the dependence-driven schedule (schedule 1).
static void prepare_tiled(dgt_solver *s) {
    if (s->sched_mode != 1) return;
    check_graphs(s, false);  // reports a wait that timed out in an earlier call, without waiting
    for (size_t b = 0; b < s->plan.size(); ++b) {
        SubPlan &P = s->plan[b];
        if (P.kind == TK_GENERIC) continue;
        if (!P.graph) build_graph(s, (int)b, P);
        if (!P.slots) P.slots = plan_slots(s, P);
        DGT_REQUIRE(P.slots > 0, DGT_EUNSUPPORTED, "the tile kernel does not fit on a compute unit");
    }
}

// Cell order of the executor within each seed tile of the sub-chain with the finest
// seed partition (the tile that runs a cell's iteration of the sub-chain's first
// loop, whose assignment is the seed partition): the cells only its own footprint
// holds first, then the cells that other tiles' footprints also gather, grouped by
// the lowest such tile, each group in seed order.  The fields
// are stored [component][node][cell], so a cell gathered as part of another tile's
// halo pulls a memory sector per component and node; with a neighbour's halo cells in
// one run those sectors are shared.  The order is only a permutation of the
// executor's layout: schedules, results and the caller's numbering are unchanged.
static void group_halo_cells(dgt_solver *s, std::vector<int32_t> &rank) {
    hipStream_t st = s->st;
    const Schedule &S = *s->sched->s;
    // the sub-chain with the finest seed partition (the most tiles)
    size_t bf = 0;
    for (size_t b = 1; b < S.sub.size(); ++b)
        if (S.sub[b].ntiles > S.sub[bf].ntiles) bf = b;
    const SubSched &sb = S.sub[bf];
    const int64_t nc = s->nc;
    if (nc == 0 || sb.ntiles == 0 || S.seed_set != 0 || s->loops[sb.first].set != 0 || S.loop_size[sb.first] != nc)
        return;
    const std::vector<int32_t> owner = S.sigma[sb.first].download(st, nc);
    const std::vector<int32_t> foff = sb.foot_off[0].download(st, sb.ntiles + 1);
    const std::vector<int32_t> foot = sb.foot[0].download(st, std::max<int64_t>(foff[sb.ntiles], 1));
    std::vector<int32_t> nbt(nc, INT32_MAX);
    for (int t = 0; t < sb.ntiles; ++t)
        for (int q = foff[t]; q < foff[t + 1]; ++q) {
            const int32_t x = foot[q];
            if (owner[x] != t) nbt[x] = std::min(nbt[x], t);
        }
    // key (seed tile, group: 0 interior, 1 + the neighbouring tile), then the seed rank
    struct Key {
        uint64_t hi;
        int32_t rank, cell;
    };
    std::vector<Key> keys(nc);
    for (int64_t x = 0; x < nc; ++x)
        keys[x] = {((uint64_t)(uint32_t)owner[x] << 32) | (uint64_t)(nbt[x] == INT32_MAX ? 0 : (uint32_t)nbt[x] + 1u),
                   rank[x], (int32_t)x};
    std::sort(keys.begin(), keys.end(),
              [](const Key &a, const Key &b) { return a.hi != b.hi ? a.hi < b.hi : a.rank < b.rank; });
    for (int64_t i = 0; i < nc; ++i) rank[keys[i].cell] = (int32_t)i;
}

static void solver_inspect_once(dgt_solver *s, const dgt_inspect_params *p, int cap) {
    hipStream_t st = s->st;
    s->inspected = false;
    ++s->gen;
    s->last_ip = *p;
    s->last_splits.assign(p->splits, p->splits + p->nsplits);
    s->last_ip.splits = nullptr;
    if (p->sub_tile_sizes) s->last_sub_ts.assign(p->sub_tile_sizes, p->sub_tile_sizes + p->nsplits + 1);
    else s->last_sub_ts.clear();
    s->last_ip.sub_tile_sizes = nullptr;
    if (p->seed_region) s->last_region.assign(p->seed_region, p->seed_region + s->nc);
    else s->last_region.clear();
    s->last_ip.seed_region = nullptr;
    s->last_cap = cap;
    delete s->sched;
    s->sched = nullptr;
    s->plan.clear();
    s->plan_status = DGT_ESTATE;
    s->plan_error = "tiled mode needs a successful dgt_solver_inspect";
    DBuf<double> cxy(2 * s->nc);
    k_centroids<<<blocks_for(s->nc, 256), 256, 0, st>>>(s->xy.p, s->c2v.p, s->nc, cxy.p);
    auto sch = std::make_unique<dgt_schedule>();
    sch->chain_copy = s->chain.c;
    sch->chain = &sch->chain_copy;
    Inspector insp(sch->chain_copy, st);
    std::vector<int32_t> splits(p->splits, p->splits + p->nsplits);
    sch->s = insp.run(p->tile_size, p->partition, nullptr, cxy.p, p->max_conflict_rounds, cap, splits,
                      s->last_sub_ts, s->last_region.empty() ? nullptr : s->last_region.data(), p->region_carry);
    s->sched = sch.release();
    // executor layout follows the seed order of the schedule
    auto rank = s->sched->s->seed_rank.download(st, s->nc);
    const char *eo = std::getenv("DGT_EXEC_ORDER");
    if (!(eo && std::string(eo) == "seed")) group_halo_cells(s, rank);
    set_exec_order(s, rank);
    // the schedule stays valid when the tiled executor cannot run its tiles
    // (footprints beyond 16,383 cells); only the tiled executor is then unavailable
    try {
        build_plan(s);
        s->plan_status = DGT_OK;
        s->inspected = true;
    } catch (const Error &e) {
        if (e.st != DGT_EUNSUPPORTED) throw;
        s->plan.clear();
        s->plan_status = e.st;
        s->plan_error = e.msg;
    }
}

dgt_status dgt_solver_inspect(dgt_solver *s, const dgt_inspect_params *p) {
    return guard([&] {
        DGT_REQUIRE(s && p, DGT_EINVAL, "NULL argument");
        DGT_REQUIRE(p->partition == 0 || p->partition == 1, DGT_EINVAL, "partition must be 0 or 1");
        DGT_REQUIRE(p->nsplits >= 0 && (p->nsplits == 0 || p->splits), DGT_EINVAL, "bad splits");
        DGT_REQUIRE(p->max_colour_tiles >= -1, DGT_EINVAL, "max_colour_tiles must be >= -1");
        if (p->seed_region) {
            // a step runs all its sub-chains after one halo exchange
            DGT_REQUIRE(p->nsplits == 0 || p->region_carry == 1, DGT_EINVAL,
                        "seed regions with several sub-chains need region_carry = 1 (one exchange per step)");
            DGT_REQUIRE(p->max_colour_tiles <= 0, DGT_EINVAL, "seed regions do not combine with max_colour_tiles");
        }
        solver_inspect_once(s, p, p->max_colour_tiles > 0 ? p->max_colour_tiles : 0);
        if (p->max_colour_tiles == -1 && !p->seed_region && s->plan_status == DGT_OK) {
            // cap the colour classes at the number of tile workgroups resident at once when
            // some class would need more than one round of them
            int slots = INT32_MAX;
            bool over = false;
            for (const auto &P : s->plan) {
                const int sl = plan_slots(s, P);
                slots = std::min(slots, sl);
                for (int c = 0; c < P.ncolors; ++c) over |= P.color_off[c + 1] - P.color_off[c] > sl;
            }
            if (over && slots > 0) solver_inspect_once(s, p, slots);
        }
    });
}

dgt_status dgt_solver_autotune(dgt_solver *s, const dgt_autotune_params *p, dgt_autotune_result *out) {
    return guard([&] {
        DGT_REQUIRE(s && p && out, DGT_EINVAL, "NULL argument");
        DGT_REQUIRE(p->ntile_sizes >= 1 && p->ntile_sizes <= 64 && p->tile_sizes, DGT_EINVAL,
                    "1..64 candidate tile sizes");
        for (int i = 0; i < p->ntile_sizes; ++i)
            DGT_REQUIRE(p->tile_sizes[i] >= 1, DGT_EINVAL, "tile sizes must be >= 1");
        DGT_REQUIRE(p->partition == 0 || p->partition == 1, DGT_EINVAL, "partition must be 0 or 1");
        DGT_REQUIRE(p->nsplits >= 0 && (p->nsplits == 0 || p->splits), DGT_EINVAL, "bad splits");
        DGT_REQUIRE(p->trial_steps >= 1 && p->trial_steps <= 1000, DGT_EINVAL, "trial_steps must be 1..1000");
        DGT_REQUIRE(p->prune >= 0, DGT_EINVAL, "prune must be >= 0");
        hipStream_t st = s->st;
        const int np = s->E.np;
        // keep the caller's state (in the mesh's numbering: the trials renumber the cells)
        DBuf<char> keep;
        const bool had = s->state_valid;
        if (had) {
            keep.alloc((size_t)5 * np * s->nc * s->esz * s->nshots);
            to_caller(s, keep.p, keep.p + (size_t)2 * np * s->nc * s->esz * s->nshots);
        }
        s->state_valid = false;
        dgt_inspect_params ip{};
        ip.partition = p->partition;
        ip.max_conflict_rounds = 64;
        ip.splits = p->splits;
        ip.nsplits = p->nsplits;
        const std::vector<uint8_t> regions = s->last_region;  // a part keeps its regions
        if (!regions.empty()) {
            ip.seed_region = regions.data();
            ip.region_carry = 1;
        }
        struct Cand { int ts; double foot; bool gmem; };
        std::vector<Cand> cands;
        int skipped = 0, timed = 0;
        // footprint model: the cells a tile gathers over all its sub-chains, summed over
        // tiles and divided by the mesh's cells, is the data a step moves per cell
        // (the halo grows as tiles shrink); candidates whose tiles fit are timed in
        // ascending model cost, and with prune > 0 a candidate whose cost exceeds
        // prune times the lowest is dropped untimed
        for (int i = 0; i < p->ntile_sizes; ++i) {
            ip.tile_size = p->tile_sizes[i];
            solver_inspect_once(s, &ip, 0);
            if (s->plan_status != DGT_OK) {
                ++skipped;
                continue;
            }
            double f = 0;
            for (const auto &sb : s->sched->s->sub) f += (double)sb.foot_len[0];
            bool gmem = false;
            for (const auto &P : s->plan) gmem |= P.gmem_bytes > 0;
            cands.push_back({p->tile_sizes[i], f / (double)s->nc, gmem});
        }
        DGT_REQUIRE(!cands.empty(), DGT_EUNSUPPORTED, "no candidate tile size has tiles the executor can run");
        // tiles whose working set leaves the LDS run from global scratch at a fraction of
        // the speed: they are timed only when no candidate fits the LDS
        if (std::any_of(cands.begin(), cands.end(), [](const Cand &c) { return !c.gmem; })) {
            const size_t before = cands.size();
            cands.erase(std::remove_if(cands.begin(), cands.end(), [](const Cand &c) { return c.gmem; }), cands.end());
            skipped += (int)(before - cands.size());
        }
        std::stable_sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.foot < b.foot; });
        double best_ms = 1e300;
        int best_ts = cands[0].ts, best_sched = 0;
        const int keep_mode = s->sched_mode;
        for (const Cand &c : cands) {
            if (p->prune > 0 && c.foot > p->prune * cands[0].foot) {
                ++skipped;
                continue;
            }
            ip.tile_size = c.ts;
            solver_inspect_once(s, &ip, 0);
            bool chain = false;
            for (const auto &P : s->plan) chain |= P.kind != TK_GENERIC;
            for (int mode = 0; mode <= (chain ? 1 : 0); ++mode) {
                s->sched_mode = mode;
                for (int f = 0; f < F_COUNT; ++f) DGT_HIP(hipMemsetAsync(s->fld[f].p, 0, s->fld[f].n, st));
                prepare_tiled(s);
                int64_t launches = 0;
                dispatch(s, [&]<int K, typename T>() {
                    step_tiled<K, T>(s, s->fuse, 0.0, launches);  // first launches: code and caches warm
                    DGT_HIP(hipEventRecord(s->ev0, st));
                    step_tiled<K, T>(s, (int64_t)p->trial_steps * s->fuse, s->p.dt * s->fuse, launches);
                    DGT_HIP(hipEventRecord(s->ev1, st));
                });
                DGT_HIP(hipGetLastError());
                DGT_HIP(hipEventSynchronize(s->ev1));
                float ms = 0;
                DGT_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
                check_graphs(s);
                ++timed;
                const double per = ms / ((double)p->trial_steps * s->fuse);
                if (per < best_ms) {
                    best_ms = per;
                    best_ts = c.ts;
                    best_sched = mode;
                }
            }
        }
        s->sched_mode = keep_mode;
        ip.tile_size = best_ts;
        solver_inspect_once(s, &ip, 0);
        s->sched_mode = best_sched;
        for (int f = 0; f < F_COUNT; ++f) DGT_HIP(hipMemsetAsync(s->fld[f].p, 0, s->fld[f].n, st));
        if (had) {
            from_caller(s, keep.p, keep.p + (size_t)2 * np * s->nc * s->esz * s->nshots);
            s->state_valid = true;
        }
        DGT_HIP(hipStreamSynchronize(st));
        s->last_ms = -1.0;
        s->last_launches = 0;
        out->tile_size = best_ts;
        out->schedule = best_sched;
        out->ms_per_step = best_ms;
        out->timed = timed;
        out->skipped = skipped;
    });
}

dgt_status dgt_solver_schedule(const dgt_solver *s, const dgt_schedule **out) {
    return guard([&] {
        DGT_REQUIRE(s && out, DGT_EINVAL, "NULL argument");
        *out = s->sched;
    });
}

dgt_status dgt_set_source(dgt_solver *s, double x, double y, double f0, double t0, double amp) {
    return guard([&] {
        DGT_REQUIRE(s, DGT_EINVAL, "solver is NULL");
        std::vector<double> xy;
        for (int q = 0; q < s->nshots; ++q) {
            xy.push_back(x);
            xy.push_back(y);
        }
        set_sources(s, xy.data(), f0, t0, amp);
    });
}

dgt_status dgt_solver_set_shots(dgt_solver *s, int32_t nshots, const double *xy, double f0, double t0,
                                double amp) {
    return guard([&] {
        DGT_REQUIRE(s && nshots >= 1 && nshots <= 65536, DGT_EINVAL, "nshots must be 1..65536");
        const int64_t words = (int64_t)5 * s->E.np * s->nc * nshots;
        DGT_REQUIRE(words * (int64_t)s->esz < ((int64_t)1 << 40), DGT_EINVAL, "state of all shots exceeds 1 TiB");
        DGT_HIP(hipStreamSynchronize(s->st));
        check_graphs(s);
        s->nshots = nshots;
        alloc_fields(s);
        s->state_valid = false;
        for (auto &P : s->plan) P.graph = false;  // counters are per shot
        s->has_src = false;
        s->src_in.assign(nshots, -1);
        s->src_vec.alloc((size_t)nshots * s->E.np * s->esz);
        DGT_HIP(hipMemsetAsync(s->src_vec.p, 0, s->src_vec.n, s->st));
        set_source_exec(s);  // no sources until set_sources succeeds
        if (xy) set_sources(s, xy, f0, t0, amp);
    });
}

dgt_status dgt_state_upload(dgt_solver *s, const void *v, const void *sig) {
    return guard([&] {
        DGT_REQUIRE(s && v && sig, DGT_EINVAL, "NULL argument");
        from_caller(s, v, sig);
        s->state_valid = true;
    });
}

dgt_status dgt_state_download(dgt_solver *s, void *v, void *sig) {
    return guard([&] {
        DGT_REQUIRE(s && v && sig, DGT_EINVAL, "NULL argument");
        DGT_REQUIRE(s->state_valid, DGT_ESTATE, "no state uploaded");
        check_graphs(s);
        to_caller(s, v, sig);
    });
}

struct dgt_cell_list {
    int64_t nc = 0, n = 0;
    int dev = 0;
    DBuf<int32_t> cells;  // mesh cell ids
};

dgt_status dgt_cell_list_create(const dgt_solver *s, int64_t n, const int32_t *cells, dgt_cell_list **out) {
    return guard([&] {
        DGT_REQUIRE(s && out && n >= 0 && (n == 0 || cells), DGT_EINVAL, "bad arguments");
        *out = nullptr;
        for (int64_t i = 0; i < n; ++i)
            DGT_REQUIRE(cells[i] >= 0 && cells[i] < s->nc, DGT_EINVAL, "cell id out of range");
        auto l = std::make_unique<dgt_cell_list>();
        l->nc = s->nc;
        l->n = n;
        l->dev = s->dev;
        l->cells.alloc(std::max<int64_t>(n, 1));
        if (n) l->cells.upload(cells, (size_t)n, s->st);
        DGT_HIP(hipStreamSynchronize(s->st));
        *out = l.release();
    });
}

void dgt_cell_list_destroy(dgt_cell_list *l) { delete l; }

static void halo_copy(dgt_solver *s, const dgt_cell_list *l, const void *v, const void *sig, bool unpack) {
    DGT_REQUIRE(s && l, DGT_EINVAL, "NULL argument");
    DGT_REQUIRE(l->nc == s->nc && l->dev == s->dev, DGT_EINVAL, "the cell list belongs to another mesh or device");
    DGT_REQUIRE(s->state_valid, DGT_ESTATE, "no state uploaded");
    if (!unpack) check_graphs(s, false);
    if (l->n == 0) return;  // empty buffers may be NULL
    DGT_REQUIRE(v && sig, DGT_EINVAL, "NULL buffer");
    dispatch(s, [&]<int K, typename T>() {
        for (int f : {F_V, F_S}) {
            const int64_t rows = field_ncomp(f) * s->E.np, total = rows * s->nshots * l->n;
            T *buf = (T *)(f == F_V ? v : sig);
            k_halo_copy<T><<<blocks_for(total, 256), 256, 0, s->st>>>((T *)s->fld[f].p, buf, s->rank.p, l->cells.p,
                                                                      l->n, rows, s->nc, total, unpack ? 1 : 0);
        }
    });
    DGT_HIP(hipGetLastError());
}

dgt_status dgt_state_pack(dgt_solver *s, const dgt_cell_list *l, void *v, void *sig) {
    return guard([&] { halo_copy(s, l, v, sig, false); });
}

dgt_status dgt_state_unpack(dgt_solver *s, const dgt_cell_list *l, const void *v, const void *sig) {
    return guard([&] { halo_copy(s, l, v, sig, true); });
}

dgt_status dgt_step(dgt_solver *s, int64_t nsteps, int32_t mode, double t0) {
    return guard([&] {
        DGT_REQUIRE(s && nsteps >= 0, DGT_EINVAL, "bad arguments");
        DGT_REQUIRE(s->state_valid, DGT_ESTATE, "state not uploaded");
        DGT_REQUIRE(mode == 0 || mode == 1, DGT_EINVAL, "mode must be 0 or 1");
        DGT_REQUIRE(mode == 0 || s->plan_status == DGT_OK, s->plan_status, s->plan_error);
        DGT_REQUIRE(mode == 0 || nsteps % s->fuse == 0, DGT_EINVAL,
                    "a chain fused over several steps runs a multiple of that many steps");
        if (mode == 1) prepare_tiled(s);
        int64_t launches = 0;
        s->npev = 0;
        DGT_HIP(hipEventRecord(s->ev0, s->st));
        dispatch(s, [&]<int K, typename T>() {
            if (mode == 0) step_untiled<K, T>(s, nsteps, t0, launches);
            else step_tiled<K, T>(s, nsteps, t0, launches);
        });
        DGT_HIP(hipGetLastError());
        DGT_HIP(hipEventRecord(s->ev1, s->st));
        if (mode == 1) post_graph_flags(s);
        s->last_launches = launches;
        s->last_ms = -1.0;
    });
}

dgt_status dgt_solver_set_schedule(dgt_solver *s, int32_t mode) {
    return guard([&] {
        DGT_REQUIRE(s && (mode == 0 || mode == 1), DGT_EINVAL, "bad arguments");
        s->sched_mode = mode;
    });
}

dgt_status dgt_solver_set_wait_limit(dgt_solver *s, int64_t polls) {
    return guard([&] {
        DGT_REQUIRE(s && polls >= 1 && polls <= (int64_t)UINT32_MAX, DGT_EINVAL, "bad arguments");
        s->wait_limit = (uint32_t)polls;
    });
}

dgt_status dgt_solver_profile(dgt_solver *s, int32_t on) {
    return guard([&] {
        DGT_REQUIRE(s && (on == 0 || on == 1), DGT_EINVAL, "bad arguments");
        s->prof = on == 1;
    });
}

dgt_status dgt_last_step_timing(const dgt_solver *s, double *total_ms, double *kernel_ms, int64_t *launches) {
    return guard([&] {
        DGT_REQUIRE(s, DGT_EINVAL, "solver is NULL");
        DGT_HIP(hipEventSynchronize(s->ev1));
        float ms = 0;
        DGT_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
        if (total_ms) *total_ms = ms;
        double kms = ms;
        if (s->npev >= 2) {
            kms = 0;
            for (size_t i = 0; i + 1 < s->npev; i += 2) {
                float d = 0;
                DGT_HIP(hipEventElapsedTime(&d, s->pev[i], s->pev[i + 1]));
                kms += d;
            }
        }
        if (kernel_ms) *kernel_ms = kms;
        if (launches) *launches = s->last_launches;
    });
}

dgt_status dgt_energy(dgt_solver *s, const void *v, const void *sig_new, const void *sig_old, double *out) {
    return guard([&] {
        DGT_REQUIRE(s && v && sig_new && sig_old && out, DGT_EINVAL, "NULL argument");
        const int64_t nc = s->nc;
        const int64_t nblk = (nc + 255) / 256;
        DBuf<double> part(nblk), res(1);
        dispatch(s, [&]<int K, typename T>() {
            k_energy<K, T><<<nblk, 256, 0, s->st>>>((const T *)v, (const T *)sig_new, (const T *)sig_old,
                                                  (const T *)s->geo.p, s->rank.p, nc, part.p);
        });
        k_sum_partials<<<1, 256, 0, s->st>>>(part.p, nblk, res.p);
        *out = res.download(s->st)[0];
    });
}

dgt_status dgt_energy_noalloc(dgt_solver *s, const void *v, const void *sig_new, const void *sig_old, double *out) {
    return guard([&] {
        DGT_REQUIRE(s && v && sig_new && sig_old && out, DGT_EINVAL, "NULL argument");
        const int64_t nc = s->nc;
        DGT_REQUIRE(nc <= ENERGY_NOALLOC_MAX_CELLS, DGT_EINVAL,
                    "dgt_energy_noalloc: " + std::to_string(nc) + " cells exceed its limit of " +
                        std::to_string(ENERGY_NOALLOC_MAX_CELLS));
        double *ptr = energy_scratch(s->dev);
        const int64_t nblk = (nc + 255) / 256;
        // every partial in [0, nblk) and the sum are written before they are read: nothing to clear
        dispatch(s, [&]<int K, typename T>() {
            k_energy<K, T><<<nblk, 256, 0, s->st>>>((const T *)v, (const T *)sig_new, (const T *)sig_old,
                                                  (const T *)s->geo.p, s->rank.p, nc, ptr);
        });
        k_sum_partials<<<1, 256, 0, s->st>>>(ptr, nblk, ptr + ENERGY_NOALLOC_BLOCKS);
        DGT_HIP(hipGetLastError());
        double h = 0.0;
        DGT_HIP(hipMemcpyAsync(&h, ptr + ENERGY_NOALLOC_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s->st));
        DGT_HIP(hipStreamSynchronize(s->st));
        *out = h;
    });
}

dgt_status dgt_solver_info(const dgt_solver *s, int64_t *np, int64_t *bytes_per_step, int64_t *lds_bytes) {
    return guard([&] {
        DGT_REQUIRE(s, DGT_EINVAL, "solver is NULL");
        if (np) *np = s->E.np;
        // state read and written once, per-cell invariants (9 geometry rows) read once
        if (bytes_per_step)
            *bytes_per_step = (int64_t)(2 * 5 * s->E.np * s->nshots + G_NROWS) * (int64_t)s->esz * s->nc;
        size_t mx = 0;
        for (auto &P : s->plan) mx = std::max(mx, P.lds_bytes);
        if (lds_bytes) *lds_bytes = (int64_t)mx;
    });
}

dgt_status dgt_solver_fuse_steps(dgt_solver *s, int32_t steps) {
    return guard([&] {
        DGT_REQUIRE(s, DGT_EINVAL, "NULL solver");
        DGT_REQUIRE(steps >= 1 && steps * loops_per_step(s->p.time_order) <= kMaxLoops, DGT_EINVAL,
                    "steps must be >= 1 with at most 64 loops in the chain");
        s->fuse = steps;
        build_loops(s);
        // the old schedule and plan describe another chain
        s->inspected = false;
        ++s->gen;
        delete s->sched;
        s->sched = nullptr;
        s->plan.clear();
        s->plan_status = DGT_ESTATE;
        s->plan_error = "tiled mode needs dgt_solver_inspect after dgt_solver_fuse_steps";
    });
}

void dgt_solver_destroy(dgt_solver *s) { delete s; }

dgt_status dgt_solver_kernels(const dgt_solver *s, int32_t *nsub, int32_t *kinds) {
    return guard([&] {
        DGT_REQUIRE(s && nsub, DGT_EINVAL, "NULL argument");
        *nsub = (int32_t)s->plan.size();
        if (kinds)
            for (size_t b = 0; b < s->plan.size(); ++b) kinds[b] = s->plan[b].gmem_bytes ? 3 : (int32_t)s->plan[b].kind;
    });
}

dgt_status dgt_refelem(int32_t degree, double *dr, double *ds, double *minv, double *lift) {
    return guard([&] {
        DGT_REQUIRE(degree >= 1 && degree <= 4, DGT_EINVAL, "degree must be 1..4");
        const RefElem E = make_refelem(degree);
        const size_t n2 = (size_t)E.np * E.np;
        if (dr) std::memcpy(dr, E.Dr.data(), n2 * sizeof(double));
        if (ds) std::memcpy(ds, E.Ds.data(), n2 * sizeof(double));
        if (minv) std::memcpy(minv, E.Minv.data(), n2 * sizeof(double));
        if (lift) std::memcpy(lift, E.lift.data(), E.lift.size() * sizeof(double));
    });
}

}  // extern "C"

#include "fwi_impl.h"
#include "batch_impl.h"
