// Several solvers advanced by shared launches -- one per colour of a sub-chain, or
// one per sub-chain under the dependence-driven schedule -- optionally replayed
// from a HIP graph (included at the end of solver.hip).  The paper runs one mesh at a time;
// the batched form serves many meshes and shots of the same discretisation, so
// it cites no passage of the paper.
//
// Each member keeps its fields, schedule, plan and source; the batch owns the
// work-queue segments and its own dependence and ticket counters, so members can
// still be stepped alone.  Graph mode captures K steps (kernel nodes only) once and
// replays them: before each replay the step offset of the source amplitudes is set
// (and, for the dependence-driven schedule, the counters cleared), outside the
// graph; the amplitudes of the whole call are uploaded at its start.

struct dgt_batch {
    std::vector<dgt_solver *> m;        // members (not owned)
    std::vector<uint64_t> gen;          // their inspection generations at creation
    hipStream_t user = nullptr;         // caller's stream
    hipStream_t gst = nullptr;          // own stream (graph capture and replay)
    hipEvent_t ev0 = nullptr, ev1 = nullptr, join = nullptr;
    int K = 0, fp32 = 0, upw = 0, order = 4, nsub = 0;
    int sched = 0;  // 0: one launch per colour of a sub-chain; 1: dependence-driven, one per sub-chain
    struct Sub {
        int o0 = 0, nops = 0, nt = 0;
        size_t lds = 0;
        int nseg = 0;
        uint32_t total = 0;
        int slots = 0;
        uint32_t epoch = 0;
        dgt::DBuf<int32_t> seg_start, seg_mesh, seg_local;
        std::vector<dgt::DBuf<uint32_t>> cnt;  // [mesh] [nshots][ntiles]
        dgt::DBuf<uint32_t> head;
        dgt::DBuf<dgt::TileArgs> args;         // [mesh] launch arguments (fixed for the batch)
        dgt::DBuf<dgt::TileArgs> args_c;       // the same for colour launches
        std::vector<int32_t> cseg;             // [ncolours + 1] segments of each colour
        std::vector<uint32_t> cstart;          // [ncolours + 1] first item of each colour
    };
    std::vector<Sub> sub;
    dgt::DBuf<int32_t> err;
    // source amplitudes of a call's steps, [mesh][amp_cap], staged through pinned memory
    dgt::DBuf<double> amp;
    double *amp_host = nullptr;
    int64_t amp_cap = 0;
    hipEvent_t amp_ev = nullptr;
    // graph mode
    int gsteps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    dgt::DBuf<int32_t> amp_base;        // step offset of the replay
    int32_t *base_host = nullptr;       // pinned, one per replay of a call
    int64_t base_cap = 0;
    // timing of the last call
    double last_ms = 0;
    int64_t launches = 0, graph_launches = 0, graph_nodes = 0;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~dgt_batch() {
        drop_graph();
        if (amp_host) (void)hipHostFree(amp_host);
        if (base_host) (void)hipHostFree(base_host);
        if (amp_ev) (void)hipEventDestroy(amp_ev);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (join) (void)hipEventDestroy(join);
        if (gst) (void)hipStreamDestroy(gst);
    }
};

namespace dgt {

template <class F>
static void dispatch_batch(const dgt_batch *b, F &&f) {
    switch (b->K * 2 + b->fp32) {
    case 2: f.template operator()<1, double>(); break;
    case 3: f.template operator()<1, float>(); break;
    case 4: f.template operator()<2, double>(); break;
    case 5: f.template operator()<2, float>(); break;
    default: throw Error{DGT_EUNSUPPORTED, "batched launches are built for degrees 1 and 2"};
    }
}

// launch arguments of member `mi` for sub-chain `bi`: the dependence-driven form of
// its own plan with the batch's counters (the epoch and source amplitude of a
// launch come with the batch arguments)
static TileArgs batch_member_args(dgt_batch *b, int bi, int mi, int persist) {
    dgt_solver *s = b->m[mi];
    const SubPlan &P = s->plan[bi];
    const SubSched &sb = s->sched->s->sub[bi];
    TileArgs A = P.args;
    for (int f = 0; f < F_COUNT; ++f) {
        A.F[f] = s->fld[f].p;
        A.fshot[f] = s->fshot(f);
    }
    A.nshots = s->nshots;
    A.src_cells = s->src_cells.p;
    A.src_vec = s->src_vec.p;
    A.dt = s->p.dt;
    A.src_amp = 0.0;
    A.persist = persist;
    A.ntiles = P.ntiles;
    A.nexec = P.nexec;
    A.tile_base = 0;
    A.need = sb.dep_need.p;
    A.succ_off = sb.dep_off.p;
    A.succ = sb.dep_succ.p;
    A.cnt = b->sub[bi].cnt[mi].p;
    A.head = b->sub[bi].head.p;
    A.err = b->err.p;
    A.epoch = 0;
    A.head_base = 0;
    A.spin_limit = s->wait_limit;
    return A;
}

static BatchArgs batch_args(dgt_batch *b, int bi, uint32_t epoch) {
    dgt_batch::Sub &S = b->sub[bi];
    BatchArgs B{};
    B.args = S.args.p;
    B.persist = 1;
    B.seg_first = 0;
    B.epoch = epoch;
    B.amp_tab = b->amp.p;
    B.amp_stride = (int32_t)b->amp_cap;
    B.nseg = S.nseg;
    B.seg_start = S.seg_start.p;
    B.seg_mesh = S.seg_mesh.p;
    B.seg_local = S.seg_local.p;
    B.head = S.head.p;
    B.head_base = (epoch - 1u) * (S.total + (uint32_t)S.slots);
    B.total = S.total;
    return B;
}

static void batch_check_members(dgt_batch *b) {
    for (size_t i = 0; i < b->m.size(); ++i)
        DGT_REQUIRE(b->m[i]->gen == b->gen[i], DGT_ESTATE,
                    "a member solver was inspected again or its shots changed: create the batch again");
}

// reports (and clears) a dependence wait that gave up in an earlier call
static void batch_check_errors(dgt_batch *b) {
    int32_t e = 0;
    DGT_HIP(hipMemcpyAsync(&e, b->err.p, sizeof(e), hipMemcpyDeviceToHost, b->user));
    DGT_HIP(hipStreamSynchronize(b->user));
    if (!e) return;
    for (auto &S : b->sub) {
        for (size_t i = 0; i < S.cnt.size(); ++i)
            DGT_HIP(hipMemsetAsync(S.cnt[i].p, 0, S.cnt[i].n * sizeof(uint32_t), b->user));
        DGT_HIP(hipMemsetAsync(S.head.p, 0, sizeof(uint32_t), b->user));
        S.epoch = 0;
    }
    DGT_HIP(hipMemsetAsync(b->err.p, 0, sizeof(int32_t), b->user));
    DGT_REQUIRE(false, DGT_ESTATE, "a dependence wait of the batched executor timed out; its results are invalid");
}

// clears the counters on stream st (outside any graph)
static void batch_reset_counters(dgt_batch *b, hipStream_t st) {
    for (auto &S : b->sub) {
        for (size_t i = 0; i < S.cnt.size(); ++i)
            DGT_HIP(hipMemsetAsync(S.cnt[i].p, 0, S.cnt[i].n * sizeof(uint32_t), st));
        DGT_HIP(hipMemsetAsync(S.head.p, 0, sizeof(uint32_t), st));
        S.epoch = 0;
    }
}

// colour c of sub-chain bi: one workgroup per item of every member
static BatchArgs batch_colour_args(dgt_batch *b, int bi, int c) {
    dgt_batch::Sub &S = b->sub[bi];
    BatchArgs B{};
    B.args = S.args_c.p;
    B.persist = 0;
    B.seg_first = S.cseg[c];
    B.nseg = S.cseg[c + 1] - S.cseg[c];
    B.ticket_base = S.cstart[c];
    B.seg_start = S.seg_start.p;
    B.seg_mesh = S.seg_mesh.p;
    B.seg_local = S.seg_local.p;
    B.total = S.cstart[c + 1] - S.cstart[c];
    B.amp_tab = b->amp.p;
    B.amp_stride = (int32_t)b->amp_cap;
    return B;
}

template <int K, typename T>
static void batch_launch(dgt_batch *b, int bi, const BatchArgs &B, hipStream_t st) {
    const dgt_batch::Sub &S = b->sub[bi];
    tile_launch_batch<K, T>(b->upw, b->order, S.o0, S.nops, S.nt, B.persist ? S.slots : (int)B.total, S.lds, st, B,
                            TA_LAUNCH);
}

// the launches of step q of sub-chain bi (amp_base: the replay's offset, or NULL)
template <int K, typename T>
static void batch_launch_step(dgt_batch *b, int bi, uint32_t epoch, const int32_t *amp_base, int32_t amp_idx,
                              hipStream_t st) {
    dgt_batch::Sub &S = b->sub[bi];
    if (b->sched == 1) {
        BatchArgs B = batch_args(b, bi, epoch);
        B.amp_base = amp_base;
        B.amp_idx = amp_idx;
        batch_launch<K, T>(b, bi, B, st);
        ++b->launches;
        return;
    }
    for (size_t c = 0; c + 1 < S.cstart.size(); ++c) {
        if (S.cstart[c + 1] == S.cstart[c]) continue;
        BatchArgs B = batch_colour_args(b, bi, (int)c);
        B.amp_base = amp_base;
        B.amp_idx = amp_idx;
        batch_launch<K, T>(b, bi, B, st);
        ++b->launches;
    }
}

// steps [first, first + n) of the call, launched one by one (amplitudes at those indices)
template <int K, typename T>
static void batch_eager(dgt_batch *b, int64_t first, int64_t n) {
    for (int64_t q = first; q < first + n; ++q)
        for (int bi = 0; bi < b->nsub; ++bi) {
            dgt_batch::Sub &S = b->sub[bi];
            const uint32_t ep = b->sched == 1 ? ++S.epoch : 0u;
            batch_launch_step<K, T>(b, bi, ep, nullptr, (int32_t)q, b->user);
        }
}

// captures gsteps steps (kernel nodes only) on the batch's own stream
template <int K, typename T>
static void batch_capture(dgt_batch *b) {
    const int G = b->gsteps;
    DGT_HIP(hipStreamBeginCapture(b->gst, hipStreamCaptureModeThreadLocal));
    try {
        const int64_t before = b->launches;
        for (int k = 0; k < G; ++k)
            for (int bi = 0; bi < b->nsub; ++bi) batch_launch_step<K, T>(b, bi, (uint32_t)(k + 1), b->amp_base.p, k, b->gst);
        b->graph_nodes = b->launches - before;
        b->launches = before;
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->gst, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    DGT_HIP(hipStreamEndCapture(b->gst, &b->graph));
    DGT_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
}

// the source amplitudes of the call's nsteps steps, uploaded on the caller's stream
static void batch_amplitudes(dgt_batch *b, int64_t nsteps, const double *t0) {
    const size_t nm = b->m.size();
    const int64_t need = std::max<int64_t>(nsteps, 1);
    if (need > b->amp_cap) {
        b->drop_graph();  // the graph holds the table's address and stride
        if (b->amp_ev) DGT_HIP(hipEventSynchronize(b->amp_ev));
        if (b->amp_host) DGT_HIP(hipHostFree(b->amp_host));
        b->amp_host = nullptr;
        b->amp_cap = std::max<int64_t>(need, 2 * b->amp_cap);
        b->amp.alloc((size_t)b->amp_cap * nm);
        DGT_HIP(hipHostMalloc((void **)&b->amp_host, (size_t)b->amp_cap * nm * sizeof(double)));
    }
    if (b->amp_ev) DGT_HIP(hipEventSynchronize(b->amp_ev));  // the previous call's upload has read the buffer
    for (size_t i = 0; i < nm; ++i) {
        dgt_solver *s = b->m[i];
        double *row = b->amp_host + i * b->amp_cap;
        for (int64_t q = 0; q < nsteps; ++q)
            row[q] = s->has_src ? s->p.dt * ricker(t0[i] + ((double)q + 0.5) * s->p.dt, s->sf0, s->st0, s->samp) : 0.0;
    }
    DGT_HIP(hipMemcpyAsync(b->amp.p, b->amp_host, (size_t)b->amp_cap * nm * sizeof(double), hipMemcpyHostToDevice,
                           b->user));
    DGT_HIP(hipEventRecord(b->amp_ev, b->user));
}

template <int K, typename T>
static void batch_step(dgt_batch *b, int64_t nsteps, const double *t0) {
    batch_amplitudes(b, nsteps, t0);
    if (b->gsteps == 0 || nsteps < b->gsteps) {
        batch_eager<K, T>(b, 0, nsteps);
        return;
    }
    const int G = b->gsteps;
    const int64_t nrep = nsteps / G, rem = nsteps % G;
    if (!b->exec) batch_capture<K, T>(b);
    if (nrep > b->base_cap) {
        DGT_HIP(hipStreamSynchronize(b->gst));
        if (b->base_host) DGT_HIP(hipHostFree(b->base_host));
        b->base_host = nullptr;
        b->base_cap = std::max<int64_t>(nrep, 2 * b->base_cap);
        DGT_HIP(hipHostMalloc((void **)&b->base_host, (size_t)b->base_cap * sizeof(int32_t)));
    }
    // the own stream follows the caller's work (the amplitudes among it), the caller's
    // stream the replays
    DGT_HIP(hipStreamSynchronize(b->gst));  // the previous call's replays have read base_host
    DGT_HIP(hipEventRecord(b->join, b->user));
    DGT_HIP(hipStreamWaitEvent(b->gst, b->join, 0));
    for (int64_t r = 0; r < nrep; ++r) {
        if (b->sched == 1) batch_reset_counters(b, b->gst);  // outside the graph
        b->base_host[r] = (int32_t)(r * G);
        DGT_HIP(hipMemcpyAsync(b->amp_base.p, b->base_host + r, sizeof(int32_t), hipMemcpyHostToDevice, b->gst));
        DGT_HIP(hipGraphLaunch(b->exec, b->gst));
        ++b->graph_launches;
        b->launches += b->graph_nodes;
    }
    // the counters now hold G epochs of every sub-chain: the remaining steps continue them
    if (b->sched == 1)
        for (auto &S : b->sub) S.epoch = (uint32_t)G;
    DGT_HIP(hipEventRecord(b->join, b->gst));
    DGT_HIP(hipStreamWaitEvent(b->user, b->join, 0));
    if (rem) batch_eager<K, T>(b, nrep * G, rem);
}

}  // namespace dgt

extern "C" {

dgt_status dgt_batch_create(dgt_solver *const *solvers, int32_t n, void *stream, dgt_batch **out) {
    return guard([&] {
        DGT_REQUIRE(solvers && out && n >= 1 && n <= 4096, DGT_EINVAL, "bad arguments");
        *out = nullptr;
        auto b = std::make_unique<dgt_batch>();
        b->user = (hipStream_t)stream;
        const dgt_solver *s0 = solvers[0];
        DGT_REQUIRE(s0, DGT_EINVAL, "NULL solver");
        b->K = s0->K;
        b->fp32 = s0->fp32;
        b->upw = s0->upw;
        b->order = s0->p.time_order;
        DGT_REQUIRE(b->K <= 2, DGT_EUNSUPPORTED, "batched launches are built for degrees 1 and 2");
        for (int32_t i = 0; i < n; ++i) {
            dgt_solver *s = solvers[i];
            DGT_REQUIRE(s, DGT_EINVAL, "NULL solver");
            for (int32_t j = 0; j < i; ++j) DGT_REQUIRE(solvers[j] != s, DGT_EINVAL, "a solver appears twice");
            DGT_REQUIRE(s->plan_status == DGT_OK && s->inspected, DGT_ESTATE,
                        "every member must be inspected with a usable plan");
            DGT_REQUIRE(s->K == b->K && s->fp32 == b->fp32 && s->upw == b->upw && s->p.time_order == b->order,
                        DGT_EINVAL, "members differ in degree, precision, flux or time order");
            DGT_REQUIRE(s->plan.size() == s0->plan.size(), DGT_EINVAL, "members differ in their fusion scheme");
            for (size_t q = 0; q < s->plan.size(); ++q) {
                const SubPlan &P = s->plan[q], &P0 = s0->plan[q];
                DGT_REQUIRE(P.kind == TK_CHAIN && P.o0 == P0.o0 && P.nops == P0.nops && P.first == P0.first &&
                                P.n == P0.n,
                            DGT_EINVAL, "members must run the same chain-kernel sub-chains");
                DGT_REQUIRE(P.tne < 0, DGT_EINVAL, "a member inspected with regions runs on its own");
                DGT_REQUIRE(s->fuse == 1, DGT_EINVAL, "a member fused over several steps runs on its own");
            }
            b->m.push_back(s);
            b->gen.push_back(s->gen);
        }
        b->nsub = (int)s0->plan.size();
        DGT_HIP(hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking));
        DGT_HIP(hipEventCreate(&b->ev0));
        DGT_HIP(hipEventCreate(&b->ev1));
        DGT_HIP(hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
        DGT_HIP(hipEventCreateWithFlags(&b->amp_ev, hipEventDisableTiming));
        b->err.alloc(1);
        DGT_HIP(hipMemsetAsync(b->err.p, 0, sizeof(int32_t), b->user));
        b->amp_base.alloc(1);
        DGT_HIP(hipMemsetAsync(b->amp_base.p, 0, sizeof(int32_t), b->user));
        int dev = 0;
        DGT_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        DGT_HIP(hipGetDeviceProperties(&prop, dev));
        b->sub.resize(b->nsub);
        for (int bi = 0; bi < b->nsub; ++bi) {
            dgt_batch::Sub &S = b->sub[bi];
            S.o0 = s0->plan[bi].o0;
            S.nops = s0->plan[bi].nops;
            std::vector<int32_t> st, me, lo;
            int maxc = 0;
            for (auto *s : b->m) {
                S.nt = std::max(S.nt, s->plan[bi].threads);
                S.lds = std::max(S.lds, s->plan[bi].lds_bytes);
                maxc = std::max(maxc, s->plan[bi].ncolors);
            }
            S.nt = std::max(S.nt, 256);
            uint64_t t = 0;
            for (int c = 0; c < maxc; ++c) {
                S.cseg.push_back((int32_t)me.size());
                S.cstart.push_back((uint32_t)t);
                for (size_t i = 0; i < b->m.size(); ++i) {
                    const SubPlan &P = b->m[i]->plan[bi];
                    if (c >= P.ncolors) continue;
                    const int64_t cnt = (int64_t)(P.color_off[c + 1] - P.color_off[c]) * b->m[i]->nshots;
                    if (cnt == 0) continue;
                    st.push_back((int32_t)t);
                    me.push_back((int32_t)i);
                    lo.push_back((int32_t)((int64_t)P.color_off[c] * b->m[i]->nshots));
                    t += (uint64_t)cnt;
                }
            }
            S.cseg.push_back((int32_t)me.size());
            S.cstart.push_back((uint32_t)t);
            DGT_REQUIRE(t < (1ull << 31), DGT_EUNSUPPORTED, "more than 2^31 work items in one batched launch");
            st.push_back((int32_t)t);
            S.nseg = (int)me.size();
            S.total = (uint32_t)t;
            S.seg_start.upload(st, b->user);
            S.seg_mesh.upload(me.empty() ? std::vector<int32_t>{0} : me, b->user);
            S.seg_local.upload(lo.empty() ? std::vector<int32_t>{0} : lo, b->user);
            S.cnt.resize(b->m.size());
            for (size_t i = 0; i < b->m.size(); ++i) {
                const size_t c = (size_t)b->m[i]->plan[bi].ntiles * b->m[i]->nshots;
                S.cnt[i].alloc(std::max<size_t>(c, 1));
                DGT_HIP(hipMemsetAsync(S.cnt[i].p, 0, S.cnt[i].n * sizeof(uint32_t), b->user));
            }
            S.head.alloc(1);
            DGT_HIP(hipMemsetAsync(S.head.p, 0, sizeof(uint32_t), b->user));
            std::vector<TileArgs> margs, cargs;
            for (size_t i = 0; i < b->m.size(); ++i) {
                margs.push_back(batch_member_args(b.get(), bi, (int)i, 1));
                cargs.push_back(batch_member_args(b.get(), bi, (int)i, 0));
            }
            S.args.upload(margs, b->user);
            S.args_c.upload(cargs, b->user);
            DGT_HIP(hipStreamSynchronize(b->user));
            int occ = 0;
            dgt_batch *bp = b.get();
            BatchArgs B{};
            dispatch_batch(bp, [&]<int KK, typename T>() {
                tile_launch_batch<KK, T>(bp->upw, bp->order, S.o0, S.nops, S.nt, 0, S.lds, bp->user, B, TA_ATTR);
                tile_launch_batch<KK, T>(bp->upw, bp->order, S.o0, S.nops, S.nt, 0, S.lds, bp->user, B, TA_OCCUPANCY,
                                         &occ);
            });
            DGT_REQUIRE(occ > 0, DGT_EUNSUPPORTED, "the batched tile kernel does not fit on a compute unit");
            S.slots = occ * prop.multiProcessorCount;
        }
        DGT_HIP(hipStreamSynchronize(b->user));
        *out = b.release();
    });
}

dgt_status dgt_batch_set_graph(dgt_batch *b, int32_t steps_per_graph) {
    return guard([&] {
        DGT_REQUIRE(b && steps_per_graph >= 0 && steps_per_graph <= 4096, DGT_EINVAL, "bad arguments");
        if (steps_per_graph != b->gsteps) b->drop_graph();
        b->gsteps = steps_per_graph;
    });
}

dgt_status dgt_batch_set_schedule(dgt_batch *b, int32_t mode) {
    return guard([&] {
        DGT_REQUIRE(b && (mode == 0 || mode == 1), DGT_EINVAL, "bad arguments");
        if (mode != b->sched) b->drop_graph();
        b->sched = mode;
    });
}

dgt_status dgt_batch_step(dgt_batch *b, int64_t nsteps, const double *t0) {
    return guard([&] {
        DGT_REQUIRE(b && t0 && nsteps >= 0, DGT_EINVAL, "bad arguments");
        batch_check_members(b);
        for (auto *s : b->m) DGT_REQUIRE(s->state_valid, DGT_ESTATE, "a member has no state uploaded");
        batch_check_errors(b);
        b->launches = 0;
        b->graph_launches = 0;
        DGT_HIP(hipEventRecord(b->ev0, b->user));
        dispatch_batch(b, [&]<int K, typename T>() {
            for (int bi = 0; bi < b->nsub; ++bi)
                tile_launch_batch<K, T>(b->upw, b->order, b->sub[bi].o0, b->sub[bi].nops, b->sub[bi].nt, 0,
                                        b->sub[bi].lds, b->user, BatchArgs{}, TA_ATTR);
            batch_step<K, T>(b, nsteps, t0);
        });
        DGT_HIP(hipGetLastError());
        DGT_HIP(hipEventRecord(b->ev1, b->user));
        b->last_ms = -1.0;
    });
}

dgt_status dgt_batch_timing(dgt_batch *b, double *ms, int64_t *launches, int64_t *graph_launches) {
    return guard([&] {
        DGT_REQUIRE(b, DGT_EINVAL, "batch is NULL");
        if (b->last_ms < 0) {
            DGT_HIP(hipEventSynchronize(b->ev1));
            float f = 0;
            DGT_HIP(hipEventElapsedTime(&f, b->ev0, b->ev1));
            b->last_ms = f;
        }
        if (ms) *ms = b->last_ms;
        if (launches) *launches = b->launches;
        if (graph_launches) *graph_launches = b->graph_launches;
    });
}

void dgt_batch_destroy(dgt_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->gst);
    (void)hipStreamSynchronize(b->user);
    delete b;
}

}  // extern "C"
