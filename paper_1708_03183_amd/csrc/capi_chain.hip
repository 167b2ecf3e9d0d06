// C ABI of tier 1: loop chain, GPU inspector, schedule read-back.
#include <cstring>
#include <sstream>

#include "common.h"
#include "inspector.h"

namespace dgt {

static thread_local std::string g_last_error = "no error";

dgt_status fail(dgt_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

}  // namespace dgt

using namespace dgt;

extern "C" {

const char *dgt_last_error(void) { return g_last_error.c_str(); }

int dgt_version(void) { return 107; }

dgt_status dgt_chain_create(dgt_chain **out) {
    return guard([&] {
        DGT_REQUIRE(out, DGT_EINVAL, "out is NULL");
        *out = new dgt_chain();
    });
}

dgt_status dgt_chain_set(dgt_chain *c, int64_t size, int32_t *set_id) {
    return guard([&] {
        DGT_REQUIRE(c && size >= 0 && size < (int64_t)INT32_MAX, DGT_EINVAL, "bad set size");
        DGT_REQUIRE(c->c.nsets < kMaxSets, DGT_EINVAL, "too many sets");
        c->c.size[c->c.nsets] = size;
        if (set_id) *set_id = c->c.nsets;
        c->c.nsets++;
    });
}

dgt_status dgt_chain_map(dgt_chain *c, int32_t from, int32_t to, int32_t arity, const int32_t *values,
                         int32_t *map_id) {
    return guard([&] {
        DGT_REQUIRE(c, DGT_EINVAL, "chain is NULL");
        DGT_REQUIRE(c->c.nmaps < kMaxMaps, DGT_EINVAL, "too many maps");
        DGT_REQUIRE(from >= 0 && from < c->c.nsets && to >= 0 && to < c->c.nsets && arity >= 1 && arity <= 8,
                    DGT_EINVAL, "bad map sets or arity");
        const int64_t n = c->c.size[from] * arity;
        DGT_REQUIRE(n == 0 || values, DGT_EINVAL, "map values are NULL");
        for (int64_t i = 0; i < n; ++i)
            DGT_REQUIRE(values[i] >= 0 && values[i] < c->c.size[to], DGT_EINVAL, "map value out of range");
        ChainMap &m = c->c.maps[c->c.nmaps];
        m.from = from;
        m.to = to;
        m.arity = arity;
        m.values.assign(values, values + n);
        if (map_id) *map_id = c->c.nmaps;
        c->c.nmaps++;
    });
}

dgt_status dgt_chain_loop(dgt_chain *c, int32_t set, int32_t ndesc, const dgt_desc *desc, int32_t *loop_id) {
    return guard([&] {
        DGT_REQUIRE(c, DGT_EINVAL, "chain is NULL");
        DGT_REQUIRE(c->c.nloops < kMaxLoops, DGT_EINVAL, "too many loops");
        DGT_REQUIRE(set >= 0 && set < c->c.nsets && ndesc >= 0 && ndesc <= kMaxDesc, DGT_EINVAL, "bad loop");
        ChainLoop &L = c->c.loops[c->c.nloops];
        L.set = set;
        L.ndesc = ndesc;
        for (int i = 0; i < ndesc; ++i) {
            const dgt_desc &d = desc[i];
            DGT_REQUIRE(d.map >= -1 && d.map < c->c.nmaps, DGT_EINVAL, "bad descriptor map");
            DGT_REQUIRE(d.map < 0 || c->c.maps[d.map].from == set, DGT_EINVAL, "descriptor map does not start at the loop set");
            DGT_REQUIRE(d.mode >= 0 && d.mode <= 2, DGT_EINVAL, "bad descriptor mode");
            L.d[i] = d;
        }
        if (loop_id) *loop_id = c->c.nloops;
        c->c.nloops++;
    });
}

void dgt_chain_destroy(dgt_chain *c) { delete c; }

dgt_status dgt_inspect(const dgt_chain *c, const dgt_inspect_params *p, void *stream, dgt_schedule **out) {
    return guard([&] {
        DGT_REQUIRE(c && p && out, DGT_EINVAL, "NULL argument");
        *out = nullptr;
        DGT_REQUIRE(p->partition == 0 || p->partition == 1, DGT_EINVAL, "partition must be 0 or 1");
        DGT_REQUIRE(p->nsplits >= 0 && (p->nsplits == 0 || p->splits), DGT_EINVAL, "bad splits");
        auto sch = std::make_unique<dgt_schedule>();
        sch->chain_copy = c->c;
        sch->chain = &sch->chain_copy;
        hipStream_t st = (hipStream_t)stream;
        Inspector insp(sch->chain_copy, st);
        std::vector<int32_t> splits(p->splits, p->splits + p->nsplits);
        DGT_REQUIRE(p->max_colour_tiles >= 0, DGT_EINVAL, "max_colour_tiles must be >= 0");
        std::vector<int32_t> sub_ts;
        if (p->sub_tile_sizes) sub_ts.assign(p->sub_tile_sizes, p->sub_tile_sizes + p->nsplits + 1);
        sch->s = insp.run(p->tile_size, p->partition, p->seed_xy, nullptr, p->max_conflict_rounds,
                          p->max_colour_tiles, splits, sub_ts, p->seed_region, p->region_carry);
        *out = sch.release();
    });
}

static const SubSched &sub_of(const dgt_schedule *s, int32_t sub) {
    DGT_REQUIRE(s && s->s && sub >= 0 && sub < (int)s->s->sub.size(), DGT_EINVAL, "bad sub-chain index");
    return s->s->sub[sub];
}

dgt_status dgt_schedule_nsub(const dgt_schedule *s, int32_t *nsub) {
    return guard([&] {
        DGT_REQUIRE(s && s->s && nsub, DGT_EINVAL, "NULL argument");
        *nsub = (int32_t)s->s->sub.size();
    });
}

dgt_status dgt_schedule_sub_info(const dgt_schedule *s, int32_t sub, int32_t *first_loop, int32_t *nloops,
                                 int32_t *ntiles, int32_t *ncolors, int32_t *rounds) {
    return guard([&] {
        const SubSched &b = sub_of(s, sub);
        if (first_loop) *first_loop = b.first;
        if (nloops) *nloops = b.n;
        if (ntiles) *ntiles = b.ntiles;
        if (ncolors) *ncolors = b.ncolors;
        if (rounds) *rounds = b.rounds;
    });
}

dgt_status dgt_schedule_colors(const dgt_schedule *s, int32_t sub, int32_t *color) {
    return guard([&] {
        const SubSched &b = sub_of(s, sub);
        auto h = b.color.download(s->s->stream, b.ntiles);
        std::memcpy(color, h.data(), sizeof(int32_t) * b.ntiles);
    });
}

dgt_status dgt_schedule_sigma(const dgt_schedule *s, int32_t loop, int32_t *sigma) {
    return guard([&] {
        DGT_REQUIRE(s && s->s && loop >= 0 && loop < s->s->nloops, DGT_EINVAL, "bad loop index");
        const int64_t n = s->s->loop_size[loop];
        auto h = s->s->sigma[loop].download(s->s->stream, n);
        if (n) std::memcpy(sigma, h.data(), sizeof(int32_t) * n);
    });
}

dgt_status dgt_schedule_iters(const dgt_schedule *s, int32_t loop, int32_t *tile_off, int32_t *iters) {
    return guard([&] {
        DGT_REQUIRE(s && s->s && loop >= 0 && loop < s->s->nloops, DGT_EINVAL, "bad loop index");
        const SubSched &b = s->s->sub[s->s->sub_of[loop]];
        const int64_t n = s->s->loop_size[loop];
        auto off = s->s->it_off[loop].download(s->s->stream, b.ntiles + 1);
        std::memcpy(tile_off, off.data(), sizeof(int32_t) * (b.ntiles + 1));
        auto it = s->s->iters[loop].download(s->s->stream, n);
        if (n) std::memcpy(iters, it.data(), sizeof(int32_t) * n);
    });
}

dgt_status dgt_schedule_footprint(const dgt_schedule *s, int32_t sub, int32_t set, int64_t *len, int32_t *off,
                                  int32_t *elem, uint32_t *acc) {
    return guard([&] {
        const SubSched &b = sub_of(s, sub);
        DGT_REQUIRE(set >= 0 && set < s->chain->nsets, DGT_EINVAL, "bad set");
        const int64_t m = b.foot_len[set];
        if (len) *len = m;
        if (off) {
            auto h = b.foot_off[set].download(s->s->stream, b.ntiles + 1);
            std::memcpy(off, h.data(), sizeof(int32_t) * (b.ntiles + 1));
        }
        if (elem && m) {
            auto h = b.foot[set].download(s->s->stream, m);
            std::memcpy(elem, h.data(), sizeof(int32_t) * m);
        }
        if (acc && m) {
            auto h = b.acc[set].download(s->s->stream, m);
            std::memcpy(acc, h.data(), sizeof(uint32_t) * m);
        }
    });
}

dgt_status dgt_schedule_tiles_by_color(const dgt_schedule *s, int32_t sub, int32_t *color_off, int32_t *tiles) {
    return guard([&] {
        const SubSched &b = sub_of(s, sub);
        auto co = b.color_off.download(s->s->stream, b.ncolors + 1);
        std::memcpy(color_off, co.data(), sizeof(int32_t) * (b.ncolors + 1));
        auto tl = b.tiles_by_color.download(s->s->stream, b.ntiles);
        std::memcpy(tiles, tl.data(), sizeof(int32_t) * b.ntiles);
    });
}

dgt_status dgt_schedule_regions(const dgt_schedule *s, int32_t sub, int32_t *info, uint8_t *region) {
    return guard([&] {
        const SubSched &b = sub_of(s, sub);
        DGT_REQUIRE(b.tne >= 0, DGT_EINVAL, "the schedule has no regions");
        if (info) {
            info[0] = b.ncore;
            info[1] = b.nbnd;
            info[2] = b.tne;
            info[3] = b.color.download(s->s->stream, b.ntiles)[b.tne];
        }
        if (region && !b.region.empty()) std::memcpy(region, b.region.data(), b.region.size());
    });
}

dgt_status dgt_schedule_summary_json(const dgt_schedule *s, char *buf, size_t len) {
    return guard([&] {
        DGT_REQUIRE(s && s->s && buf && len > 0, DGT_EINVAL, "NULL argument");
        std::ostringstream o;
        o << "{\"inspector_gpu_ms\": " << s->s->gpu_ms << ", \"inspector_wall_ms\": " << s->s->wall_ms
          << ", \"subchains\": [";
        for (size_t i = 0; i < s->s->sub.size(); ++i) {
            const SubSched &b = s->s->sub[i];
            if (i) o << ", ";
            o << "{\"first_loop\": " << b.first << ", \"nloops\": " << b.n << ", \"ntiles\": " << b.ntiles
              << ", \"ncolors\": " << b.ncolors << ", \"rounds\": " << b.rounds
              << ", \"dependences\": " << b.dep_edges << ", \"footprint\": [";
            for (int st = 0; st < s->chain->nsets; ++st) o << (st ? ", " : "") << b.foot_len[st];
            o << "]}";
        }
        o << "]}";
        std::string str = o.str();
        std::strncpy(buf, str.c_str(), len - 1);
        buf[len - 1] = '\0';
    });
}

void dgt_schedule_destroy(dgt_schedule *s) { delete s; }

}  // extern "C"
