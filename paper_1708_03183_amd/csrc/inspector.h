// Loop chain model and GPU inspector of libdgtile (internal).
#pragma once
#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace dgt {

constexpr int kMaxSets = 8, kMaxMaps = 8, kMaxLoops = 64, kMaxDesc = 8;

struct ChainMap {
    int from = 0, to = 0, arity = 1;
    std::vector<int32_t> values;
};

struct ChainLoop {
    int set = 0, ndesc = 0;
    dgt_desc d[kMaxDesc];
};

// Sets, maps and loops of a loop chain (Sec. 2); host copy.
struct ChainDesc {
    int nsets = 0, nmaps = 0, nloops = 0;
    int64_t size[kMaxSets] = {0};
    ChainMap maps[kMaxMaps];
    ChainLoop loops[kMaxLoops];
};

// One sub-chain of a fusion scheme: its tiles, colours and footprints.
struct SubSched {
    int first = 0, n = 0;
    int32_t ntiles = 0, ncolors = 0, rounds = 0;
    DBuf<int32_t> color, color_off, tiles_by_color;
    int64_t foot_len[kMaxSets] = {0};
    DBuf<int32_t> foot_off[kMaxSets], foot[kMaxSets];
    DBuf<uint32_t> acc[kMaxSets];
    // dependence graph for the dependence-driven executor: edge a -> b when the
    // footprints of tiles a and b share an element of any set and a has the lower colour
    int64_t dep_edges = 0;
    DBuf<int32_t> dep_need, dep_off, dep_succ;  // [ntiles], [ntiles+1], [dep_edges]
    // regions (Sec. 3.3): core tiles [0, ncore), boundary tiles [ncore, tne), the
    // never-executed tile tne (highest colour); tne < 0 without regions
    int32_t ncore = 0, nbnd = 0, tne = -1;
    std::vector<uint8_t> region;  // seed regions this sub-chain was inspected with
};

// Output of the inspector, resident in device memory.
struct Schedule {
    int nloops = 0;
    std::vector<SubSched> sub;
    int64_t loop_size[kMaxLoops] = {0};
    int sub_of[kMaxLoops] = {0};
    DBuf<int32_t> sigma[kMaxLoops], it_off[kMaxLoops], iters[kMaxLoops];
    DBuf<int32_t> seed_rank;  // position of each seed iteration in the seed order
    int seed_set = 0;
    double gpu_ms = 0, wall_ms = 0;
    hipStream_t stream = nullptr;
};

// device radix sorts (unique keys give deterministic results)
void sort_keys(DBuf<uint64_t> &keys, int64_t n, hipStream_t st, int end_bit = 64);
void sort_pairs(DBuf<uint64_t> &keys, DBuf<uint32_t> &vals, int64_t n, hipStream_t st);

class Inspector {
   public:
    Inspector(const ChainDesc &c, hipStream_t st);
    std::unique_ptr<Schedule> run(int64_t ts, int partition, const double *xy_host, const double *xy_dev,
                                  int max_rounds, int cap, const std::vector<int32_t> &splits,
                                  const std::vector<int32_t> &sub_ts = {}, const uint8_t *region = nullptr,
                                  int carry = 0);
    const ChainDesc &chain;
    hipStream_t stream;
    DBuf<int32_t> dmap[kMaxMaps], inv_off[kMaxMaps], inv_val[kMaxMaps];

   private:
    Schedule *cur = nullptr;
    // unique touches of each set from the last conflict pass (reused by footprints)
    bool tk_valid = false;
    int64_t tk_len[kMaxSets] = {0};
    DBuf<uint64_t> tk_keys[kMaxSets];
    DBuf<uint32_t> tk_bits[kMaxSets];
    void build_inverse(const ChainDesc &c, int mi, hipStream_t st);
    void seed_partition(int seedset, int64_t ts, int partition, const double *xy_host, const double *xy_dev,
                        DBuf<int32_t> &tile0, DBuf<int32_t> &rank);
    void region_partition(int64_t n0, int64_t ts, const DBuf<int32_t> &rank, SubSched &sb, DBuf<int32_t> &tile0);
    int64_t seed_edges(int first, int nl, const DBuf<int32_t> &tile0, DBuf<uint64_t> &edges);
    int colour(int32_t ntiles, const DBuf<uint64_t> &edges, int64_t ne, DBuf<int32_t> &color, int cap,
               const SubSched *regions = nullptr);
    void run_sub(Schedule &S, SubSched &sb, int64_t ts, int partition, const double *xy_host,
                 const double *xy_dev, int max_rounds, int cap);
    void carry_stale(const Schedule &S, const SubSched &sb, std::vector<uint8_t> &region);
    int64_t touches(int first, int nl, int s, DBuf<uint64_t> &keys, DBuf<uint32_t> &bits, const Schedule &S);
    int64_t conflicts(int first, int nl, const DBuf<int32_t> &color, DBuf<uint64_t> &edges, int64_t &ne);
    void footprints(int first, int nl, SubSched &sb);
    void dependences(SubSched &sb, const DBuf<uint64_t> *keys, const int64_t *len);
};

}  // namespace dgt

struct dgt_chain {
    dgt::ChainDesc c;
};

struct dgt_schedule {
    std::unique_ptr<dgt::Schedule> s;
    const dgt::ChainDesc *chain = nullptr;  // chain sizes for read-back
    dgt::ChainDesc chain_copy;
};
