// Host-side mesh of libdgtile (internal).
#pragma once
#include <vector>

#include "common.h"

namespace dgt {

struct Mesh {
    int64_t nv = 0, nc = 0, nf = 0, nb = 0;
    std::vector<double> xy;
    std::vector<int32_t> c2v;
    std::vector<int32_t> f2c, b2c;  // [nf][2], [nb]
    std::vector<int8_t> f2l, b2l, bside;
    double bbox[4] = {0, 0, 0, 0};  // xmin, xmax, ymin, ymax
};

Mesh build_mesh(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int periodic);

}  // namespace dgt

struct dgt_mesh {
    dgt::Mesh m;
};
