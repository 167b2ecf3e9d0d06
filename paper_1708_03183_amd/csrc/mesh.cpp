// Host-side mesh derivation of libdgtile (set-up only): facet maps and
// boundary sides from cell-to-vertex connectivity.
//
// Numbering convention shared with every other user of these maps: local
// facet l of a cell joins its vertices l and l+1 (mod 3); interior facets are
// listed by ascending lower cell id and local facet, exterior facets by
// ascending cell id and local facet.
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace dgt {

Mesh build_mesh(int64_t nv, const double *xy, int64_t nc, const int32_t *c2v, int periodic) {
    DGT_REQUIRE(nv >= 0 && nc >= 0 && (nv == 0 || xy) && (nc == 0 || c2v), DGT_EINVAL, "bad mesh arrays");
    DGT_REQUIRE(nc < (int64_t)1 << 30, DGT_EINVAL, "too many cells");
    Mesh m;
    m.nv = nv;
    m.nc = nc;
    m.xy.assign(xy, xy + 2 * nv);
    m.c2v.assign(c2v, c2v + 3 * nc);
    for (int64_t i = 0; i < 3 * nc; ++i)
        DGT_REQUIRE(c2v[i] >= 0 && c2v[i] < nv, DGT_EINVAL, "vertex id out of range");
    for (int64_t c = 0; c < nc; ++c) {
        const double *a = xy + 2 * c2v[3 * c], *b = xy + 2 * c2v[3 * c + 1], *d = xy + 2 * c2v[3 * c + 2];
        const double det = (b[0] - a[0]) * (d[1] - a[1]) - (d[0] - a[0]) * (b[1] - a[1]);
        DGT_REQUIRE(det > 0.0, DGT_EINVAL, "cell " + std::to_string(c) + " is clockwise or degenerate");
    }
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int64_t v = 0; v < nv; ++v)
        for (int a = 0; a < 2; ++a) {
            lo[a] = std::min(lo[a], xy[2 * v + a]);
            hi[a] = std::max(hi[a], xy[2 * v + a]);
        }
    for (int a = 0; a < 2; ++a) {
        m.bbox[2 * a] = lo[a];
        m.bbox[2 * a + 1] = hi[a];
    }
    // neighbour across each (cell, local facet) by hashing the vertex pair
    std::vector<int32_t> nbr(3 * nc, -1);
    std::vector<int8_t> nbrl(3 * nc, -1);
    std::unordered_map<uint64_t, int64_t> open;
    open.reserve((size_t)(3 * nc / 2 + 16));
    for (int64_t c = 0; c < nc; ++c)
        for (int l = 0; l < 3; ++l) {
            const uint32_t a = (uint32_t)c2v[3 * c + l], b = (uint32_t)c2v[3 * c + (l + 1) % 3];
            const uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            auto it = open.find(key);
            if (it == open.end()) {
                open.emplace(key, 3 * c + l);
            } else {
                const int64_t o = it->second;
                DGT_REQUIRE(o >= 0, DGT_EINVAL, "an edge is shared by more than two cells");
                const int64_t oc = o / 3;
                const int ol = (int)(o % 3);
                nbr[3 * c + l] = (int32_t)oc;
                nbrl[3 * c + l] = (int8_t)ol;
                nbr[o] = (int32_t)c;
                nbrl[o] = (int8_t)l;
                it->second = -1;  // closed: a third cell would be an error
            }
        }
    const double ext = std::max(hi[0] - lo[0], hi[1] - lo[1]);
    const double tol = 1e-9 * (ext > 0 ? ext : 1.0);
    // periodic pairing: boundary edges on opposite sides, sorted by midpoint
    for (int dir = 0; dir < 2; ++dir) {
        if (!(periodic & (1 << dir))) continue;
        std::vector<std::pair<double, int64_t>> side[2];
        for (int64_t c = 0; c < nc; ++c)
            for (int l = 0; l < 3; ++l) {
                if (nbr[3 * c + l] >= 0) continue;
                const double *pa = xy + 2 * c2v[3 * c + l], *pb = xy + 2 * c2v[3 * c + (l + 1) % 3];
                for (int sd = 0; sd < 2; ++sd) {
                    const double wall = sd ? hi[dir] : lo[dir];
                    if (std::fabs(pa[dir] - wall) <= tol && std::fabs(pb[dir] - wall) <= tol)
                        side[sd].push_back({0.5 * (pa[1 - dir] + pb[1 - dir]), 3 * c + l});
                }
            }
        DGT_REQUIRE(side[0].size() == side[1].size(), DGT_EINVAL, "periodic sides do not match");
        std::sort(side[0].begin(), side[0].end());
        std::sort(side[1].begin(), side[1].end());
        for (size_t i = 0; i < side[0].size(); ++i) {
            DGT_REQUIRE(std::fabs(side[0][i].first - side[1][i].first) <= tol, DGT_EINVAL,
                        "periodic edges do not line up");
            const int64_t a = side[0][i].second, b = side[1][i].second;
            nbr[a] = (int32_t)(b / 3);
            nbrl[a] = (int8_t)(b % 3);
            nbr[b] = (int32_t)(a / 3);
            nbrl[b] = (int8_t)(a % 3);
        }
    }
    for (int64_t c = 0; c < nc; ++c)
        for (int l = 0; l < 3; ++l) {
            const int32_t o = nbr[3 * c + l];
            DGT_REQUIRE(o != c, DGT_EINVAL, "a cell neighbours itself");
            if (o < 0) {
                m.b2c.push_back((int32_t)c);
                m.b2l.push_back((int8_t)l);
                const double *pa = xy + 2 * c2v[3 * c + l], *pb = xy + 2 * c2v[3 * c + (l + 1) % 3];
                const double mx = 0.5 * (pa[0] + pb[0]), my = 0.5 * (pa[1] + pb[1]);
                int8_t sd = -1;
                if (std::fabs(mx - lo[0]) <= tol) sd = 0;
                else if (std::fabs(mx - hi[0]) <= tol) sd = 1;
                else if (std::fabs(my - lo[1]) <= tol) sd = 2;
                else if (std::fabs(my - hi[1]) <= tol) sd = 3;
                m.bside.push_back(sd);
            } else if (o > c) {
                m.f2c.push_back((int32_t)c);
                m.f2c.push_back(o);
                m.f2l.push_back((int8_t)l);
                m.f2l.push_back(nbrl[3 * c + l]);
            }
        }
    m.nf = (int64_t)m.f2l.size() / 2;
    m.nb = (int64_t)m.b2c.size();
    return m;
}

}  // namespace dgt
