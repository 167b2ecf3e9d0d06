// Nodal P_k reference triangle of libdgtile (host, set-up only).
#pragma once
#include <functional>
#include <vector>

namespace dgt {

struct RefElem {
    int k = 0, np = 0, nfp = 0;
    std::vector<double> nodes;   // [np][2]
    std::vector<double> M, Minv; // [np][np] reference mass and inverse
    std::vector<double> Dr, Ds;  // [np][np], D[i*np+j] = d phi_j / dr at node i
    std::vector<double> M1;      // [nfp][nfp] facet mass on [0,1]
    std::vector<double> lift;    // [3][np][nfp] = Minv E_f M1
    std::vector<int> fnodes;     // [3][nfp] cell node of facet node m
    std::function<void(double, double, double *)> phi;  // basis values at (r,s)
};

RefElem make_refelem(int k);

}  // namespace dgt
