// Host FP64 geometry precompute of the immersed boundary (see precompute.cpp).
#pragma once

#include <array>
#include <string>
#include <vector>

namespace lbmib {

struct GeomInput {
    int dim;
    long long dims[3];      // nx, ny, nz (nz = 1 in 2D)
    int m;
    const double* X;        // m * dim
    const double* n;        // m * dim, outward unit normals
    int method;             // 0 DIBM, 1 FODIBM, 2 FODIBM-R
    int kernel;             // 0 cosine (d = 2), 1 ROMA3
};

struct Geometry {
    int dim = 0, m = 0, n_active = 0;
    std::vector<long long> supp_ptr, supp_node;      // one-sided (or DIBM two-sided) supports
    std::vector<double> supp_w;
    std::vector<std::array<long long, 3>> supp_c;
    std::vector<double> phi, xstar, dbv, W;
    std::vector<long long> rows, row_ptr, col_marker; // node -> marker CSR
    std::vector<double> col_s;
    std::vector<long long> proj_ptr, proj_node;      // projection point, d = 1
    std::vector<double> proj_w;
    std::vector<long long> tw_ptr, tw_node;          // two-sided d = 2 at X_l (error metrics)
    std::vector<double> tw_w;
    std::vector<long long> interior;                 // candidate nodes flagged interior (ascending)
};

int build_geometry(const GeomInput& in, Geometry& g, std::string& err);

}  // namespace lbmib
