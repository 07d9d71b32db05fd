// Per-geometry precompute of the immersed boundary, host FP64 (Secs. 2.3-2.4).
//
// For every marker l: the kernel support (strict |x_ia - X_la| < d per axis), restricted
// to the closed interior set Omega' for the one-sided methods; the weights delta_il of
// Eqs. (18)-(19); phi_l (Eq. (16)); the effective boundary X*_l (Eq. (25)); d_BV = |X_l - X*_l|;
// the improved weight W_l (Eq. (17)); the projection point P_l = X_l + 1.5 n_l with its
// two-sided d = 1 support; the two-sided d = 2 support used for boundary errors; and the
// node -> marker CSR of the spreading weights s_ik = phi_k delta_ik W_k (Eq. (15)).
//
// Omega' membership: node i is interior iff (x_i - X_l*) . n_l* <= 0 where l* is the
// marker nearest to x_i (ties: lowest index). Squared distances and dot products are
// summed left to right and this file is compiled without floating-point contraction,
// so the integer lists are reproducible bit for bit.
#include "precompute.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>

namespace lbmib {

namespace {

constexpr double PI = 3.14159265358979323846;

double cos_kernel(double r, double d) {
    if (std::fabs(r) > d) return 0.0;
    return (1.0 + std::cos(PI * r / d)) / (2.0 * d);
}

double roma3_kernel(double r) {
    const double a = std::fabs(r);
    if (a <= 0.5) return (1.0 + std::sqrt(std::max(1.0 - 3.0 * a * a, 0.0))) / 3.0;
    if (a <= 1.5) return (5.0 - 3.0 * a - std::sqrt(std::max(1.0 - 3.0 * (1.0 - a) * (1.0 - a), 0.0))) / 6.0;
    return 0.0;
}

// Nodes with |i_a - c_a| < radius on every axis, x fastest.
void box(int D, const double* c, double radius, std::vector<std::array<long long, 3>>& out) {
    long long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
        lo[a] = (long long)std::ceil(c[a] - radius);
        hi[a] = (long long)std::floor(c[a] + radius);
    }
    out.clear();
    for (long long z = lo[2]; z <= hi[2]; ++z) {
        if (D == 3 && !(std::fabs((double)z - c[2]) < radius)) continue;
        for (long long y = lo[1]; y <= hi[1]; ++y) {
            if (!(std::fabs((double)y - c[1]) < radius)) continue;
            for (long long x = lo[0]; x <= hi[0]; ++x) {
                if (!(std::fabs((double)x - c[0]) < radius)) continue;
                out.push_back({x, y, D == 3 ? z : 0});
            }
        }
    }
}

long long lin(const std::array<long long, 3>& p, const long long* dims) {
    return p[0] + dims[0] * (p[1] + dims[1] * p[2]);
}

double weight(int D, int kernel, double radius, const std::array<long long, 3>& p, const double* X) {
    double w = 1.0;
    for (int a = 0; a < D; ++a) {
        const double r = (double)p[a] - X[a];
        w = w * (kernel == 0 ? cos_kernel(r, radius) : roma3_kernel(r));
    }
    return w;
}

}  // namespace

int build_geometry(const GeomInput& in, Geometry& g, std::string& err) {
    const int D = in.dim, M = in.m;
    g = Geometry();
    g.dim = D;
    g.m = M;
    if (M == 0) return 0;
    const double radius = in.kernel == 0 ? 2.0 : 1.5;
    const bool one_sided = in.method != 0;
    const long long* dims = in.dims;

    std::vector<std::vector<std::array<long long, 3>>> boxes(M);
    for (int l = 0; l < M; ++l) box(D, &in.X[(size_t)l * D], radius, boxes[l]);

    // Interior flags of every node touched by a marker support.
    std::unordered_map<long long, char> interior;
    if (one_sided) {
        std::vector<long long> cand;
        for (int l = 0; l < M; ++l)
            for (auto& p : boxes[l]) cand.push_back(lin(p, dims));
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        interior.reserve(cand.size() * 2);
        for (long long v : cand) {
            double p[3];
            p[0] = (double)(v % dims[0]);
            p[1] = (double)((v / dims[0]) % dims[1]);
            p[2] = (double)(v / (dims[0] * dims[1]));
            int best = 0;
            double bestd = 0.0;
            for (int l = 0; l < M; ++l) {
                const double* X = &in.X[(size_t)l * D];
                double d0 = p[0] - X[0];
                double dd = d0 * d0;
                for (int a = 1; a < D; ++a) {
                    const double da = p[a] - X[a];
                    dd = dd + da * da;
                }
                if (l == 0 || dd < bestd) {
                    best = l;
                    bestd = dd;
                }
            }
            const double* X = &in.X[(size_t)best * D];
            const double* n = &in.n[(size_t)best * D];
            double dot = (p[0] - X[0]) * n[0];
            for (int a = 1; a < D; ++a) dot = dot + (p[a] - X[a]) * n[a];
            const char inside = dot <= 0.0 ? 1 : 0;
            interior[v] = inside;
            if (inside) g.interior.push_back(v);
        }
    }

    // Supports and weights.
    g.supp_ptr.assign(M + 1, 0);
    for (int l = 0; l < M; ++l) {
        for (auto& p : boxes[l]) {
            const long long v = lin(p, dims);
            if (one_sided && !interior[v]) continue;
            g.supp_node.push_back(v);
            g.supp_w.push_back(weight(D, in.kernel, radius, p, &in.X[(size_t)l * D]));
            g.supp_c.push_back(p);
        }
        g.supp_ptr[l + 1] = (long long)g.supp_node.size();
    }

    // phi (Eq. (16)), X* (Eq. (25)), d_BV.
    g.phi.assign(M, 0.0);
    g.xstar.assign((size_t)M * D, 0.0);
    g.dbv.assign(M, 0.0);
    g.n_active = 0;
    for (int l = 0; l < M; ++l) {
        double s = 0.0;
        for (long long e = g.supp_ptr[l]; e < g.supp_ptr[l + 1]; ++e) s += g.supp_w[e];
        for (int a = 0; a < D; ++a) g.xstar[(size_t)l * D + a] = in.X[(size_t)l * D + a];
        if (s > 0.0) {
            g.phi[l] = one_sided ? 1.0 / s : 1.0;
            g.n_active++;
            for (int a = 0; a < D; ++a) {
                double acc = 0.0;
                for (long long e = g.supp_ptr[l]; e < g.supp_ptr[l + 1]; ++e)
                    acc += (double)g.supp_c[e][a] * g.supp_w[e];
                g.xstar[(size_t)l * D + a] = g.phi[l] * acc;
            }
        }
        double d2 = 0.0;
        for (int a = 0; a < D; ++a) {
            const double d = in.X[(size_t)l * D + a] - g.xstar[(size_t)l * D + a];
            d2 += d * d;
        }
        g.dbv[l] = std::sqrt(d2);
    }

    // W (Eq. (17)) through the node density sum_k phi_k delta_ik.
    std::unordered_map<long long, double> density;
    for (int l = 0; l < M; ++l)
        for (long long e = g.supp_ptr[l]; e < g.supp_ptr[l + 1]; ++e) density[g.supp_node[e]] += g.phi[l] * g.supp_w[e];
    g.W.assign(M, 0.0);
    for (int l = 0; l < M; ++l) {
        if (g.phi[l] <= 0.0) continue;
        double tot = 0.0;
        for (long long e = g.supp_ptr[l]; e < g.supp_ptr[l + 1]; ++e)
            tot += g.phi[l] * g.supp_w[e] * density[g.supp_node[e]];
        g.W[l] = 1.0 / tot;
    }

    // Node -> marker CSR.
    std::map<long long, std::vector<std::pair<int, double>>> rows;
    for (int l = 0; l < M; ++l) {
        if (g.phi[l] <= 0.0) continue;
        for (long long e = g.supp_ptr[l]; e < g.supp_ptr[l + 1]; ++e)
            rows[g.supp_node[e]].push_back({l, g.phi[l] * g.supp_w[e] * g.W[l]});
    }
    g.row_ptr.push_back(0);
    for (auto& kv : rows) {
        auto& ent = kv.second;
        std::sort(ent.begin(), ent.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
            return a.first < b.first;
        });
        g.rows.push_back(kv.first);
        for (auto& pr : ent) {
            g.col_marker.push_back(pr.first);
            g.col_s.push_back(pr.second);
        }
        g.row_ptr.push_back((long long)g.col_marker.size());
    }

    // Projection points (two-sided, d = 1) and the two-sided d = 2 support at X_l.
    g.proj_ptr.assign(M + 1, 0);
    g.tw_ptr.assign(M + 1, 0);
    std::vector<std::array<long long, 3>> b;
    for (int l = 0; l < M; ++l) {
        double P[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) P[a] = in.X[(size_t)l * D + a] + 1.5 * in.n[(size_t)l * D + a];
        box(D, P, 1.0, b);
        for (auto& p : b) {
            g.proj_node.push_back(lin(p, dims));
            g.proj_w.push_back(weight(D, 0, 1.0, p, P));
        }
        g.proj_ptr[l + 1] = (long long)g.proj_node.size();
        box(D, &in.X[(size_t)l * D], 2.0, b);
        for (auto& p : b) {
            g.tw_node.push_back(lin(p, dims));
            g.tw_w.push_back(weight(D, 0, 2.0, p, &in.X[(size_t)l * D]));
        }
        g.tw_ptr[l + 1] = (long long)g.tw_node.size();
    }
    (void)err;
    return 0;
}

}  // namespace lbmib
