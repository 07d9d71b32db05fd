// Velocity sets and discrete Hermite polynomials as compile-time tables.
//
// D3Q19 uses the velocity order of the paper's Appendix A, Eq. (A.1), with the
// standard weights by speed class (1/3, 1/18, 1/36); the weights printed in
// Eq. (A.2) contain three entries inconsistent with the velocity list.
// D2Q9 (0:(0,0), 1-4 axis, 5-8 diagonals) is the two-dimensional analogue.
// The third-order "3r" basis is that of Eq. (A.6) (D3Q19) and {H_xxy, H_xyy}
// (D2Q9); the equilibrium and off-equilibrium third-order terms are orthogonal
// projections on it, normalised by N_k = sum_i w_i H3r_ik^2.
#pragma once

#include <hip/hip_runtime.h>

namespace lbmib {

constexpr double CS2 = 1.0 / 3.0;

struct D2Q9 {
    static constexpr int D = 2, Q = 9, K3 = 2, NOFF = 1;
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    // 3r combinations: list of (sign, a, b, g) pairs; 2D uses single components.
    static constexpr int combo[2][2][4] = {{{1, 0, 0, 1}, {0, 0, 0, 0}},   // H_xxy
                                           {{1, 0, 1, 1}, {0, 0, 0, 0}}};  // H_xyy
};

struct D3Q19 {
    static constexpr int D = 3, Q = 19, K3 = 6, NOFF = 3;
    static constexpr int c[19][3] = {{0, 0, 0},   {1, 0, 0},   {1, 0, 1},  {0, 0, 1},   {-1, 0, 1},
                                     {0, 1, 0},   {0, 1, 1},   {0, -1, 1}, {1, 1, 0},   {-1, 1, 0},
                                     {-1, 0, 0},  {-1, 0, -1}, {0, 0, -1}, {1, 0, -1},  {0, -1, 0},
                                     {0, -1, -1}, {0, 1, -1},  {-1, -1, 0}, {1, -1, 0}};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 36, 1.0 / 18, 1.0 / 36,
                                     1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 18, 1.0 / 36, 1.0 / 18, 1.0 / 36, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    // Eq. (A.6): xxy+yzz, xzz+xyy, yyz+xxz, xxy-yzz, xzz-xyy, yyz-xxz
    static constexpr int combo[6][2][4] = {{{1, 0, 0, 1}, {1, 1, 2, 2}},  {{1, 0, 2, 2}, {1, 0, 1, 1}},
                                           {{1, 1, 1, 2}, {1, 0, 0, 2}},  {{1, 0, 0, 1}, {-1, 1, 2, 2}},
                                           {{1, 0, 2, 2}, {-1, 0, 1, 1}}, {{1, 1, 1, 2}, {-1, 0, 0, 2}}};
};

// H^(3)_{i,abg} of Eq. (A.5).
template <class L>
__host__ __device__ constexpr double h3(int i, int a, int b, int g) {
    const double ca = L::c[i][a], cb = L::c[i][b], cg = L::c[i][g];
    return ca * cb * cg - CS2 * ((a == b ? cg : 0.0) + (b == g ? ca : 0.0) + (a == g ? cb : 0.0));
}

template <class L>
__host__ __device__ constexpr double h3r(int i, int k) {
    double s = 0.0;
    for (int t = 0; t < 2; ++t) {
        const int sg = L::combo[k][t][0];
        if (sg != 0) s += sg * h3<L>(i, L::combo[k][t][1], L::combo[k][t][2], L::combo[k][t][3]);
    }
    return s;
}

template <class L>
__host__ __device__ constexpr double h3r_norm(int k) {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += L::w[i] * h3r<L>(i, k) * h3r<L>(i, k);
    return s;
}

// Index of the opposite velocity.
template <class L>
__host__ __device__ constexpr int opp(int i) {
    for (int j = 0; j < L::Q; ++j)
        if (L::c[j][0] == -L::c[i][0] && L::c[j][1] == -L::c[i][1] && L::c[j][2] == -L::c[i][2]) return j;
    return -1;
}

// Symmetric D x D tensor stored as xx, yy, [zz], xy, [xz, yz].
template <int D>
struct SymIdx;
template <>
struct SymIdx<2> {
    static constexpr int N = 3;
    __host__ __device__ static constexpr int at(int a, int b) { return a == b ? a : 2; }
};
template <>
struct SymIdx<3> {
    static constexpr int N = 6;
    __host__ __device__ static constexpr int at(int a, int b) {
        return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
    }
};

}  // namespace lbmib
