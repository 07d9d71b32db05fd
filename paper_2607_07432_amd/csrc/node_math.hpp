// Per-node arithmetic of the hybrid LBM step, shared by every sweep kernel.
//
// Populations are handled as deviations from the lattice weights, f~_i = f_i - w_i
// (reference density 1), so that FP32 storage keeps its precision: every
// quantity below is computed from deviations without forming f_i itself.
//
// Equations (paper numbering): Eq. (6) LBE with pull streaming, Eq. (7) force
// populations, Eq. (9) half-force velocity, Eq. (A.3) equilibrium, Eq. (A.4)
// regularised off-equilibrium, Eq. (A.7) HRR Pi^(2), Eq. (A.8) recursive Pi^(3),
// Eq. (A.9) force moment a^F, Eqs. (A.11)-(A.13) LB face fluxes,
// Eqs. (A.14)-(A.16) MUSCL-Hancock face values, Eq. (11) energy flux.
#pragma once

#include "lattice.hpp"

namespace lbmib {

// Gas and model constants in the arithmetic type R of the kernel that reads them.
template <class R>
struct GasT {
    R mu, lambda_, gamma, sigma, Cv, Cp;
    int with_aC;
    R inv_Cv;           // 1 / Cv
};
using Gas = GasT<double>;

template <class C>
__host__ __device__ inline GasT<C> gas_as(const Gas& g) {
    return {C(g.mu), C(g.lambda_), C(g.gamma), C(g.sigma), C(g.Cv), C(g.Cp), g.with_aC, C(g.inv_Cv)};
}

template <class L, class C>
struct Node {
    C rho;          // density
    C inv_rho;      // 1 / rho
    C u[3];         // velocity with the half-force correction, Eq. (9)
    C T;            // temperature of the predicted (force-free) state
};

// Third-order 3r coefficients of the symmetric tensor t3(a,b,g) = x_a x_b x_g * s.
template <class L, class C>
__host__ __device__ __forceinline__ void a3r_of_uuu(const C* u, C s, C* out) {
#pragma unroll
    for (int k = 0; k < L::K3; ++k) {
        C v = 0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int sg = L::combo[k][t][0];
            if (sg != 0) {
                const int a = L::combo[k][t][1], b = L::combo[k][t][2], g = L::combo[k][t][3];
                v += C(sg) * u[a] * u[b] * u[g];
            }
        }
        out[k] = v * s;
    }
}

// Eq. (A.8) projected on the 3r basis: Pi3_abg = u_a Pi_bg + u_b Pi_ga + u_g Pi_ab.
template <class L, class C>
__device__ __forceinline__ void pi3r_of(const C* u, const C (*Pi)[3], C* out) {
#pragma unroll
    for (int k = 0; k < L::K3; ++k) {
        C v = 0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int sg = L::combo[k][t][0];
            if (sg != 0) {
                const int a = L::combo[k][t][1], b = L::combo[k][t][2], g = L::combo[k][t][3];
                v += C(sg) * (u[a] * Pi[b][g] + u[b] * Pi[g][a] + u[g] * Pi[a][b]);
            }
        }
        out[k] = v;
    }
}

// f^eq_i - w_i of Eq. (A.3) for all i.
template <class L, class C>
__host__ __device__ __forceinline__ void feq_dev(C rho, const C* u, C theta, C* feqd) {
    constexpr int D = L::D;
    C uu = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) uu += u[a] * u[a];
    C a3[L::K3];
    a3r_of_uuu<L, C>(u, rho, a3);
    const C drho = rho - C(1);
    const C rtm1 = rho * (theta - C(1));
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        C cu = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) cu += C(L::c[i][a]) * u[a];
        C h = 0;
#pragma unroll
        for (int k = 0; k < L::K3; ++k) h += C(h3r<L>(i, k) / h3r_norm<L>(k)) * a3[k];
        const C rest = C((L::w[i] - (i == 0 ? 1.0 : 0.0)) / L::w[i]);
        feqd[i] = C(L::w[i]) * (drho + rest * rtm1 + C(3) * rho * cu + C(4.5) * rho * (cu * cu - C(CS2) * uu) + h);
    }
}

// Neighbour data the collision at a node needs (central differences, Eq. (A.9)).
template <class C>
struct Stencil {
    C du[3][3];     // du[a][b] = d u_a / d x_b
    C div_rhou;     // div (rho u)
    C u_grad_p;     // u . grad(rho T)  (= u . grad p / cs^2)
    C dmu3[3];      // d/dx_a (rho u_a^3)
};

// Post-collision deviations f^col_i - w_i (Eq. (6)) and the new force history
// H2 = dev(a^F) (the deviatoric sum_i (c c - delta c^2/D) F_i, Eq. (A.7)).
// fd: population deviations at the node; H2: previous history (full symmetric
// tensor, H2[a][b]); fib: momentum forcing of the node.
//
// f^col = f^eq + (1 - 1/taubar) f^neq + F/2 is a Hermite series of order 3 in every
// term (Eqs. (A.3), (A.4), (7)), so the three are summed coefficient by coefficient and
// reconstructed once per population:
//   f^col_i - w_i = w_i [ (rho - 1) + r_i rho (theta - 1) + 3 c_i . J
//                         + 9/2 (c_i c_i : A - cs^2 tr A) + sum_k H3r_ik B_k / N_k ],
//   J = rho u + f/2,  A = rho u u + (1 - 1/taubar) Pi + a^F/2,
//   B = (rho u u u)^(3r) + (1 - 1/taubar) Pi^(3r).
// The population part of Pi (Eq. (A.7)) uses the exact lattice moment
// sum_i c c (f^eq_i - w_i) = rho u u + (rho theta - 1) cs^2 I, whose deviatoric part is dev(rho u u).
template <class L, class C, class R>
__device__ __forceinline__ void collide(const GasT<R>& g, const C* fd, const Node<L, C>& n, const Stencil<C>& s,
                                        const C* fib, const C (*H2)[3], C* fcol, C (*H2new)[3]) {
    constexpr int D = L::D;
    const C rho = n.rho;
    const C theta = n.T;
    const C* u = n.u;
    C div = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) div += s.du[a][a];

    // Eq. (A.9). d/dt[rho(1 - theta)] from the Euler balance laws:
    //   d rho/dt = -div(rho u),  d(rho theta)/dt = -u.grad(rho theta) - gamma rho theta div u.
    const C dgdt = -s.div_rhou + s.u_grad_p + C(g.gamma) * rho * theta * div;
    const C iso = C(2.0 / D) * rho * C(CS2) * div - C(CS2) * dgdt;
    C aF[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            C v = fib[a] * u[b] + fib[b] * u[a];
            if (a == b) {
                v += iso;
                if (g.with_aC) v -= s.dmu3[a];
            }
            aF[a][b] = v;
            aF[b][a] = v;
        }
    C tra = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) tra += aF[a][a];

    // Second moment of the populations.
    C M2[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M2[a][b] = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                if (L::c[i][a] * L::c[i][b] != 0) M2[a][b] += C(L::c[i][a] * L::c[i][b]) * fd[i];

    // Eq. (A.7): Pi = sigma [dev(M2) - dev(rho u u) + H2/2] - (1 - sigma) rho cs^2 taubar S.
    const C taubar = C(3) * C(g.mu) * n.inv_rho + C(0.5);   // tau = nu / cs^2, Eq. (6)
    const C om = C(1) - C(1) / taubar;
    C trP = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) trP += M2[a][a] - rho * u[a] * u[a];
    const C sig = C(g.sigma);
    const C fdc = (C(1) - sig) * rho * C(CS2) * taubar;
    C Pi[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Pi[a][b] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            C pop = M2[a][b] - rho * u[a] * u[b] + C(0.5) * H2[a][b];
            C S = s.du[a][b] + s.du[b][a];
            if (a == b) {
                pop -= trP * C(1.0 / D);
                S -= C(2.0 / D) * div;
            }
            Pi[a][b] = sig * pop - fdc * S;
            Pi[b][a] = Pi[a][b];
        }

    // Combined Hermite coefficients.
    C J[3], A[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a) J[a] = rho * u[a] + C(0.5) * fib[a];
    C trA = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            A[a][b] = rho * u[a] * u[b] + om * Pi[a][b] + C(0.5) * aF[a][b];
            if (a == b) trA += A[a][a];
        }
    C B3[L::K3], P3[L::K3];
    a3r_of_uuu<L, C>(u, rho, B3);
    pi3r_of<L, C>(u, Pi, P3);
#pragma unroll
    for (int k = 0; k < L::K3; ++k) B3[k] += om * P3[k];
    const C base = (rho - C(1));
    const C rtm1 = rho * (theta - C(1));
    const C iso2 = C(CS2) * trA;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        C cJ = 0, ccA = 0, h = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (L::c[i][a]) cJ += C(L::c[i][a]) * J[a];
#pragma unroll
            for (int b = a; b < D; ++b)
                if (L::c[i][a] * L::c[i][b] != 0) ccA += C((a == b ? 1 : 2) * L::c[i][a] * L::c[i][b]) * A[a][b];
        }
#pragma unroll
        for (int k = 0; k < L::K3; ++k)
            if (h3r<L>(i, k) != 0.0) h += C(h3r<L>(i, k) / h3r_norm<L>(k)) * B3[k];
        const C rest = C((L::w[i] - (i == 0 ? 1.0 : 0.0)) / L::w[i]);
        fcol[i] = C(L::w[i]) * (base + rest * rtm1 + C(3) * cJ + C(4.5) * (ccA - iso2) + h);
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) H2new[a][b] = aF[a][b] - (a == b ? tra * C(1.0 / D) : C(0));
}

// Velocities below U_ZERO count as zero in both sign decisions of the MUSCL operator
// (sign(u) in eta and the upwind test): the operator is discontinuous at u = 0 and a
// velocity that vanishes by symmetry is a rounding residue of either sign.
constexpr double U_ZERO = 1e-7;

template <class C>
__device__ __forceinline__ C sgn(C v) {
    return C((v > C(U_ZERO)) - (v < C(-U_ZERO)));
}

// Cell quantities of the energy flux.
template <class L, class C>
struct Cell {
    C rho, u[3], T;
};

// MUSCL-Hancock face value on the face between cells 1 and 2 of a 4-cell stencil
// (Eqs. (A.14)-(A.16)) is linear in Phi for given face-normal velocities:
//   F*(Phi) = sum_t w_t Phi_t. Left state (u~ >= 0): s = (1 - u_1)/4,
//   w = (-s (1 + eta_1), 1 + 2 s eta_1, s (1 - eta_1), 0); right state: s = (1 + u_2)/4,
//   w = (0, s (1 + eta_2), 1 - 2 s eta_2, -s (1 - eta_2)); eta = (2 u - sign(u))/3.
template <class C>
__device__ __forceinline__ void muscl_weights(C ua, C ub, C* w) {
    if (C(0.5) * (ua + ub) >= C(-U_ZERO)) {
        const C eta = (C(2) * ua - sgn(ua)) * C(1.0 / 3.0);
        const C s = (C(1) - ua) * C(0.25);
        w[0] = -s * (C(1) + eta);
        w[1] = C(1) + C(2) * s * eta;
        w[2] = s * (C(1) - eta);
        w[3] = 0;
    } else {
        const C eta = (C(2) * ub - sgn(ub)) * C(1.0 / 3.0);
        const C s = (C(1) + ub) * C(0.25);
        w[0] = 0;
        w[1] = s * (C(1) + eta);
        w[2] = C(1) - C(2) * s * eta;
        w[3] = -s * (C(1) - eta);
    }
}

// Energy flux through the face between cells 1 and 2 of the 4-cell stencil c4 along axis a
// (Eq. (11)), given the LB mass flux Fr and momentum fluxes Fm[b] (lattice-weight part
// cs^2 delta_ab removed) through that face:
//   F = F*(rho H u_a) + (h - k)_f [Fr - F*(rho u_a)] + sum_b u_b,f [Fm_b - F*(rho u_a u_b + p' delta_ab)]
//       - lambda (T_2 - T_1),
// with p' = p - cs^2, H = k + Cp T, h = Cp T, k = |u|^2/2, (.)_f the mean of cells 1 and 2.
// By linearity of F* this is F*(Psi) + (h - k)_f Fr + sum_b u_b,f Fm_b - lambda (T_2 - T_1),
// Psi = rho u_a (k + Cp T) - (h - k)_f rho u_a - sum_b u_b,f rho u_a u_b - u_a,f p'.
template <class L, class C, class R>
__device__ __forceinline__ C energy_flux(const GasT<R>& g, int a, const Cell<L, C>* c4, C Fr, const C* Fm) {
    constexpr int D = L::D;
    C k[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        C uu = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) uu += c4[t].u[b] * c4[t].u[b];
        k[t] = C(0.5) * uu;
    }
    const C Cp = C(g.Cp);
    const C hk = C(0.5) * ((Cp * c4[1].T - k[1]) + (Cp * c4[2].T - k[2]));
    C ubf[3];
#pragma unroll
    for (int b = 0; b < D; ++b) ubf[b] = C(0.5) * (c4[1].u[b] + c4[2].u[b]);
    C w[4];
    muscl_weights<C>(c4[1].u[a], c4[2].u[a], w);
    C fs = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const C ru = c4[t].rho * c4[t].u[a];
        C ub_u = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) ub_u += ubf[b] * c4[t].u[b];
        const C pd = (c4[t].rho * c4[t].T - C(1)) * C(CS2);
        const C psi = ru * (k[t] + Cp * c4[t].T - hk - ub_u) - ubf[a] * pd;
        fs += w[t] * psi;
    }
    C flux = fs + hk * Fr;
#pragma unroll
    for (int b = 0; b < D; ++b) flux += ubf[b] * Fm[b];
    flux -= C(g.lambda_) * (c4[2].T - c4[1].T);
    return flux;
}

// Outlet of the inflow/outflow closure: the last two columns take the new state of column
// nx - 3 rescaled by s = p_inf / p (populations and total energy alike), so the pressure there is
// the free-stream one while u and T keep zero gradient. p is proportional to the internal energy
// density rho E - |j|^2 / (2 rho), so s is the ratio of those. With deviation storage
// (f~ = f - w, e = rho E - e_ref) the rescaled values are s f~ + (s - 1) w and s e + (s - 1) e_ref.
// fnew, enew: the column's new f~ and e; eint_inf = rho_inf Cv T_inf.
template <class L, class C>
__device__ __forceinline__ C outlet_scale(const C* fnew, C enew, C e_ref, C eint_inf) {
    C drho = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        drho += fnew[i];
#pragma unroll
        for (int b = 0; b < L::D; ++b)
            if (L::c[i][b]) j[b] += C(L::c[i][b]) * fnew[i];
    }
    C jj = 0;
#pragma unroll
    for (int b = 0; b < L::D; ++b) jj += j[b] * j[b];
    return eint_inf / ((enew + e_ref) - C(0.5) * jj / (C(1) + drho));
}

}  // namespace lbmib
