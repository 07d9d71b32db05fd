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

struct Gas {
    double mu, lambda_, gamma, sigma, Cv, Cp;
    int with_aC;
};

template <class L, class C>
struct Node {
    C rho;          // density
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

// Eq. (A.4): w_i [H2_i : Pi / (2 cs^4) + sum_k H3r_ik Pi3r_k / N_k].
template <class L, class C>
__device__ __forceinline__ void fneq_of(const C (*Pi)[3], const C* u, C* fneq) {
    constexpr int D = L::D;
    C p3[L::K3];
    pi3r_of<L, C>(u, Pi, p3);
    C tr = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) tr += Pi[a][a];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        C s = 0;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (L::c[i][a] * L::c[i][b] != 0) s += C(L::c[i][a] * L::c[i][b]) * Pi[a][b];
        C h = 0;
#pragma unroll
        for (int k = 0; k < L::K3; ++k) h += C(h3r<L>(i, k) / h3r_norm<L>(k)) * p3[k];
        fneq[i] = C(L::w[i]) * (C(4.5) * (s - C(CS2) * tr) + h);
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
template <class L, class C>
__device__ __forceinline__ void collide(const Gas& g, const C* fd, const Node<L, C>& n, const Stencil<C>& s,
                                        const C* fib, const C (*H2)[3], C* fcol, C (*H2new)[3]) {
    constexpr int D = L::D;
    const C rho = n.rho;
    const C theta = n.T;
    C div = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) div += s.du[a][a];

    // Eq. (A.9). d/dt[rho(1 - theta)] from the Euler balance laws:
    //   d rho/dt = -div(rho u),  d(rho theta)/dt = -u.grad(rho theta) - gamma rho theta div u.
    const C dgdt = -s.div_rhou + s.u_grad_p + C(g.gamma) * rho * theta * div;
    C aF[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            C v = fib[a] * n.u[b] + fib[b] * n.u[a];
            if (a == b) {
                v += C(2.0 / D) * rho * C(CS2) * div - C(CS2) * dgdt;
                if (g.with_aC) v -= s.dmu3[a];
            }
            aF[a][b] = v;
        }

    C feqd[L::Q];
    feq_dev<L, C>(rho, n.u, theta, feqd);

    // Eq. (A.7): Pi = sigma [sum_i dev(cc) (f_i - f^eq_i) + H2/2] - (1 - sigma) rho cs^2 taubar S.
    const C taubar = C(g.mu) / (rho * C(CS2)) + C(0.5);   // tau = nu / cs^2, Eq. (6)
    C m2[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m2[a][b] = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const C gi = fd[i] - feqd[i];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                if (L::c[i][a] * L::c[i][b] != 0) m2[a][b] += C(L::c[i][a] * L::c[i][b]) * gi;
    }
    C trm = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) trm += m2[a][a];
    const C sig = C(g.sigma);
    const C fdc = (C(1) - sig) * rho * C(CS2) * taubar;
    C Pi[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            C pop = m2[a][b] + C(0.5) * H2[a][b];
            C S = s.du[a][b] + s.du[b][a];
            if (a == b) {
                pop -= trm / C(D);
                S -= C(2.0 / D) * div;
            }
            Pi[a][b] = sig * pop - fdc * S;
            Pi[b][a] = Pi[a][b];
        }
    C fneq[L::Q];
    fneq_of<L, C>(Pi, n.u, fneq);

    // Eq. (7): F_i = w_i [c_i . f / cs^2 + H2_i : a^F / (2 cs^4)].
    C tra = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) tra += aF[a][a];
    const C om = C(1) - C(1) / taubar;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        C cf = 0, cac = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cf += C(L::c[i][a]) * fib[a];
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (L::c[i][a] * L::c[i][b] != 0) cac += C(L::c[i][a] * L::c[i][b]) * aF[a][b];
        }
        const C Fi = C(L::w[i]) * (C(3) * cf + C(4.5) * (cac - C(CS2) * tra));
        fcol[i] = feqd[i] + om * fneq[i] + C(0.5) * Fi;
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) H2new[a][b] = aF[a][b] - (a == b ? tra / C(D) : C(0));
}

// MUSCL-Hancock face value on the face between cells a and b = a + e (Eqs. (A.14)-(A.16)),
// from Phi at cells a-1, a, b, b+1 and the face-normal velocity at a and b.
// Velocities below U_ZERO count as zero in both sign decisions (sign(u) in eta and the
// upwind test): the operator is discontinuous at u = 0 and a velocity that vanishes by
// symmetry is a rounding residue of either sign.
constexpr double U_ZERO = 1e-7;

template <class C>
__device__ __forceinline__ C sgn(C v) {
    return C((v > C(U_ZERO)) - (v < C(-U_ZERO)));
}

template <class C>
__device__ __forceinline__ C muscl(C pm, C pa, C pb, C pp, C ua, C ub) {
    const C ut = C(0.5) * (ua + ub);
    if (ut >= C(-U_ZERO)) {
        const C eta = (C(2) * ua - sgn(ua)) / C(3);
        const C slope = C(0.5) * ((C(1) + eta) * (pa - pm) + (C(1) - eta) * (pb - pa));
        return pa + C(0.5) * slope * (C(1) - ua);
    }
    const C eta = (C(2) * ub - sgn(ub)) / C(3);
    const C slope = C(0.5) * ((C(1) + eta) * (pb - pa) + (C(1) - eta) * (pp - pb));
    return pb - C(0.5) * slope * (C(1) + ub);
}

// Cell quantities of the energy flux. p' = p - cs^2 keeps the pressure as a deviation
// (the lattice-weight part of the LB momentum flux is cs^2 delta_ab exactly).
template <class L, class C>
struct Cell {
    C rho, u[3], T;
};

// Energy flux through the face between cells A (index 1 of the 4-cell stencil) and B
// (index 2) along axis a (Eq. (11)), given the LB mass flux Fr and deviation momentum
// fluxes Fm[b] (lattice-weight part removed) through that face.
template <class L, class C>
__device__ __forceinline__ C energy_flux(const Gas& g, int a, const Cell<L, C>* c4, C Fr, const C* Fm) {
    constexpr int D = L::D;
    C phiH[4], phiM[4], k[4], pd[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        C uu = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) uu += c4[t].u[b] * c4[t].u[b];
        k[t] = C(0.5) * uu;
        pd[t] = (c4[t].rho * c4[t].T - C(1)) * C(CS2);        // p - cs^2
        phiH[t] = c4[t].rho * (k[t] + C(g.Cp) * c4[t].T) * c4[t].u[a];
        phiM[t] = c4[t].rho * c4[t].u[a];
    }
    const C ua = c4[1].u[a], ub = c4[2].u[a];
    C flux = muscl(phiH[0], phiH[1], phiH[2], phiH[3], ua, ub);
    const C hk = C(0.5) * ((C(g.Cp) * c4[1].T - k[1]) + (C(g.Cp) * c4[2].T - k[2]));
    flux += hk * (Fr - muscl(phiM[0], phiM[1], phiM[2], phiM[3], ua, ub));
#pragma unroll
    for (int b = 0; b < D; ++b) {
        C ph[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) ph[t] = c4[t].rho * c4[t].u[a] * c4[t].u[b] + (a == b ? pd[t] : C(0));
        const C ubf = C(0.5) * (c4[1].u[b] + c4[2].u[b]);
        flux += ubf * (Fm[b] - muscl(ph[0], ph[1], ph[2], ph[3], ua, ub));
    }
    flux -= C(g.lambda_) * (c4[2].T - c4[1].T);
    return flux;
}

}  // namespace lbmib
