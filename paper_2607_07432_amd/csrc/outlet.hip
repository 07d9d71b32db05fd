// Characteristic outlet (the far-field closure the paper applies with Poinsot and Lele's
// characteristic conditions, Sec. 2.4): after the sweep has written every column but x = nx-2,
// nx-1, those two columns advance by the locally one-dimensional inviscid characteristic (LODI)
// relations. The outgoing amplitudes come from first-order backward differences of the old state,
// the incoming one is relaxed to the free-stream pressure:
//   L5 = (u + c)(dp + rho c du), L2 = u (c^2 drho - dp), L3,4 = u dv, u dw, L1 = K (p - p_inf),
//   K = sigma_c (1 - Ma^2) c / nx;
//   rho' = rho - (L2 + (L5 + L1)/2)/c^2, p' = p - (L5 + L1)/2, u' = u - (L5 - L1)/(2 rho c),
//   v' = v - L3, w' = w - L4;
// p = rho R T, c^2 = gamma p / rho; an amplitude travelling into the domain (u or u + c < 0) is
// zero. The new populations are the equilibrium of Eq. (A.3) at (rho', u', T') plus the
// non-equilibrium part of column nx-3 of the new state; rho E follows from the new fields and the
// diagonal force history is that of column nx-3.
#include "kernels.hpp"

namespace lbmib {

namespace {

constexpr int TPB_OUT = 256;

template <class L, class S>
__global__ void __launch_bounds__(TPB_OUT) k_outlet_char(SweepArgs a, StateP<S> Old, StateP<S> New, double sigma_c) {
    using C = S;
    constexpr int D = L::D, Q = L::Q;
    const long long lines = (long long)a.grid.ny * (D == 3 ? a.grid.nz : 1);
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= lines) return;
    const int nx = a.grid.nx;
    const long long N = a.grid.N;
    const long long base = (long long)nx * line;           // node (0, y[, z])
    const GasT<C> g = gas_as<C>(a.gas);
    const C R = C(CS2);
    const C e_ref = C(a.fs.e_ref);
    // force-free macros (rho, u, T) of node n of a state
    auto macros = [&](const StateP<S>& st, long long n, C& rho, C* u, C& T) {
        C drho = 0, j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const C fv = C(st.f[i * N + n]);
            drho += fv;
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (L::c[i][b]) j[b] += C(L::c[i][b]) * fv;
        }
        rho = C(1) + drho;
        const C ir = C(1) / rho;
        C uu = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            u[b] = b < D ? j[b] * ir : C(0);
            uu += u[b] * u[b];
        }
        T = ((C(st.e[n]) + e_ref) * ir - C(0.5) * uu) * g.inv_Cv;
    };
    // non-equilibrium part and diagonal history of column nx-3, new state
    C fneq[Q];
    {
        C r3, u3[3], T3, feq3[Q];
        macros(New, base + nx - 3, r3, u3, T3);
        feq_dev<L, C>(r3, u3, T3, feq3);
#pragma unroll
        for (int i = 0; i < Q; ++i) fneq[i] = C(New.f[i * N + base + nx - 3]) - feq3[i];
    }
    const S h0 = New.h2[base + nx - 3];
    const S h1 = D == 3 ? New.h2[N + base + nx - 3] : S(0);
    // old macros of columns nx-3, nx-2, nx-1
    C ro[3], uo[3][3], To[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) macros(Old, base + nx - 3 + k, ro[k], uo[k], To[k]);
    const C p_inf = C(a.fs.rho_inf) * R * C(a.fs.T_inf);
#pragma unroll
    for (int k = 1; k <= 2; ++k) {
        const C r = ro[k], pp = r * R * To[k];
        const C pm = ro[k - 1] * R * To[k - 1];
        const C c = sqrt(g.gamma * pp / r);
        const C dr = r - ro[k - 1], dp = pp - pm;
        const C ux = uo[k][0];
        const C du = ux - uo[k - 1][0];
        const C L5 = ux + c > C(0) ? (ux + c) * (dp + r * c * du) : C(0);
        const C L2 = ux > C(0) ? ux * (c * c * dr - dp) : C(0);
        const C ma = ux / c;
        const C K = C(sigma_c) * (C(1) - ma * ma) * c / C(nx);
        const C L1 = K * (pp - p_inf);
        const C rn = r - (L2 + C(0.5) * (L5 + L1)) / (c * c);
        const C pn = pp - C(0.5) * (L5 + L1);
        C un[3] = {0, 0, 0};
        un[0] = ux - (L5 - L1) / (C(2) * r * c);
#pragma unroll
        for (int b = 1; b < D; ++b) {
            const C Lt = ux > C(0) ? ux * (uo[k][b] - uo[k - 1][b]) : C(0);
            un[b] = uo[k][b] - Lt;
        }
        const C Tn = pn / (rn * R);
        C feq[Q];
        feq_dev<L, C>(rn, un, Tn, feq);
        const long long n = base + nx - 3 + k;
#pragma unroll
        for (int i = 0; i < Q; ++i) New.f[i * N + n] = S(feq[i] + fneq[i]);
        C uu = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) uu += un[b] * un[b];
        New.e[n] = S(rn * (C(0.5) * uu + g.Cv * Tn) - e_ref);
        New.h2[n] = h0;
        if (D == 3) New.h2[N + n] = h1;
    }
}

}  // namespace

template <class L, class S>
hipError_t launch_outlet_char(const SweepArgs& a, StateP<S> Old, StateP<S> New, double sigma_c, hipStream_t st) {
    const long long lines = (long long)a.grid.ny * (L::D == 3 ? a.grid.nz : 1);
    const unsigned blocks = (unsigned)((lines + TPB_OUT - 1) / TPB_OUT);
    hipLaunchKernelGGL((k_outlet_char<L, S>), dim3(blocks), dim3(TPB_OUT), 0, st, a, Old, New, sigma_c);
    return hipGetLastError();
}

template hipError_t launch_outlet_char<D2Q9, float>(const SweepArgs&, StateP<float>, StateP<float>, double, hipStream_t);
template hipError_t launch_outlet_char<D2Q9, double>(const SweepArgs&, StateP<double>, StateP<double>, double, hipStream_t);
template hipError_t launch_outlet_char<D3Q19, float>(const SweepArgs&, StateP<float>, StateP<float>, double, hipStream_t);
template hipError_t launch_outlet_char<D3Q19, double>(const SweepArgs&, StateP<double>, StateP<double>, double, hipStream_t);

}  // namespace lbmib
