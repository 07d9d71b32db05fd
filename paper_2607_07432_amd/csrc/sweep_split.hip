// Node-parallel kernels of the time step (three passes) and the state utilities.
//
// Pass 1 (k_macros): predicted macros of every node: rho, the half-force velocity of
//   Eq. (9) and the temperature from rho E (Sec. 2.5 step 1 variables).
// Pass 2 (k_collide): HRR collision with forcing (Eqs. (6), (7), (A.3)-(A.9)), keeping
//   the post-collision populations and the new force history.
// Pass 3 (k_stream_energy): pull streaming (Eq. (6)), LB face fluxes (Eqs. (A.11)-(A.13)),
//   MUSCL-Hancock energy flux (Eq. (11), Eqs. (A.14)-(A.16)) and the rho E update
//   (Eq. (10) with the operators of Eq. (A.10)), plus the inflow/outflow closure.
#include "kernels.hpp"

namespace lbmib {

namespace {

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ long long nid(const GridP& g, int x, int y, int z) {
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

__device__ __forceinline__ void decode(const GridP& g, long long n, int& x, int& y, int& z) {
    x = (int)(n % g.nx);
    const long long r = n / g.nx;
    y = (int)(r % g.ny);
    z = (int)(r / g.ny);
}

__device__ __forceinline__ long long shifted(const GridP& g, int x, int y, int z, int dx, int dy, int dz) {
    return nid(g, wrapi(x + dx, g.nx), wrapi(y + dy, g.ny), wrapi(z + dz, g.nz));
}

template <class L, class C>
__device__ __forceinline__ Cell<L, C> cell_at(const C* M, long long N, long long n) {
    Cell<L, C> c;
    c.rho = C(1) + M[n];
#pragma unroll
    for (int a = 0; a < L::D; ++a) c.u[a] = M[(1 + a) * N + n];
    c.u[2] = L::D == 3 ? c.u[2] : C(0);
    c.T = M[(1 + L::D) * N + n];
    return c;
}

constexpr int TPB = 256;

inline unsigned blocks_for(long long n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

// ---------------------------------------------------------------------------------- pass 1

template <class L, class S, class C>
__global__ void __launch_bounds__(TPB) k_macros(SweepArgs a, StateP<S> A, C* M) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    constexpr int D = L::D;
    C drho = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const C f = C(A.f[i * N + n]);
        drho += f;
#pragma unroll
        for (int b = 0; b < D; ++b)
            if (L::c[i][b]) j[b] += C(L::c[i][b]) * f;
    }
    const C rho = C(1) + drho;
    const C e = C(A.e[n]) + C(a.fs.e_ref);
    C uu = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) uu += (j[b] / rho) * (j[b] / rho);
    const C T = (e / rho - C(0.5) * uu) / C(a.gas.Cv);
    const int r = a.rows.rowmap[n];
    M[n] = drho;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const C fib = r >= 0 ? C(a.rows.fib[(long long)b * a.rows.nrows + r]) : C(0);
        M[(1 + b) * N + n] = (j[b] + C(0.5) * fib) / rho;
    }
    M[(1 + D) * N + n] = T;
}

// ---------------------------------------------------------------------------------- pass 2

template <class L, class S, class C>
__global__ void __launch_bounds__(TPB) k_collide(SweepArgs a, StateP<S> A, StateP<S> B, const C* M, C* fcol) {
    const GridP& g = a.grid;
    const long long N = g.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    constexpr int D = L::D;
    int x, y, z;
    decode(g, n, x, y, z);

    C fd[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) fd[i] = C(A.f[i * N + n]);

    const Cell<L, C> c0 = cell_at<L, C>(M, N, n);
    Node<L, C> nd;
    nd.rho = c0.rho;
    nd.inv_rho = C(1) / c0.rho;
    nd.T = c0.T;
#pragma unroll
    for (int b = 0; b < 3; ++b) nd.u[b] = c0.u[b];

    Stencil<C> s;
    s.div_rhou = 0;
    s.u_grad_p = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        s.dmu3[b] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) s.du[q][b] = 0;
    }
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const int ex = b == 0, ey = b == 1, ez = b == 2;
        const Cell<L, C> cp = cell_at<L, C>(M, N, shifted(g, x, y, z, ex, ey, ez));
        const Cell<L, C> cm = cell_at<L, C>(M, N, shifted(g, x, y, z, -ex, -ey, -ez));
#pragma unroll
        for (int q = 0; q < D; ++q) s.du[q][b] = C(0.5) * (cp.u[q] - cm.u[q]);
        s.div_rhou += C(0.5) * (cp.rho * cp.u[b] - cm.rho * cm.u[b]);
        s.u_grad_p += nd.u[b] * C(0.5) * (cp.rho * cp.T - cm.rho * cm.T);
        s.dmu3[b] = C(0.5) * (cp.rho * cp.u[b] * cp.u[b] * cp.u[b] - cm.rho * cm.u[b] * cm.u[b] * cm.u[b]);
    }

    C H2[3][3];
    const int r = a.rows.rowmap[n];
    const int nr = a.rows.nrows;
    H2[0][0] = C(A.h2[n]);
    if (D == 3) {
        H2[1][1] = C(A.h2[N + n]);
        H2[2][2] = -(H2[0][0] + H2[1][1]);
    } else {
        H2[1][1] = -H2[0][0];
    }
    C fib[3] = {0, 0, 0};
    C off[3] = {0, 0, 0};
    if (r >= 0) {
#pragma unroll
        for (int b = 0; b < D; ++b) fib[b] = C(a.rows.fib[(long long)b * nr + r]);
#pragma unroll
        for (int k = 0; k < L::NOFF; ++k) off[k] = C(a.rows.h2off[(long long)k * nr + r]);
    }
    H2[0][1] = H2[1][0] = off[0];
    if (D == 3) {
        H2[0][2] = H2[2][0] = off[1];
        H2[1][2] = H2[2][1] = off[2];
    }

    C fc[L::Q];
    C H2n[3][3];
    collide<L, C>(a.gas, fd, nd, s, fib, H2, fc, H2n);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) fcol[i * N + n] = fc[i];
    if (r >= 0) {
        a.rows.h2off_out[r] = H2n[0][1];
        if (D == 3) {
            a.rows.h2off_out[(long long)nr + r] = H2n[0][2];
            a.rows.h2off_out[2LL * nr + r] = H2n[1][2];
        }
    }
    // New diagonal history into B, with the closure of the x boundaries.
    int copies = 1;
    if (g.bc_x >= 1) {
        if (x < 2) {
            B.h2[n] = S(0);
            if (D == 3) B.h2[N + n] = S(0);
            return;
        }
        if (x >= g.nx - 2) return;
        if (x == g.nx - 3 && g.bc_x == 1) copies = 3;
    }
    for (int k = 0; k < copies; ++k) {
        B.h2[n + k] = S(H2n[0][0]);
        if (D == 3) B.h2[N + n + k] = S(H2n[1][1]);
    }
}

// ---------------------------------------------------------------------------------- pass 3

template <class L, class C>
__device__ __forceinline__ void lb_face_flux(const GridP& g, const C* fcol, int x, int y, int z, int ax, C& Fr,
                                             C* Fm) {
    const long long N = g.N;
    Fr = 0;
    Fm[0] = Fm[1] = Fm[2] = 0;
    const int e[3] = {ax == 0, ax == 1, ax == 2};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int ci = L::c[i][ax];
        if (ci == 0) continue;
        C v;
        if (ci == 1) {
            v = C(0.5) * (fcol[i * N + nid(g, x, y, z)] +
                          fcol[i * N + shifted(g, x, y, z, e[0] - L::c[i][0], e[1] - L::c[i][1], e[2] - L::c[i][2])]);
        } else {
            v = -C(0.5) * (fcol[i * N + shifted(g, x, y, z, e[0], e[1], e[2])] +
                           fcol[i * N + shifted(g, x, y, z, -L::c[i][0], -L::c[i][1], -L::c[i][2])]);
        }
        Fr += v;
#pragma unroll
        for (int b = 0; b < L::D; ++b)
            if (L::c[i][b]) Fm[b] += C(L::c[i][b]) * v;
    }
}

template <class L, class S, class C>
__global__ void __launch_bounds__(TPB)
    k_stream_energy(SweepArgs a, StateP<S> A, StateP<S> B, const C* M, const C* fcol) {
    const GridP& g = a.grid;
    const long long N = g.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    constexpr int D = L::D;
    int x, y, z;
    decode(g, n, x, y, z);
    if (g.bc_x >= 1) {
        if (x < 2) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i) B.f[i * N + n] = S(a.fs.fdev[i]);
            B.e[n] = S(0);
            return;
        }
        if (x >= g.nx - 2) return;
    }
    C fnew[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        fnew[i] = fcol[i * N + shifted(g, x, y, z, -L::c[i][0], -L::c[i][1], -L::c[i][2])];

    C ediv = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const int ex = ax == 0, ey = ax == 1, ez = ax == 2;
        Cell<L, C> c5[5];
#pragma unroll
        for (int t = 0; t < 5; ++t)
            c5[t] = cell_at<L, C>(M, N, shifted(g, x, y, z, (t - 2) * ex, (t - 2) * ey, (t - 2) * ez));
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int bx = x - side * ex, by = y - side * ey, bz = z - side * ez;
            C Fr, Fm[3];
            lb_face_flux<L, C>(g, fcol, wrapi(bx, g.nx), wrapi(by, g.ny), wrapi(bz, g.nz), ax, Fr, Fm);
            const C FE = energy_flux<L, C>(a.gas, ax, &c5[1 - side], Fr, Fm);
            ediv += side == 0 ? FE : -FE;
        }
    }
    const int r = a.rows.rowmap[n];
    const C fE = r >= 0 ? C(a.rows.fE[r]) : C(0);
    const C enew = C(A.e[n]) - ediv + fE;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) B.f[i * N + n] = S(fnew[i]);
    B.e[n] = S(enew);
    if (g.bc_x == 1 && x == g.nx - 3) {                    // outlet columns nx - 2, nx - 1
        const C eref = C(a.fs.e_ref);
        const C sc = outlet_scale<L, C>(fnew, enew, eref, C(a.fs.eint_inf));
        for (int k = 1; k < 3; ++k) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i) B.f[i * N + n + k] = S(sc * fnew[i] + (sc - C(1)) * C(L::w[i]));
            B.e[n + k] = S(sc * enew + (sc - C(1)) * eref);
        }
    }
}

template <class L, class S, class C>
hipError_t launch_split_step(const SweepArgs& a, StateP<S> A, StateP<S> B, C* M, C* fcol, hipStream_t st) {
    const unsigned nb = blocks_for(a.grid.N);
    hipLaunchKernelGGL((k_macros<L, S, C>), dim3(nb), dim3(TPB), 0, st, a, A, M);
    hipLaunchKernelGGL((k_collide<L, S, C>), dim3(nb), dim3(TPB), 0, st, a, A, B, (const C*)M, fcol);
    hipLaunchKernelGGL((k_stream_energy<L, S, C>), dim3(nb), dim3(TPB), 0, st, a, A, B, (const C*)M,
                       (const C*)fcol);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------- utilities

template <class L, class S>
__global__ void k_init_state(SweepArgs a, StateP<S> A) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) A.f[i * N + n] = S(a.fs.fdev[i]);
    A.e[n] = S(0);
    for (int k = 0; k < L::D - 1; ++k) A.h2[k * N + n] = S(0);
}

template <class L, class S>
__global__ void k_set_fields(SweepArgs a, StateP<S> A, const double* rho, const double* u, const double* T) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    double uu[3] = {0, 0, 0};
    double u2 = 0;
    for (int b = 0; b < L::D; ++b) {
        uu[b] = u[b * N + n];
        u2 += uu[b] * uu[b];
    }
    double fd[L::Q];
    feq_dev<L, double>(rho[n], uu, T[n], fd);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) A.f[i * N + n] = S(fd[i]);
    A.e[n] = S(rho[n] * (0.5 * u2 + a.gas.Cv * T[n]) - a.fs.e_ref);
    for (int k = 0; k < L::D - 1; ++k) A.h2[k * N + n] = S(0);
}

template <class L, class S, class O>
__global__ void k_fields(SweepArgs a, StateP<S> A, O* rho, O* u, O* T, O* p) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    double drho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < L::Q; ++i) {
        const double f = double(A.f[i * N + n]);
        drho += f;
        for (int b = 0; b < L::D; ++b) j[b] += L::c[i][b] * f;
    }
    const double r = 1.0 + drho;
    double u2 = 0;
    for (int b = 0; b < L::D; ++b) u2 += (j[b] / r) * (j[b] / r);
    const double t = ((double(A.e[n]) + a.fs.e_ref) / r - 0.5 * u2) / a.gas.Cv;
    if (rho) rho[n] = O(r);
    if (u)
        for (int b = 0; b < L::D; ++b) u[b * N + n] = O(j[b] / r);
    if (T) T[n] = O(t);
    if (p) p[n] = O(r * t * CS2);
}

// Canonical FP64 state, one component at a time: c < Q populations f_c; c == Q rho E;
// c = Q + 1 + a*D + b the force history H2_ab.
template <class L, class S>
__global__ void k_export(SweepArgs a, StateP<S> A, int c, double* out) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    constexpr int D = L::D;
    if (c < L::Q) {
        out[n] = double(A.f[(long long)c * N + n]) + L::w[c];
        return;
    }
    if (c == L::Q) {
        out[n] = double(A.e[n]) + a.fs.e_ref;
        return;
    }
    const int t = c - L::Q - 1, p = t / D, q = t % D;
    double v = 0.0;
    if (p == q) {
        if (p < D - 1) {
            v = double(A.h2[(long long)p * N + n]);
        } else {
            for (int k = 0; k < D - 1; ++k) v -= double(A.h2[(long long)k * N + n]);
        }
    } else {
        const int r = a.rows.rowmap[n];
        if (r >= 0) {
            const int lo = p < q ? p : q, hi = p < q ? q : p;
            const int k = (lo == 0 && hi == 1) ? 0 : (lo == 0 ? 1 : 2);
            v = a.rows.h2off[(long long)k * a.rows.nrows + r];
        }
    }
    out[n] = v;
}

template <class L, class S>
__global__ void k_import(SweepArgs a, StateP<S> A, int c, const double* in, int* bad) {
    const long long N = a.grid.N;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    constexpr int D = L::D;
    if (c < L::Q) {
        A.f[(long long)c * N + n] = S(in[n] - L::w[c]);
        return;
    }
    if (c == L::Q) {
        A.e[n] = S(in[n] - a.fs.e_ref);
        return;
    }
    const int t = c - L::Q - 1, p = t / D, q = t % D;
    if (p == q) {
        if (p < D - 1) A.h2[(long long)p * N + n] = S(in[n]);
        return;
    }
    if (p > q) return;
    const int r = a.rows.rowmap[n];
    const int k = (p == 0 && q == 1) ? 0 : (p == 0 ? 1 : 2);
    if (r >= 0)
        a.rows.h2off_out[(long long)k * a.rows.nrows + r] = in[n];
    else if (in[n] != 0.0)
        atomicOr(bad, 1);
}

// FP64 residual of the velocity change between two states, plus a non-finite check.
template <class L, class S>
__global__ void __launch_bounds__(TPB) k_residual(SweepArgs a, StateP<S> Old, StateP<S> New, double* partials) {
    const long long N = a.grid.N;
    __shared__ double red[TPB];
    __shared__ int nf[TPB];
    double acc = 0;
    int bad = 0;
    for (long long n = (long long)blockIdx.x * TPB + threadIdx.x; n < N; n += (long long)gridDim.x * TPB) {
        double r0 = 1, r1 = 1, j0[3] = {0, 0, 0}, j1[3] = {0, 0, 0};
        for (int i = 0; i < L::Q; ++i) {
            const double f0 = double(Old.f[i * N + n]);
            const double f1 = double(New.f[i * N + n]);
            r0 += f0;
            r1 += f1;
            for (int b = 0; b < L::D; ++b) {
                j0[b] += L::c[i][b] * f0;
                j1[b] += L::c[i][b] * f1;
            }
        }
        const double e1 = double(New.e[n]);
        double d2 = 0;
        for (int b = 0; b < L::D; ++b) {
            const double d = j1[b] / r1 - j0[b] / r0;
            d2 += d * d;
        }
        acc += d2;
        if (!isfinite(d2) || !isfinite(e1) || !isfinite(r1)) bad = 1;
    }
    red[threadIdx.x] = acc;
    nf[threadIdx.x] = bad;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x] += red[threadIdx.x + s];
            nf[threadIdx.x] |= nf[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0];
        partials[2 * blockIdx.x + 1] = nf[0] ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(TPB) k_residual_final(const double* partials, int nparts, double scale, double* out) {
    __shared__ double red[TPB];
    __shared__ double nf[TPB];
    double acc = 0, bad = 0;
    for (int k = threadIdx.x; k < nparts; k += TPB) {
        acc += partials[2 * k];
        bad = fmax(bad, partials[2 * k + 1]);
    }
    red[threadIdx.x] = acc;
    nf[threadIdx.x] = bad;
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x] += red[threadIdx.x + s];
            nf[threadIdx.x] = fmax(nf[threadIdx.x], nf[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sqrt(red[0]) * scale;
        out[1] = (nf[0] > 0.0 || !isfinite(red[0])) ? 1.0 : 0.0;
    }
}

int residual_parts(long long N) {
    const long long b = (N + TPB - 1) / TPB;
    return (int)(b < 1024 ? b : 1024);
}

template <class L, class S>
hipError_t launch_init_state(const SweepArgs& a, StateP<S> A, hipStream_t st) {
    hipLaunchKernelGGL((k_init_state<L, S>), dim3(blocks_for(a.grid.N)), dim3(TPB), 0, st, a, A);
    return hipGetLastError();
}
template <class L, class S>
hipError_t launch_set_fields(const SweepArgs& a, StateP<S> A, const double* rho, const double* u, const double* T,
                             hipStream_t st) {
    hipLaunchKernelGGL((k_set_fields<L, S>), dim3(blocks_for(a.grid.N)), dim3(TPB), 0, st, a, A, rho, u, T);
    return hipGetLastError();
}
template <class L, class S, class O>
hipError_t launch_fields(const SweepArgs& a, StateP<S> A, O* rho, O* u, O* T, O* p, hipStream_t st) {
    hipLaunchKernelGGL((k_fields<L, S, O>), dim3(blocks_for(a.grid.N)), dim3(TPB), 0, st, a, A, rho, u, T, p);
    return hipGetLastError();
}
template <class L, class S>
hipError_t launch_export(const SweepArgs& a, StateP<S> A, int c, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_export<L, S>), dim3(blocks_for(a.grid.N)), dim3(TPB), 0, st, a, A, c, out);
    return hipGetLastError();
}
template <class L, class S>
hipError_t launch_import(const SweepArgs& a, StateP<S> A, int c, const double* in, int* bad, hipStream_t st) {
    hipLaunchKernelGGL((k_import<L, S>), dim3(blocks_for(a.grid.N)), dim3(TPB), 0, st, a, A, c, in, bad);
    return hipGetLastError();
}
template <class L>
hipError_t launch_residual_final(const SweepArgs& a, const double* partials, int nparts, double* out, hipStream_t st) {
    double ur = 0;
    for (int b = 0; b < L::D; ++b) ur += a.fs.u_inf[b] * a.fs.u_inf[b];
    ur = sqrt(ur);
    const double scale = ur > 0 ? 1.0 / (ur * sqrt((double)a.grid.N)) : 1.0 / sqrt((double)a.grid.N);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(TPB), 0, st, partials, nparts, scale, out);
    return hipGetLastError();
}
template hipError_t launch_residual_final<D2Q9>(const SweepArgs&, const double*, int, double*, hipStream_t);
template hipError_t launch_residual_final<D3Q19>(const SweepArgs&, const double*, int, double*, hipStream_t);

template <class L, class S>
hipError_t launch_residual(const SweepArgs& a, StateP<S> Old, StateP<S> New, double* partials, int nparts,
                           double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_residual<L, S>), dim3(nparts), dim3(TPB), 0, st, a, Old, New, partials);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_residual_final<L>(a, partials, nparts, out, st);
}

#define LBMIB_INST_S(L, S)                                                                                     \
    template hipError_t launch_split_step<L, S, S>(const SweepArgs&, StateP<S>, StateP<S>, S*, S*, hipStream_t); \
    template hipError_t launch_init_state<L, S>(const SweepArgs&, StateP<S>, hipStream_t);                     \
    template hipError_t launch_set_fields<L, S>(const SweepArgs&, StateP<S>, const double*, const double*,     \
                                                const double*, hipStream_t);                                   \
    template hipError_t launch_fields<L, S, float>(const SweepArgs&, StateP<S>, float*, float*, float*, float*, \
                                                   hipStream_t);                                               \
    template hipError_t launch_fields<L, S, double>(const SweepArgs&, StateP<S>, double*, double*, double*,    \
                                                    double*, hipStream_t);                                     \
    template hipError_t launch_export<L, S>(const SweepArgs&, StateP<S>, int, double*, hipStream_t);           \
    template hipError_t launch_import<L, S>(const SweepArgs&, StateP<S>, int, const double*, int*, hipStream_t); \
    template hipError_t launch_residual<L, S>(const SweepArgs&, StateP<S>, StateP<S>, double*, int, double*,   \
                                              hipStream_t);

LBMIB_INST_S(D2Q9, float)
LBMIB_INST_S(D2Q9, double)
LBMIB_INST_S(D3Q19, float)
LBMIB_INST_S(D3Q19, double)

}  // namespace lbmib
