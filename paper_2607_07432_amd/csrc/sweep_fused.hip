// Fused single-pass grid sweep: collision, pull streaming, LB face fluxes, MUSCL-Hancock
// energy flux and the rho E update of one time step in one kernel (Eqs. (6), (7), (10),
// (11), (A.3)-(A.16)); every node update reads and writes the state once.
//
// A workgroup owns a TX x TY tile of the plane normal to the marching axis (z in 3D,
// y in 2D) and marches along that axis over a chunk of planes. Rings in LDS:
//   mac  : predicted macros (rho, half-force velocity, T) of 4 planes on the tile + 2 halo;
//   fcA  : post-collision populations moving +1 along the marching axis, 3 planes, tile + 1;
//   fcB  : the other post-collision populations, 2 planes, tile + 1;
//   fex/fey : in-plane face fluxes of the last two output planes.
// Per iteration p: (a) macros of plane p+2; barrier; (b) collision of plane p+1 (needs macros
// of p..p+2 for the velocity gradients) and the end of the output of plane p-1 (flux
// divergence, energy update, stores); barrier; (c) the first part of the output of plane p:
// pull streaming from planes p-1..p+1 into registers, face fluxes of the +x/+y faces (into the
// flux buffer) and of the p+1/2 face (the p-1/2 face is carried in a register).
// Each node of the tile + 1 halo is loaded once per plane, one iteration ahead, and kept in
// registers from its macros to its collision. Only the in-plane halo is recomputed; along the
// marching axis each plane is computed once per chunk (plus a 2-plane warm-up).
#include "kernels.hpp"

namespace lbmib {

namespace {

// Marching-axis component of population i and its slot in the two rings.
template <class L>
__host__ __device__ constexpr int cm(int i) {
    return L::c[i][L::D - 1];
}
template <class L>
__host__ __device__ constexpr int count_up() {
    int n = 0;
    for (int i = 0; i < L::Q; ++i) n += cm<L>(i) == 1;
    return n;
}
template <class L>
__host__ __device__ constexpr int slot_of(int i) {
    int n = 0;
    const bool up = cm<L>(i) == 1;
    for (int j = 0; j < i; ++j) n += (cm<L>(j) == 1) == up;
    return n;
}

__device__ __forceinline__ int wrapm(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Periodic index for |v| < 2n (grids at least a tile plus its halo wide).
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <class L, int TX, int TY>
struct FG {
    static constexpr int D = L::D;
    static constexpr int W1 = TX + 2, H1 = D == 3 ? TY + 2 : 1;
    static constexpr int T = W1 * H1;               // one thread per node of the tile + 1 halo
    static constexpr int W2 = TX + 4, H2 = D == 3 ? TY + 4 : 1;
    static constexpr int N1 = W1 * H1, N2 = W2 * H2;
    static constexpr int OY = D == 3 ? 1 : 0;      // y offset of R1 inside R2 (and of the tile inside R1)
    static constexpr int NA = count_up<L>(), NB = L::Q - count_up<L>();
    static constexpr int NM = D + 2;                // rho, u[D], T
    static constexpr int MA = D - 1;                // marching axis
};

template <class L, class S, class C, int TX, int TY>
struct FusedSmem {
    using G = FG<L, TX, TY>;
    C mac[4][G::NM][G::N2];
    C fcA[3][G::NA][G::N1];
    C fcB[2][G::NB][G::N1];
    C fex[2][TY][TX + 1];
    C fey[2][G::D == 3 ? TY + 1 : 1][G::D == 3 ? TX : 1];   // unused in 2D
};

struct FusedArgs {
    int tiles_x, tiles_y, chunks, chunk, total, per_xcd;
    int small;      // a grid dimension is smaller than a tile plus halo: use the general modulo
    int fb[6];      // bounding box of the forced nodes (x, y, marching axis; empty if min > max)
    double* rpart;  // residual partials (sum of |u_new - u_old|^2, non-finite flag) per workgroup
};

}  // namespace

// One work item: the tile at (x0, y0) of planes [z0, z1) of one grid. Periodic indices: SM = 0
// by one conditional wrap (valid while a grid dimension exceeds the tile), SM = 1 by the general
// modulo, SM = 2 as the runtime flag small says.
// OUT: the tile holds column nx - 3 under the inflow/outflow closure, so its outlet columns are
// rescaled here. FRC: the tile's footprint (tile + 2 nodes, planes z0 - 2 .. z1 + 1) may hold
// forced nodes; without it the row map is not read and the forcing path compiles away. INL: the
// tile holds the inlet columns 0, 1. They are template flags so that the common tiles' loop is
// compiled without these rare paths.
// RES: the step's residual terms are accumulated on the way (FP64, from the stored states):
// racc += |u_new - u_old|^2 over the tile's output nodes, rbad = 1 on a non-finite value.
template <class L, class S, class C, int TX, int TY, int SM, bool OUT = false, bool FRC = true, bool INL = true,
          bool RES = false>
__device__ __forceinline__ void fused_tile(const FusedK<C>& a, StateP<S> A, StateP<S> B, int x0, int y0, int z0,
                                           int z1, bool small, FusedSmem<L, S, C, TX, TY>& sm, double* racc = nullptr,
                                           int* rbad = nullptr) {
    using G = FG<L, TX, TY>;
    constexpr int D = L::D;
    const FusedK<C>& g = a;
    const long long N = g.N;
    // Every state and forcing array lives in device memory: accessed through pointers typed in
    // the global address space, also when they were read from a device table.
    using GS = __attribute__((address_space(1))) S;
    using GD = __attribute__((address_space(1))) double;
    using GI = __attribute__((address_space(1))) const int;
    GS* const Af = (GS*)A.f;
    GS* const Ae = (GS*)A.e;
    GS* const Ah = (GS*)A.h2;
    GS* const Bf = (GS*)B.f;
    GS* const Be = (GS*)B.e;
    GS* const Bh = (GS*)B.h2;
    GI* const rowmap = (GI*)a.rows.rowmap;
    GD* const rfib = (GD*)a.rows.fib;
    GD* const rfE = (GD*)a.rows.fE;
    const GD* const rh2off = (const GD*)a.rows.h2off;
    GD* const rh2out = (GD*)a.rows.h2off_out;
    const int nm = D == 3 ? g.nz : g.ny;               // length of the marching axis
    const int t = threadIdx.x;

    auto wr = [&](int v, int n) {
        if (SM == 0) return wrap1(v, n);
        if (SM == 1) return wrapm(v, n);
        return small ? wrapm(v, n) : wrap1(v, n);
    };
    auto gnode = [&](int x, int y, int m) -> long long {
        const int xw = wr(x, g.nx);
        if (D == 3) return (long long)xw + (long long)g.nx * ((long long)wr(y, g.ny) + (long long)g.ny * wr(m, nm));
        return (long long)xw + (long long)g.nx * wr(m, nm);
    };
    auto s4 = [](int q) { return (q + 8) % 4; };  // macros ring
    auto s3 = [](int q) { return (q + 6) % 3; };  // post-collision +z movers
    auto s2 = [](int q) { return (q + 6) % 2; };  // other post-collision populations, flux buffers

    // ---- Loads. Every node of the tile + 1 halo (R1, one per thread) is read once per plane: its
    // populations, energy, history and row serve first the macros (stage a) and one plane later
    // its collision (stage b), so they are kept in registers across one iteration (cur: plane of
    // the next collision, nxt: plane of the next macros). The outer ring of the tile + 2 halo
    // (R2 minus R1) only needs macros; threads t < NRING load one ring node each.
    struct Own {
        S f[L::Q];
        S e;
        S h[2];
        int r;
    };
    constexpr int NRING = D == 3 ? 2 * G::W2 + 2 * (G::H2 - 2) : 2;
    static_assert(NRING <= G::T, "ring larger than the workgroup");
    const int jx1 = t % G::W1, jy1 = D == 3 ? t / G::W1 : 0;
    const int k2own = (jx1 + 1) + G::W2 * (jy1 + G::OY);                        // R2 coords of the own node
    const bool ring = t < NRING;
    int rjx, rjy;                                                               // R2 coords of the ring node
    if (D == 3) {
        if (t < G::W2) {
            rjx = t;
            rjy = 0;
        } else if (t < 2 * G::W2) {
            rjx = t - G::W2;
            rjy = G::H2 - 1;
        } else {
            const int k = t - 2 * G::W2;
            rjx = (k & 1) ? G::W2 - 1 : 0;
            rjy = 1 + k / 2;
        }
    } else {
        rjx = t == 0 ? 0 : G::W2 - 1;
        rjy = 0;
    }
    const int k2ring = rjx + G::W2 * rjy;
    Own cur, nxt;
    S rf[L::Q];
    S re = S(0);
    int rr = -1;
    auto load_plane = [&](int q) {
        const long long n = gnode(x0 - 1 + jx1, y0 - G::OY + jy1, q);
#pragma unroll
        for (int i = 0; i < L::Q; ++i) nxt.f[i] = Af[i * N + n];
        nxt.e = Ae[n];
        nxt.h[0] = Ah[n];
        nxt.h[1] = D == 3 ? Ah[N + n] : S(0);
        nxt.r = FRC ? rowmap[n] : -1;
        if (ring) {
            const long long m = gnode(x0 - 2 + rjx, y0 - 2 * G::OY + rjy, q);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) rf[i] = Af[i * N + m];
            re = Ae[m];
            rr = FRC ? rowmap[m] : -1;
        }
    };
    auto shift_planes = [&]() { cur = nxt; };

    // ---- (a) predicted macros (rho, half-force velocity, T) of one node into the ring slot sl.
    auto write_macros = [&](const S* f, S e, int r, int k, int sl) {
        C drho = 0, j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const C fv = C(f[i]);
            drho += fv;
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (L::c[i][b]) j[b] += C(L::c[i][b]) * fv;
        }
        const C rho = C(1) + drho;
        const C ir = C(1) / rho;
        C uu = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) uu += (j[b] * ir) * (j[b] * ir);
        const C T = ((C(e) + a.e_ref) * ir - C(0.5) * uu) * a.gas.inv_Cv;
        sm.mac[sl][0][k] = rho;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const C fib = r >= 0 ? C(rfib[(long long)b * a.rows.nrows + r]) : C(0);
            sm.mac[sl][1 + b][k] = (j[b] + C(0.5) * fib) * ir;
        }
        sm.mac[sl][1 + D][k] = T;
    };
    auto compute_macros = [&](int q) {
        const int sl = s4(q);
        write_macros(nxt.f, nxt.e, nxt.r, k2own, sl);
        if (ring) write_macros(rf, re, rr, k2ring, sl);
    };

    auto mcell = [&](int sl, int k2) {
        Cell<L, C> c;
        c.rho = sm.mac[sl][0][k2];
#pragma unroll
        for (int b = 0; b < 3; ++b) c.u[b] = b < D ? sm.mac[sl][1 + b][k2] : C(0);
        c.T = sm.mac[sl][1 + D][k2];
        return c;
    };

    // ---- residual (RES): u^n of the own node from its collision, kept until its output plane
    // is finished two planes later (ru0: the older, ru1: the newer collided plane)
    double ru_new[3] = {0, 0, 0}, ru0[3] = {0, 0, 0}, ru1[3] = {0, 0, 0};
    auto res_push = [&]() {
        if constexpr (RES) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                ru0[b] = ru1[b];
                ru1[b] = ru_new[b];
            }
        }
    };

    // ---- (b) collision of plane q on the tile + 1 halo (one node per thread, from cur)
    auto compute_collide = [&](int q) {
        const int sl = s4(q), slm = s4(q - 1), slp = s4(q + 1);
        const int sa = s3(q), sb = s2(q);
        {
            const int k = t;
            const int jx = k % G::W1, jy = k / G::W1;
            const int k2 = (jx + 1) + G::W2 * (jy + G::OY);
            const int xu = x0 - 1 + jx, yu = y0 - G::OY + jy;
            const long long n = gnode(xu, yu, q);
            C fd[L::Q];
#pragma unroll
            for (int i = 0; i < L::Q; ++i) fd[i] = C(cur.f[i]);
            if constexpr (RES) {
                // force-free velocity of the stored state, FP64 (the residual's u^n)
                double r0 = 1, j0[3] = {0, 0, 0};
#pragma unroll
                for (int i = 0; i < L::Q; ++i) {
                    const double fv = double(cur.f[i]);
                    r0 += fv;
#pragma unroll
                    for (int b = 0; b < D; ++b)
                        if (L::c[i][b]) j0[b] += L::c[i][b] * fv;
                }
                const double ir0 = 1.0 / r0;
#pragma unroll
                for (int b = 0; b < D; ++b) ru_new[b] = j0[b] * ir0;
            }
            const Cell<L, C> c0 = mcell(sl, k2);
            Node<L, C> nd;
            nd.rho = c0.rho;
            nd.inv_rho = C(1) / c0.rho;
            nd.T = c0.T;
#pragma unroll
            for (int b = 0; b < 3; ++b) nd.u[b] = c0.u[b];
            Stencil<C> st;
            st.div_rhou = 0;
            st.u_grad_p = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                st.dmu3[b] = 0;
#pragma unroll
                for (int qq = 0; qq < 3; ++qq) st.du[qq][b] = 0;
            }
#pragma unroll
            for (int b = 0; b < D; ++b) {
                Cell<L, C> cp, cmn;
                if (b == G::MA) {
                    cp = mcell(slp, k2);
                    cmn = mcell(slm, k2);
                } else {
                    const int stride = b == 0 ? 1 : G::W2;
                    cp = mcell(sl, k2 + stride);
                    cmn = mcell(sl, k2 - stride);
                }
#pragma unroll
                for (int qq = 0; qq < D; ++qq) st.du[qq][b] = C(0.5) * (cp.u[qq] - cmn.u[qq]);
                st.div_rhou += C(0.5) * (cp.rho * cp.u[b] - cmn.rho * cmn.u[b]);
                st.u_grad_p += nd.u[b] * C(0.5) * (cp.rho * cp.T - cmn.rho * cmn.T);
                st.dmu3[b] = C(0.5) * (cp.rho * cp.u[b] * cp.u[b] * cp.u[b] - cmn.rho * cmn.u[b] * cmn.u[b] * cmn.u[b]);
            }
            C H2[3][3];
            H2[0][0] = C(cur.h[0]);
            if (D == 3) {
                H2[1][1] = C(cur.h[1]);
                H2[2][2] = -(H2[0][0] + H2[1][1]);
            } else {
                H2[1][1] = -H2[0][0];
            }
            const int r = cur.r;
            const int nr = a.rows.nrows;
            C fib[3] = {0, 0, 0}, off[3] = {0, 0, 0};
            if (r >= 0) {
#pragma unroll
                for (int b = 0; b < D; ++b) fib[b] = C(rfib[(long long)b * nr + r]);
#pragma unroll
                for (int kk = 0; kk < L::NOFF; ++kk) off[kk] = C(rh2off[(long long)kk * nr + r]);
            }
            H2[0][1] = H2[1][0] = off[0];
            if (D == 3) {
                H2[0][2] = H2[2][0] = off[1];
                H2[1][2] = H2[2][1] = off[2];
            }
            C fc[L::Q];
            C H2n[3][3];
            collide<L, C>(a.gas, fd, nd, st, fib, H2, fc, H2n);
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                if (cm<L>(i) == 1)
                    sm.fcA[sa][slot_of<L>(i)][k] = fc[i];
                else
                    sm.fcB[sb][slot_of<L>(i)][k] = fc[i];
            }
            // Tile nodes (not halo, not beyond the grid) write the new history.
            const bool tile = jx >= 1 && jx <= TX && (D == 2 || (jy >= 1 && jy <= TY)) && xu < g.nx &&
                              (D == 2 || yu < g.ny);
            if (tile) {
                if (r >= 0) {
                    rh2out[r] = H2n[0][1];
                    if (D == 3) {
                        rh2out[(long long)nr + r] = H2n[0][2];
                        rh2out[2LL * nr + r] = H2n[1][2];
                    }
                }
                int copies = 1;
                bool write = true;
                if (g.bc_x >= 1) {
                    if (INL && xu < 2) {
                        Bh[n] = S(0);
                        if (D == 3) Bh[N + n] = S(0);
                        write = false;
                    } else if (xu >= g.nx - 2) {
                        write = false;
                    } else if (xu == g.nx - 3 && g.bc_x == 1) {
                        copies = 3;
                    }
                }
                if (write)
                    for (int c = 0; c < copies; ++c) {
                        Bh[n + c] = S(H2n[0][0]);
                        if (D == 3) Bh[N + n + c] = S(H2n[1][1]);
                    }
            }
        }
    };

    // Post-collision population i at R1 coords (jx, jy) of plane q.
    auto fcr = [&](int i, int jx, int jy, int q) -> C {
        const int k = jx + G::W1 * jy;
        if (cm<L>(i) == 1) return sm.fcA[s3(q)][slot_of<L>(i)][k];
        return sm.fcB[s2(q)][slot_of<L>(i)][k];
    };

    // LB mass and momentum (lattice-weight part removed) flux through the face base + e_ax/2,
    // base at R1 coords (bx, by) of plane q; ax is a physical axis (Eqs. (A.11)-(A.13)).
    auto lb_flux = [&](int ax, int bx, int by, int q, C& Fr, C* Fm) {
        Fr = 0;
        Fm[0] = Fm[1] = Fm[2] = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const int ci = L::c[i][ax];
            if (ci == 0) continue;
            const int cx = L::c[i][0], cy = D == 3 ? L::c[i][1] : 0, cmi = cm<L>(i);
            C v;
            if (ax == G::MA) {
                if (ci == 1)
                    v = C(0.5) * (fcr(i, bx, by, q) + fcr(i, bx - cx, by - cy, q));
                else
                    v = -C(0.5) * (fcr(i, bx, by, q + 1) + fcr(i, bx - cx, by - cy, q + 1));
            } else {
                const int ex = ax == 0, ey = ax == 1;
                if (ci == 1)
                    v = C(0.5) * (fcr(i, bx, by, q) + fcr(i, bx + ex - cx, by + ey - cy, q - cmi));
                else
                    v = -C(0.5) * (fcr(i, bx + ex, by + ey, q) + fcr(i, bx - cx, by - cy, q - cmi));
            }
            Fr += v;
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (L::c[i][b]) Fm[b] += C(L::c[i][b]) * v;
        }
    };

    // In-plane energy flux through the face base + e_ax/2 (base at R1 coords), plane q.
    auto inplane_flux = [&](int ax, int bx, int by, int q) -> C {
        C Fr, Fm[3];
        lb_flux(ax, bx, by, q, Fr, Fm);
        const int sl = s4(q);
        const int k2 = (bx + 1) + G::W2 * (by + G::OY);
        const int stride = ax == 0 ? 1 : G::W2;
        Cell<L, C> c4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c4[u] = mcell(sl, k2 + (u - 1) * stride);
        return energy_flux<L, C>(a.gas, ax, c4, Fr, Fm);
    };

    // Node of this thread in the tile + 1 halo (R1 coords); interior threads own an output node.
    const bool own_out = jx1 >= 1 && jx1 <= TX && (D == 2 || (jy1 >= 1 && jy1 <= TY));
    const bool own_fx = jx1 <= TX && (D == 2 || (jy1 >= 1 && jy1 <= TY));      // face base + e_x/2
    const bool own_fy = D == 3 && jx1 >= 1 && jx1 <= TX && jy1 <= TY;          // face base + e_y/2
    const int bx1 = jx1, by1 = jy1;
    const int xo = x0 - 1 + jx1, yo = y0 - G::OY + jy1;
    const bool real = own_out && xo < g.nx && (D == 2 || yo < g.ny);
    const int frow = D == 3 ? jy1 - 1 : 0;

    // ---- prologue: macros of z0-2 .. z0+1, collisions of z0-1 and z0
    load_plane(z0 - 2);
    compute_macros(z0 - 2);
    load_plane(z0 - 1);
    compute_macros(z0 - 1);
    shift_planes();                                 // cur: plane z0 - 1
    load_plane(z0);
    compute_macros(z0);
    __syncthreads();
    compute_collide(z0 - 1);
    res_push();
    shift_planes();                                 // cur: plane z0
    __syncthreads();
    Cell<L, C> cm2 = mcell(s4(z0 - 2), k2own);
    Cell<L, C> prev = mcell(s4(z0 - 1), k2own);   // own column, plane p - 1
    __syncthreads();
    load_plane(z0 + 1);
    compute_macros(z0 + 1);
    __syncthreads();
    compute_collide(z0);
    res_push();
    // energy and row of the own node for its output one plane later (its forcing is prefetched)
    S ekeep = cur.e;
    int rkeep = cur.r;
    C fEkeep = rkeep >= 0 ? C(rfE[rkeep]) : C(0);
    shift_planes();                                 // cur: plane z0 + 1
    __syncthreads();
    C fm_prev = 0;                                  // energy flux through the p - 1/2 face
    if (own_out) {
        C Fr, Fm[3];
        lb_flux(G::MA, bx1, by1, z0 - 1, Fr, Fm);
        Cell<L, C> c4[4] = {cm2, prev, mcell(s4(z0), k2own), mcell(s4(z0 + 1), k2own)};
        fm_prev = energy_flux<L, C>(a.gas, G::MA, c4, Fr, Fm);
    }
    load_plane(z0 + 2);                             // nxt: plane z0 + 2

    // The output of plane p is prepared after the second barrier of iteration p (streaming into
    // registers, face fluxes into the buffer p % 2) and finished after the first barrier of
    // iteration p + 1 (flux divergence, energy update, stores), so each plane needs two barriers.
    C pf[L::Q];                                     // streamed populations of the pending plane
    C pfm = 0, pfmp = 0;                            // its p + 1/2 and p - 1/2 face fluxes
    S pe = S(0);
    C pfE = 0;
    // u^{n+1} of the pending output plane from the values stored for it (the free stream at the
    // inlet; at the outlet copies, column nx - 3, whose rescaled copy has the same velocity)
    auto res_acc = [&]() {
        if constexpr (RES) {
            if (!real) return;
            const bool inl = INL && g.bc_x >= 1 && xo < 2;
            double r1 = 1, j1[3] = {0, 0, 0};
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const double fv = inl ? double(S(a.fdev[i])) : double(S(pf[i]));
                r1 += fv;
#pragma unroll
                for (int b = 0; b < D; ++b)
                    if (L::c[i][b]) j1[b] += L::c[i][b] * fv;
            }
            const double ir1 = 1.0 / r1;
            double d2 = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const double d = j1[b] * ir1 - ru0[b];
                d2 += d * d;
            }
            *racc += d2;
            if (!isfinite(d2) || !isfinite(r1)) *rbad = 1;
        }
    };
    auto finish = [&](int q) {
        if (!real) return;
        const int fb = s2(q);
        C ediv = (sm.fex[fb][frow][jx1] - sm.fex[fb][frow][jx1 - 1]) + (pfm - pfmp);
        if constexpr (D == 3) ediv += sm.fey[fb][jy1][jx1 - 1] - sm.fey[fb][jy1 - 1][jx1 - 1];
        const long long n = gnode(xo, yo, q);
        if (g.bc_x >= 1) {
            if (INL && xo < 2) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i) Bf[i * N + n] = S(a.fdev[i]);
                Be[n] = S(0);
                return;
            }
            if (xo >= g.nx - 2) return;
        }
        const C enew = C(pe) - ediv + pfE;
        if constexpr (RES)
            if (!isfinite(double(enew))) *rbad = 1;
        if constexpr (OUT) {
            // outlet columns nx - 2, nx - 1: column nx - 3 rescaled by p_inf / p
#pragma unroll
            for (int i = 0; i < L::Q; ++i) Bf[i * N + n] = S(pf[i]);
            Be[n] = S(enew);
            if (g.bc_x == 1 && xo == g.nx - 3) {
                const C sc = outlet_scale<L, C>(pf, enew, a.e_ref, a.eint_inf);
                if constexpr (RES)
                    if (!isfinite(double(sc))) *rbad = 1;
                for (int c = 1; c < 3; ++c) {
#pragma unroll
                    for (int i = 0; i < L::Q; ++i) Bf[i * N + n + c] = S(sc * pf[i] + (sc - C(1)) * C(L::w[i]));
                    Be[n + c] = S(sc * enew + (sc - C(1)) * a.e_ref);
                }
            }
        } else {
            // (written as a copy loop, which other tiles never repeat: this form of the store
            // compiles to the faster 3D loop, 1.282 against 1.312 ms per sweep for a single store)
            const int copies = (g.bc_x == 1 && xo == g.nx - 3) ? 3 : 1;
            for (int c = 0; c < copies; ++c) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i) Bf[i * N + n + c] = S(pf[i]);
                Be[n + c] = S(enew);
            }
        }
    };

    for (int p = z0; p < z1; ++p) {
        compute_macros(p + 2);
        __syncthreads();
        if (RES && p > z0) res_acc();               // plane p - 1 (ru0), before the next push
        compute_collide(p + 1);
        res_push();
        if (p > z0) finish(p - 1);
        __syncthreads();
        // Issue the next plane's global loads now; they complete while plane p is prepared.
        const S eout = ekeep;                       // own node, plane p
        const C fEout = fEkeep;
        ekeep = cur.e;                              // plane p + 1
        rkeep = cur.r;
        fEkeep = rkeep >= 0 ? C(rfE[rkeep]) : C(0);
        shift_planes();                             // cur: plane p + 2
        if (p + 1 < z1) load_plane(p + 3);

        // ---- (c) output plane p, first part
        const int fb = s2(p);
        if (own_out) {
            // (RES: the outlet copies take the populations of column nx - 3, in the same tile, for
            // their u^{n+1}; they store nothing themselves)
            int sx = 0;
            if constexpr (RES && OUT)
                if (g.bc_x == 1 && xo >= g.nx - 2) sx = xo - (g.nx - 3);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                pf[i] = fcr(i, bx1 - sx - L::c[i][0], by1 - (D == 3 ? L::c[i][1] : 0), p - cm<L>(i));
        }
        if (own_fx) sm.fex[fb][frow][jx1] = inplane_flux(0, bx1, by1, p);
        if constexpr (D == 3) if (own_fy) sm.fey[fb][jy1][jx1 - 1] = inplane_flux(1, bx1, by1, p);
        C fm_now = 0;
        if (own_out) {
            C Fr, Fm[3];
            lb_flux(G::MA, bx1, by1, p, Fr, Fm);
            const Cell<L, C> cp0 = mcell(s4(p), k2own);
            Cell<L, C> c4[4] = {prev, cp0, mcell(s4(p + 1), k2own), mcell(s4(p + 2), k2own)};
            fm_now = energy_flux<L, C>(a.gas, G::MA, c4, Fr, Fm);
            prev = cp0;
        }
        pfm = fm_now;
        pfmp = fm_prev;
        pe = eout;
        pfE = fEout;
        fm_prev = fm_now;
    }
    __syncthreads();
    if constexpr (RES) res_acc();                   // plane z1 - 1
    finish(z1 - 1);
}

template <class L, class S, class C, int TX, int TY, int SM, bool RES>
__global__ void __launch_bounds__((TX + 2) * (L::D == 3 ? TY + 2 : 1)) k_fused(FusedK<C> a, FusedArgs fa, StateP<S> A, StateP<S> B) {
    __shared__ FusedSmem<L, S, C, TX, TY> sm;
    constexpr int D = L::D;
    // XCD-aware placement: consecutive logical workgroups (neighbouring tiles) share an XCD.
    const int w = blockIdx.x;
    const int logical = (w % 8) * fa.per_xcd + w / 8;
    if (logical >= fa.total) return;
    const int per_plane = fa.tiles_x * fa.tiles_y;
    const int chunk = logical / per_plane;
    const int rem = logical % per_plane;
    const int x0 = (rem % fa.tiles_x) * TX;
    const int y0 = D == 3 ? (rem / fa.tiles_x) * TY : 0;
    const int nm = D == 3 ? a.nz : a.ny;
    const int z0 = chunk * fa.chunk;
    const int z1 = min(z0 + fa.chunk, nm);
    // Rare paths in their own instantiations (in every tile's loop they slow the 3D sweep through
    // code generation: the outlet rescaling by 4.5 %, the forcing path by 3 %, the inlet reset by
    // 2.4 %). Four instantiations: the common tile, inlet-only, outlet-only, and one with every
    // path, which is correct for any tile (forced tiles, small grids, a tile with both closures).
    const bool out = a.bc_x == 1 && x0 <= a.nx - 3 && a.nx - 3 <= x0 + TX - 1;
    const bool inl = a.bc_x >= 1 && x0 < 2;
    const int* fb = fa.fb;
    const bool frc = SM == 1 || (fb[0] <= fb[1] && x0 - 2 <= fb[1] && x0 + TX + 1 >= fb[0] &&
                                 (D == 2 || (y0 - 2 <= fb[3] && y0 + TY + 1 >= fb[2])) && z0 - 2 <= fb[5] &&
                                 z1 + 1 >= fb[4]);
    double racc = 0;
    int rbad = 0;
    if (!frc && !out && !inl)
        fused_tile<L, S, C, TX, TY, SM, false, false, false, RES>(a, A, B, x0, y0, z0, z1, SM == 1, sm, &racc, &rbad);
    else if (!frc && !out)
        fused_tile<L, S, C, TX, TY, SM, false, false, true, RES>(a, A, B, x0, y0, z0, z1, SM == 1, sm, &racc, &rbad);
    else if (!frc && !inl)
        fused_tile<L, S, C, TX, TY, SM, true, false, false, RES>(a, A, B, x0, y0, z0, z1, SM == 1, sm, &racc, &rbad);
    else
        fused_tile<L, S, C, TX, TY, SM, true, true, true, RES>(a, A, B, x0, y0, z0, z1, SM == 1, sm, &racc, &rbad);
    if constexpr (RES) {
        // workgroup sum in a fixed order (LDS reused), one partial per logical workgroup
        constexpr int NT = (TX + 2) * (L::D == 3 ? TY + 2 : 1);
        static_assert(sizeof(sm) >= NT * (sizeof(double) + sizeof(int)), "reduction space");
        __syncthreads();
        double* red = reinterpret_cast<double*>(&sm);
        int* bad = reinterpret_cast<int*>(red + NT);
        const int t = threadIdx.x;
        red[t] = racc;
        bad[t] = rbad;
        __syncthreads();
        constexpr int P2 = NT <= 64 ? 64 : (NT <= 128 ? 128 : (NT <= 256 ? 256 : (NT <= 512 ? 512 : 1024)));
        static_assert(NT <= P2 && P2 <= 1024, "workgroup size");
#pragma unroll
        for (int h = P2 / 2; h > 0; h >>= 1) {
            if (t < h && t + h < NT) {
                red[t] += red[t + h];
                bad[t] |= bad[t + h];
            }
            __syncthreads();
        }
        if (t == 0) {
            fa.rpart[2 * logical] = red[0];
            fa.rpart[2 * logical + 1] = bad[0] ? 1.0 : 0.0;
        }
    }
}

// Persistent sweep over the work items of a batch of 2D grids. The items of one case are
// consecutive (rows of tiles, then chunks along y); each XCD takes a contiguous range of the
// item list and its workgroups stride through it, so that neighbouring tiles share an L2.
template <class L, class S, int TX>
__global__ void __launch_bounds__(TX + 2) k_fused_batch(const CaseDesc<S>* __restrict__ cases, int ncases, int total,
                                                        int g) {
    static_assert(L::D == 2, "batches hold 2D grids");
    __shared__ FusedSmem<L, S, S, TX, 1> sm;
    const int per_xcd = (total + 7) / 8;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, nslots = gridDim.x / 8;
    for (int k = slot; k < per_xcd; k += nslots) {
        const int w = xcd * per_xcd + k;
        if (w >= total) break;
        int lo = 0, hi = ncases - 1;                  // last case with item0 <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (cases[mid].item0 <= w) lo = mid; else hi = mid - 1;
        }
        const CaseDesc<S>& cd = cases[lo];
        const int cur = (cd.cur0 + g) & 1;
        const int local = w - cd.item0;
        const int chunk = local / cd.tiles_x;
        const int x0 = (local % cd.tiles_x) * TX;
        const int z0 = chunk * cd.chunk;
        const int z1 = min(z0 + cd.chunk, cd.k[0].ny);
        // the case's arguments in registers for the whole item
        const FusedK<S> ka = cd.k[cur];
        const StateP<S> A = cd.st[cur], B = cd.st[cur ^ 1];
        const bool small = cd.small != 0;
        // the same four instantiations as the single-grid sweep, chosen per item
        const bool out = ka.bc_x == 1 && x0 <= ka.nx - 3 && ka.nx - 3 <= x0 + TX - 1;
        const bool inl = ka.bc_x == 1 && x0 < 2;
        const bool frc = small || (cd.fb[0] <= cd.fb[1] && x0 - 2 <= cd.fb[1] && x0 + TX + 1 >= cd.fb[0] &&
                                   z0 - 2 <= cd.fb[5] && z1 + 1 >= cd.fb[4]);
        __syncthreads();                              // the previous item's LDS reads are done
        if (!frc && !out && !inl)
            fused_tile<L, S, S, TX, 1, 2, false, false, false>(ka, A, B, x0, 0, z0, z1, small, sm);
        else if (!frc && !out)
            fused_tile<L, S, S, TX, 1, 2, false, false, true>(ka, A, B, x0, 0, z0, z1, small, sm);
        else if (!frc && !inl)
            fused_tile<L, S, S, TX, 1, 2, true, false, false>(ka, A, B, x0, 0, z0, z1, small, sm);
        else
            fused_tile<L, S, S, TX, 1, 2, true, true, true>(ka, A, B, x0, 0, z0, z1, small, sm);
    }
}

namespace {

template <class L, class S>
struct Tile;
template <>
struct Tile<D3Q19, float> {
    static constexpr int TX = 30, TY = 14, CHUNK = 48;
};
template <>
struct Tile<D3Q19, double> {
    static constexpr int TX = 30, TY = 6, CHUNK = 16;
};
template <>
struct Tile<D2Q9, float> {
    static constexpr int TX = 254, TY = 1, CHUNK = 32;
};
template <>
struct Tile<D2Q9, double> {
    static constexpr int TX = 254, TY = 1, CHUNK = 32;
};

}  // namespace

template <class L, class S, int TX, int TY>
hipError_t launch_fused_tile(const SweepArgs& a, StateP<S> A, StateP<S> B, int chunk, int default_chunk,
                             const int* fbox, hipStream_t st, double* rpart, int rcap, int* rparts) {
    const GridP& g = a.grid;
    FusedArgs fa;
    fa.tiles_x = (g.nx + TX - 1) / TX;
    fa.tiles_y = L::D == 3 ? (g.ny + TY - 1) / TY : 1;
    const int nm = L::D == 3 ? g.nz : g.ny;
    fa.chunk = chunk > 0 ? chunk : default_chunk;
    fa.chunks = (nm + fa.chunk - 1) / fa.chunk;
    fa.total = fa.tiles_x * fa.tiles_y * fa.chunks;
    fa.per_xcd = (fa.total + 7) / 8;
    fa.small = (g.nx <= TX) || (L::D == 3 && g.ny <= TY) || nm < 4;
    for (int i = 0; i < 6; ++i) fa.fb[i] = fbox[i];
    // The residual is formed in the sweep when every workgroup has a partial slot and the outlet
    // copies share a tile with their source column nx - 3; otherwise the caller runs k_residual.
    const bool res = rpart && fa.total <= rcap && (g.bc_x == 0 || (g.bc_x == 1 && (g.nx - 3) % TX <= TX - 3));
    fa.rpart = res ? rpart : nullptr;
    if (rparts) *rparts = res ? fa.total : 0;
    const int grid = fa.per_xcd * 8;
    constexpr int threads = (TX + 2) * (L::D == 3 ? TY + 2 : 1);
    const FusedK<S> k = fused_args<S>(a);
    if (fa.small && res)
        hipLaunchKernelGGL((k_fused<L, S, S, TX, TY, 1, true>), dim3(grid), dim3(threads), 0, st, k, fa, A, B);
    else if (fa.small)
        hipLaunchKernelGGL((k_fused<L, S, S, TX, TY, 1, false>), dim3(grid), dim3(threads), 0, st, k, fa, A, B);
    else if (res)
        hipLaunchKernelGGL((k_fused<L, S, S, TX, TY, 0, true>), dim3(grid), dim3(threads), 0, st, k, fa, A, B);
    else
        hipLaunchKernelGGL((k_fused<L, S, S, TX, TY, 0, false>), dim3(grid), dim3(threads), 0, st, k, fa, A, B);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_fused_step(const SweepArgs& a, StateP<S> A, StateP<S> B, int chunk, const int* fbox,
                             hipStream_t st, double* rpart, int rcap, int* rparts) {
    using TL = Tile<L, S>;
    return launch_fused_tile<L, S, TL::TX, TL::TY>(a, A, B, chunk, TL::CHUNK, fbox, st, rpart, rcap, rparts);
}

// Planes per work item for a grid on a device with `cus` compute units. A work item costs about
// its planes plus three (a chunk's first planes recompute what the previous chunk's last ones
// computed; the choice moves the states only through which tile code covers a plane, to
// rounding), and the items run in rounds of as many
// workgroups as the chip holds at once; the chunk minimising rounds x (planes + 3) over 64, 48, 32,
// 24, 16, 12 and 8 planes is taken, the longer one on a tie. Measured sweep times order the
// chunks as this estimate does on 384x192x192, 384x192x96, 256x128x128 (FP32) and on 384x192x192
// and 192x96x96 (FP64).
template <class L, class S>
int fused_auto_chunk(const GridP& g, int cus) {
    using TL = Tile<L, S>;
    constexpr int threads = (TL::TX + 2) * (L::D == 3 ? TL::TY + 2 : 1);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fused<L, S, S, TL::TX, TL::TY, 0, false>, threads, 0) !=
            hipSuccess ||
        occ < 1)
        occ = 1;
    const long long slots = (long long)occ * (cus > 0 ? cus : 256);
    const long long tiles = (long long)((g.nx + TL::TX - 1) / TL::TX) * (L::D == 3 ? (g.ny + TL::TY - 1) / TL::TY : 1);
    const int nm = L::D == 3 ? g.nz : g.ny;
    int best = TL::CHUNK;
    long long best_cost = -1;
    for (int c : {64, 48, 32, 24, 16, 12, 8}) {
        const int planes = c < nm ? c : nm;
        const long long items = tiles * ((nm + planes - 1) / planes);
        const long long cost = (items + slots - 1) / slots * (planes + 3);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = planes;
        }
    }
    return best;
}

template <class L, class S>
hipError_t launch_fused_batch(const CaseDesc<S>* cases, int ncases, int total_items, int tx, int grid, int g,
                              hipStream_t st) {
    if (total_items <= 0) return hipSuccess;
    if (grid < 8 || grid % 8) return hipErrorInvalidValue;
    switch (tx) {
        case 62:
            hipLaunchKernelGGL((k_fused_batch<L, S, 62>), dim3(grid), dim3(64), 0, st, cases, ncases, total_items, g);
            break;
        case 126:
            hipLaunchKernelGGL((k_fused_batch<L, S, 126>), dim3(grid), dim3(128), 0, st, cases, ncases, total_items, g);
            break;
        case 254:
            hipLaunchKernelGGL((k_fused_batch<L, S, 254>), dim3(grid), dim3(256), 0, st, cases, ncases, total_items, g);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class L, class S>
int fused_batch_occupancy(int tx) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (tx == 62) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused_batch<L, S, 62>, 64, 0);
    if (tx == 126) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused_batch<L, S, 126>, 128, 0);
    if (tx == 254) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused_batch<L, S, 254>, 256, 0);
    return e == hipSuccess ? nb : 0;
}

template hipError_t launch_fused_batch<D2Q9, float>(const CaseDesc<float>*, int, int, int, int, int, hipStream_t);
template hipError_t launch_fused_batch<D2Q9, double>(const CaseDesc<double>*, int, int, int, int, int, hipStream_t);
template int fused_batch_occupancy<D2Q9, float>(int);
template int fused_batch_occupancy<D2Q9, double>(int);
template int fused_auto_chunk<D2Q9, float>(const GridP&, int);
template int fused_auto_chunk<D2Q9, double>(const GridP&, int);
template int fused_auto_chunk<D3Q19, float>(const GridP&, int);
template int fused_auto_chunk<D3Q19, double>(const GridP&, int);

template hipError_t launch_fused_step<D2Q9, float>(const SweepArgs&, StateP<float>, StateP<float>, int, const int*, hipStream_t,
                                                  double*, int, int*);
template hipError_t launch_fused_step<D2Q9, double>(const SweepArgs&, StateP<double>, StateP<double>, int, const int*, hipStream_t,
                                                  double*, int, int*);
template hipError_t launch_fused_step<D3Q19, float>(const SweepArgs&, StateP<float>, StateP<float>, int, const int*, hipStream_t,
                                                  double*, int, int*);
template hipError_t launch_fused_step<D3Q19, double>(const SweepArgs&, StateP<double>, StateP<double>, int, const int*, hipStream_t,
                                                  double*, int, int*);

}  // namespace lbmib
