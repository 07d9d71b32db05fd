// Two-level grid refinement (ratio 2): a fine handle embedded in a coarse one, coupled by a band
// refilled from the coarse grid and by restriction of the fine block (contract in include/lbmib.h).
//
// Both transfers are gathers with one thread per destination node, FP64 arithmetic whatever the
// storage precision. A band node combines the y (and z) corners of its coarse column, from two
// coarse states after the first fine step (time interpolation) and from one after the second; an
// odd-x node takes the neighbouring column from the next lane. A restricted coarse node reads one
// fine node.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"

namespace lbmib {
namespace {

constexpr int RTPB = 256;

struct RefineGeom {
    int nc[3];          // coarse nodes per axis (x, y, z; 1 past the dimension)
    int nf[3];          // fine nodes per axis
    int org[3];         // coarse node of fine node 0
    int G;              // band width (fine nodes)
    long long Nc, Nf;   // nodes per grid
    long long nband;    // band nodes
    int rlo[3], rn[3];  // restriction: first fine index (even) and number of restricted nodes per axis
    long long nrest;
};

struct RefineGas {
    double mu_c, mu_f;  // viscosities of the two levels (lattice units)
    double inv_Cv;
    double e_ref;       // reference of the stored energy deviation (equal on both levels)
};

__device__ __forceinline__ double taubar_of(double mu, double rho) { return mu * 3.0 / rho + 0.5; }

// Workgroups are dispatched to the eight XCDs in turn (workgroup w on XCD w % 8). Logical block
// (w % 8) * per + w / 8 gives each XCD a contiguous range of items, so that the workgroups reading
// the same coarse (or fine) lines share one L2; -1 for the padding workgroups of the last range.
__device__ __forceinline__ long long xcd_block(long long nblocks) {
    const long long per = (nblocks + 7) / 8;
    const long long w = blockIdx.x;
    const long long lb = (w % 8) * per + w / 8;
    return lb < nblocks ? lb : -1;
}

// Fine coordinates of band node k: in 3D the z slabs first, then, plane by plane, the y rows and the
// x columns of the ring of one plane.
template <int D>
__device__ __forceinline__ void band_node(const RefineGeom& g, long long k, int* x) {
    const int nx = g.nf[0], ny = g.nf[1], nz = g.nf[2], G = g.G;
    x[2] = 0;
    if (D == 3) {
        const long long slab = (long long)2 * G * nx * ny;
        if (k < slab) {
            const int zi = (int)(k / ((long long)nx * ny));
            const long long r = k % ((long long)nx * ny);
            x[2] = zi < G ? zi : nz - 2 * G + zi;
            x[1] = (int)(r / nx);
            x[0] = (int)(r % nx);
            return;
        }
        k -= slab;
        const long long ring = (long long)nx * ny - (long long)(nx - 2 * G) * (ny - 2 * G);
        x[2] = G + (int)(k / ring);
        k %= ring;
    }
    const long long rows = (long long)2 * G * nx;
    if (k < rows) {
        const int yi = (int)(k / nx);
        x[1] = yi < G ? yi : ny - 2 * G + yi;
        x[0] = (int)(k % nx);
        return;
    }
    k -= rows;
    x[1] = G + (int)(k / (2 * G));
    const int c = (int)(k % (2 * G));
    x[0] = c < G ? c : nx - 2 * G + c;
}

// Fine coordinates of item k: every fine node (ALL, x fastest) or the band nodes.
template <int D, bool ALL>
__device__ __forceinline__ void node_of(const RefineGeom& g, long long k, int* x) {
    if (ALL) {
        x[0] = (int)(k % g.nf[0]);
        const long long r = k / g.nf[0];
        x[1] = (int)(r % g.nf[1]);
        x[2] = (int)(r / g.nf[1]);
    } else {
        band_node<D>(g, k, x);
    }
}

// Values of coarse column ix combined over the y (and z) corners of a fine node: for the Q
// populations f~, e and the D - 1 stored history components, sum over corners of w_yz times the
// state (1 - wt) A + wt B (B alone unless TWO). The sums are taken in the storage type (the
// weights 1/2 and 1/4 are exact; FP32 storage keeps the register footprint, and so the number of
// load round trips, half that of FP64 sums).
template <class L, class S, bool TWO>
__device__ __forceinline__ void gather_yz(const RefineGeom& g, const StateP<S>& A, const StateP<S>& B, S wt, int ix,
                                          const int* i0, const S* fr, S* Y) {
    constexpr int D = L::D, Q = L::Q, NV = Q + D;
#pragma unroll
    for (int v = 0; v < NV; ++v) Y[v] = S(0);
    const S wa = S(1) - wt;
#pragma unroll
    for (int cb = 0; cb < (1 << (D - 1)); ++cb) {
        const int by = cb & 1, bz = (cb >> 1) & 1;
        S w = by ? fr[1] : S(1) - fr[1];
        if (D == 3) w *= bz ? fr[2] : S(1) - fr[2];
        if (w == S(0)) continue;   // the same for every node of a row
        const long long n = ix + (long long)g.nc[0] * ((i0[1] + by) + (long long)g.nc[1] * (i0[2] + bz));
        auto at = [&](const S* a, const S* b, long long off) {
            const S vb = b[off];
            return TWO ? wa * a[off] + wt * vb : vb;
        };
#pragma unroll
        for (int i = 0; i < Q; ++i) Y[i] += w * at(A.f, B.f, (long long)i * g.Nc + n);
        Y[Q] += w * at(A.e, B.e, n);
#pragma unroll
        for (int c = 0; c < D - 1; ++c) Y[Q + 1 + c] += w * at(A.h2, B.h2, (long long)c * g.Nc + n);
    }
}

// Populations f~ (deviations), e and h2 interpolated at a fine node from the coarse states
// (1 - wt) A + wt B (multilinear in space), rescaled to the fine level and stored.
// Separable: each lane combines the y/z corners of its own coarse column; an odd-x node takes the
// next column from the next lane when that lane holds the next node of the row (a row's nodes are
// consecutive items), else it gathers that column itself.
template <class L, class S, bool ALL, bool TWO>
__global__ void __launch_bounds__(RTPB) k_refine_prolong(RefineGeom g, RefineGas q, StateP<S> A, StateP<S> B,
                                                         double wt, StateP<S> F) {
    constexpr int D = L::D, Q = L::Q, NV = Q + D;
    const long long total = ALL ? g.Nf : g.nband;
    const long long lb = xcd_block((total + RTPB - 1) / RTPB);
    if (lb < 0) return;
    const long long kk = lb * RTPB + threadIdx.x;
    const bool active = kk < total;
    const long long k = active ? kk : total - 1;   // idle lanes still take part in the shuffle
    int x[3] = {0, 0, 0}, xn[3] = {0, 0, 0};
    node_of<D, ALL>(g, k, x);
    node_of<D, ALL>(g, k + 1 < total ? k + 1 : k, xn);
    const bool next_ok = (threadIdx.x & 63) != 63 && xn[0] == x[0] + 1 && xn[1] == x[1] && xn[2] == x[2];
    int i0[3];
    S fr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        i0[a] = a < D ? g.org[a] + (x[a] >> 1) : 0;
        fr[a] = a < D ? S(0.5) * S(x[a] & 1) : S(0);
    }
    S Ys[NV], Yn[NV];
    gather_yz<L, S, TWO>(g, A, B, S(wt), i0[0], i0, fr, Ys);
#pragma unroll
    for (int v = 0; v < NV; ++v) Yn[v] = __shfl_down(Ys[v], 1, 64);
    if (x[0] & 1) {
        if (!next_ok) gather_yz<L, S, TWO>(g, A, B, S(wt), i0[0] + 1, i0, fr, Yn);
#pragma unroll
        for (int v = 0; v < NV; ++v) Ys[v] = S(0.5) * Ys[v] + S(0.5) * Yn[v];
    }
    if (!active) return;
    double Y[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Y[v] = double(Ys[v]);
    double rho = 1.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += Y[i];
#pragma unroll
        for (int a = 0; a < D; ++a) j[a] += double(L::c[i][a]) * Y[i];
    }
    const double ir = 1.0 / rho;
    double u[3] = {0.0, 0.0, 0.0}, uu = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = j[a] * ir;
        uu += u[a] * u[a];
    }
    const double e = Y[Q];
    const double T = ((e + q.e_ref) * ir - 0.5 * uu) * q.inv_Cv;
    double feq[Q];
    feq_dev<L, double>(rho, u, T, feq);
    const double s = taubar_of(q.mu_f, rho) / (2.0 * taubar_of(q.mu_c, rho));
    const long long nf = x[0] + (long long)g.nf[0] * (x[1] + (long long)g.nf[1] * x[2]);
#pragma unroll
    for (int i = 0; i < Q; ++i) F.f[(long long)i * g.Nf + nf] = S(feq[i] + s * (Y[i] - feq[i]));
    F.e[nf] = S(e);
#pragma unroll
    for (int c = 0; c < D - 1; ++c) F.h2[(long long)c * g.Nf + nf] = S(0.5 * Y[Q + 1 + c]);
}

// Coarse node of restriction item k takes the values of its fine node, rescaled to the coarse level.
template <class L, class S>
__global__ void __launch_bounds__(RTPB) k_refine_restrict(RefineGeom g, RefineGas q, StateP<S> F, StateP<S> C) {
    constexpr int D = L::D, Q = L::Q;
    const long long lb = xcd_block((g.nrest + RTPB - 1) / RTPB);
    if (lb < 0) return;
    const long long k = lb * RTPB + threadIdx.x;
    if (k >= g.nrest) return;
    int xf[3] = {0, 0, 0};
    xf[0] = g.rlo[0] + 2 * (int)(k % g.rn[0]);
    const long long r = k / g.rn[0];
    xf[1] = g.rlo[1] + 2 * (int)(r % g.rn[1]);
    if (D == 3) xf[2] = g.rlo[2] + 2 * (int)(r / g.rn[1]);
    const long long nf = xf[0] + (long long)g.nf[0] * (xf[1] + (long long)g.nf[1] * xf[2]);
    const long long nc = (g.org[0] + (xf[0] >> 1)) +
                         (long long)g.nc[0] * ((g.org[1] + (xf[1] >> 1)) +
                                               (long long)g.nc[1] * (D == 3 ? g.org[2] + (xf[2] >> 1) : 0));
    double fd[Q], rho = 1.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fd[i] = double(F.f[(long long)i * g.Nf + nf]);
        rho += fd[i];
#pragma unroll
        for (int a = 0; a < D; ++a) j[a] += double(L::c[i][a]) * fd[i];
    }
    const double e = double(F.e[nf]);
    const double ir = 1.0 / rho;
    double u[3] = {0.0, 0.0, 0.0}, uu = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = j[a] * ir;
        uu += u[a] * u[a];
    }
    const double T = ((e + q.e_ref) * ir - 0.5 * uu) * q.inv_Cv;
    double feq[Q];
    feq_dev<L, double>(rho, u, T, feq);
    const double s = 2.0 * taubar_of(q.mu_c, rho) / taubar_of(q.mu_f, rho);
#pragma unroll
    for (int i = 0; i < Q; ++i) C.f[(long long)i * g.Nc + nc] = S(feq[i] + s * (fd[i] - feq[i]));
    C.e[nc] = S(e);
#pragma unroll
    for (int c = 0; c < D - 1; ++c) C.h2[(long long)c * g.Nc + nc] = S(2.0 * double(F.h2[(long long)c * g.Nf + nf]));
}

// Workgroups for n items: whole blocks, rounded up to a multiple of the eight XCDs (see xcd_block).
unsigned blocks_of(long long n) { return (unsigned)(((n + RTPB - 1) / RTPB + 7) / 8 * 8); }


thread_local std::string g_refine_error;

}  // namespace
}  // namespace lbmib

using namespace lbmib;

struct lbm_refine {
    lbm_handle* coarse = nullptr;
    lbm_handle* fine = nullptr;
    RefineGeom g{};
    RefineGas q{};
    int margin = 0;
    lbm_refine* child = nullptr;    // coupling of the fine handle with a finer block, or NULL
    lbm_refine* parent = nullptr;   // coupling whose fine handle is this one's coarse handle
    // Two coupled steps (every level returns to its state index) captured as a HIP graph on a
    // private stream, for the key below: coarse state index, then per level its handle, state
    // index and body version (an outermost coupling only).
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<long long> graph_key;
    // The coarse step of a coupled step runs on `side` beside the first fine step; ev_fork and
    // ev_join order it within the coupled step.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::string err;
};

namespace {

int rfail(lbm_refine* r, int code, const std::string& msg) {
    if (r)
        r->err = msg;
    else
        g_refine_error = msg;
    return code;
}

bool close_rel(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::fabs(b); }

// Body requirements of one coupling, which ib_set_markers may change between steps.
int check_bodies_one(lbm_refine* r) {
    const lbm_handle* c = r->coarse;
    const lbm_handle* f = r->fine;
    if (c->markers_set) return rfail(r, LBM_E_INVAL, "the coarse handle holds a body");
    if (f->markers_set) {
        const int* fb = f->fbox;
        const int D = f->D, M = r->margin;
        // fbox: x, y, marching axis (y in 2D, z in 3D)
        const int lo[3] = {fb[0], D == 3 ? fb[2] : fb[4], fb[4]};
        const int hi[3] = {fb[1], D == 3 ? fb[3] : fb[5], fb[5]};
        for (int a = 0; a < D; ++a)
            if (lo[a] < M || hi[a] > r->g.nf[a] - 1 - M)
                return rfail(r, LBM_E_INVAL, "fine body forced nodes closer than margin to the block edge");
    }
    return LBM_OK;
}

// The same for a coupling and every coupling nested inside it.
int check_bodies(lbm_refine* r) {
    if (r->child) {
        if (int rc = check_bodies_one(r)) return rc;
        if (int rc = check_bodies(r->child)) return rfail(r, rc, "inner level: " + r->child->err);
        return LBM_OK;
    }
    return check_bodies_one(r);
}

// One coupled step of r: the coarse step, then two steps of the fine level (each a coupled step
// of the nested coupling if there is one) each followed by its band refill, then the restriction.
int coupled_step(lbm_refine* r) {
    lbm_handle *c = r->coarse, *f = r->fine;
    // The coarse step and the first fine step are independent (the fine step reads the fine state
    // alone, whose band the previous coupled step refilled): the coarse step runs on the side
    // stream beside it, so that the work items of both sweeps share the chip, and the band refill
    // after the first fine step waits for both.
    const hipStream_t main = c->stream;
    hipError_t e = hipEventRecord(r->ev_fork, main);
    if (e == hipSuccess) e = hipStreamWaitEvent(r->side, r->ev_fork, 0);
    if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("coarse step fork: ") + hipGetErrorString(e));
    c->stream = r->side;
    const int crc = step_handle(c, 1, false);
    c->stream = main;
    if (crc) return rfail(r, crc, std::string("coarse step: ") + c->err);
    e = hipEventRecord(r->ev_join, r->side);
    if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("coarse step join: ") + hipGetErrorString(e));
    for (int k = 1; k <= 2; ++k) {
        if (r->child) {
            if (int rc = coupled_step(r->child)) return rfail(r, rc, "inner level: " + r->child->err);
        } else if (int rc = step_handle(f, 1, false)) {
            return rfail(r, rc, std::string("fine step: ") + f->err);
        }
        if (k == 1) {
            e = hipStreamWaitEvent(main, r->ev_join, 0);
            if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("coarse step join: ") + hipGetErrorString(e));
        }
        // coarse: the previous state is the one before this coupled step, the current one after it
        e = dispatch(c, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            // at k = 2 the band takes the coarse state after the step alone
            if (r->g.nband > 0 && k == 1)
                hipLaunchKernelGGL((k_refine_prolong<LT, ST, false, true>), dim3(blocks_of(r->g.nband)), dim3(RTPB), 0,
                                   c->stream, r->g, r->q, other<ST>(c), current<ST>(c), 0.5, current<ST>(f));
            else if (r->g.nband > 0)
                hipLaunchKernelGGL((k_refine_prolong<LT, ST, false, false>), dim3(blocks_of(r->g.nband)), dim3(RTPB),
                                   0, c->stream, r->g, r->q, other<ST>(c), current<ST>(c), 1.0, current<ST>(f));
            return hipGetLastError();
        });
        if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("refine band: ") + hipGetErrorString(e));
    }
    e = dispatch(c, [&](auto L, auto S) {
        using LT = decltype(L);
        using ST = decltype(S);
        if (r->g.nrest > 0)
            hipLaunchKernelGGL((k_refine_restrict<LT, ST>), dim3(blocks_of(r->g.nrest)), dim3(RTPB), 0, c->stream,
                               r->g, r->q, current<ST>(f), current<ST>(c));
        return hipGetLastError();
    });
    if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("refine restrict: ") + hipGetErrorString(e));
    return LBM_OK;
}

// Every handle of the nest, coarsest first.
std::vector<lbm_handle*> nest_handles(lbm_refine* r) {
    std::vector<lbm_handle*> hs{r->coarse};
    for (lbm_refine* p = r; p; p = p->child) hs.push_back(p->fine);
    return hs;
}

std::vector<long long> nest_key(lbm_refine* r) {
    std::vector<long long> k;
    for (lbm_handle* h : nest_handles(r)) {
        k.push_back(reinterpret_cast<long long>(h));
        k.push_back(h->cur);
        k.push_back(h->geom_version);
    }
    return k;
}

// Capture (once per key) two coupled steps from the current states. Nothing runs during the
// capture, and every level's state index ends where it started.
int ensure_nest_graph(lbm_refine* r) {
    const std::vector<long long> key = nest_key(r);
    if (r->graph_exec && r->graph_key == key) return LBM_OK;
    if (r->graph_exec) {
        hipGraphExecDestroy(r->graph_exec);
        r->graph_exec = nullptr;
    }
    if (!r->cap_stream) {
        const hipError_t e = hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("graph stream: ") + hipGetErrorString(e));
    }
    const std::vector<lbm_handle*> hs = nest_handles(r);
    std::vector<int> cur0, stepped, any;
    for (lbm_handle* h : hs) {
        cur0.push_back(h->cur);
        stepped.push_back(h->stepped);
        any.push_back(h->any_step);
    }
    hipStream_t user = r->coarse->stream;
    hipError_t e = hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    for (lbm_handle* h : hs) h->stream = r->cap_stream;
    int rc = coupled_step(r);
    if (rc == LBM_OK) rc = coupled_step(r);
    for (lbm_handle* h : hs) h->stream = user;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(r->cap_stream, &g);
    for (size_t i = 0; i < hs.size(); ++i) {
        hs[i]->stepped = stepped[i];
        hs[i]->any_step = any[i];
        if (hs[i]->cur != cur0[i]) {   // a failed capture may stop part way
            hs[i]->cur = cur0[i];
            refresh_handle_args(hs[i]);
        }
    }
    if (rc != LBM_OK || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return rc != LBM_OK ? rc : rfail(r, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&r->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        r->graph_exec = nullptr;
        return rfail(r, LBM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    r->graph_key = key;
    return LBM_OK;
}

// Calls of at least this many coupled steps replay the two-step graph.
constexpr int kNestGraphMinSteps = 3;

}  // namespace

extern "C" {

int lbm_refine_create(lbm_handle* coarse, lbm_handle* fine, const int* origin, int band, int margin,
                      lbm_refine** out) {
    if (!out) return rfail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!coarse || !fine || !origin || coarse == fine) return rfail(nullptr, LBM_E_INVAL, "bad handles or origin");
    const lbm_params &pc = coarse->p, &pf = fine->p;
    const int D = pc.dim;
    if (pf.dim != D) return rfail(nullptr, LBM_E_INVAL, "handles of different dimensions");
    if (pf.precision != pc.precision) return rfail(nullptr, LBM_E_INVAL, "handles of different precisions");
    if (coarse->device != fine->device || coarse->stream != fine->stream)
        return rfail(nullptr, LBM_E_INVAL, "handles on different devices or streams");
    bool same = pf.gamma == pc.gamma && pf.sigma == pc.sigma && pf.rho_inf == pc.rho_inf && pf.T_inf == pc.T_inf &&
                pf.with_aC == pc.with_aC;
    for (int a = 0; a < 3; ++a) same = same && pf.u_inf[a] == pc.u_inf[a];
    if (!same) return rfail(nullptr, LBM_E_INVAL, "gas or free-stream parameters differ between the levels");
    if (!close_rel(pf.mu, 2.0 * pc.mu) || !close_rel(pf.lambda_, 2.0 * pc.lambda_))
        return rfail(nullptr, LBM_E_INVAL, "fine mu and lambda_ must be twice the coarse ones");
    if (pf.bc_x != LBM_BC_PERIODIC) return rfail(nullptr, LBM_E_INVAL, "the fine handle must be periodic");
    if (band < 2 || margin < band) return rfail(nullptr, LBM_E_INVAL, "need 2 <= band <= margin");
    const int nc[3] = {pc.nx, pc.ny, pc.nz}, nf[3] = {pf.nx, pf.ny, pf.nz};
    RefineGeom g{};
    g.G = band;
    for (int a = 0; a < 3; ++a) {
        g.nc[a] = nc[a];
        g.nf[a] = nf[a];
        g.org[a] = a < D ? origin[a] : 0;
        g.rlo[a] = 0;
        g.rn[a] = 1;
    }
    g.Nc = coarse->N;
    g.Nf = fine->N;
    long long inner = 1;
    g.nrest = 1;
    for (int a = 0; a < D; ++a) {
        if (nf[a] % 2 != 0 || nf[a] <= 2 * band)
            return rfail(nullptr, LBM_E_INVAL, "fine node counts must be even and exceed twice the band");
        if (g.org[a] < 0 || g.org[a] + nf[a] / 2 > nc[a] - 1)
            return rfail(nullptr, LBM_E_INVAL, "block outside the coarse grid");
        inner *= nf[a] - 2 * band;
        // even fine indices in [margin, nf - 1 - margin]
        const int lo = (margin + 1) & ~1, hi = nf[a] - 1 - margin;
        g.rlo[a] = lo;
        g.rn[a] = hi >= lo ? (hi - lo) / 2 + 1 : 0;
        g.nrest *= g.rn[a];
    }
    if (pc.bc_x != LBM_BC_PERIODIC && (g.org[0] < 2 || g.org[0] + nf[0] / 2 > nc[0] - 3))
        return rfail(nullptr, LBM_E_INVAL, "block overlaps the inflow or outflow columns");
    g.nband = g.Nf - inner;
    RefineGas q{};
    q.mu_c = pc.mu;
    q.mu_f = pf.mu;
    q.inv_Cv = (pc.gamma - 1.0) * 3.0;
    q.e_ref = coarse->args.fs.e_ref;
    if (fine->args.fs.e_ref != q.e_ref) return rfail(nullptr, LBM_E_INVAL, "energy references differ");
    lbm_refine* r = new (std::nothrow) lbm_refine();
    if (!r) return rfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    hipError_t se = hipStreamCreateWithFlags(&r->side, hipStreamNonBlocking);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&r->ev_join, hipEventDisableTiming);
    if (se != hipSuccess) {
        lbm_refine_destroy(r);
        return rfail(nullptr, LBM_E_HIP, std::string("side stream: ") + hipGetErrorString(se));
    }
    r->coarse = coarse;
    r->fine = fine;
    r->g = g;
    r->q = q;
    r->margin = margin;
    *out = r;
    return LBM_OK;
}

int lbm_refine_prolong(lbm_refine* r) {
    if (!r) return LBM_E_INVAL;
    lbm_handle *c = r->coarse, *f = r->fine;
    hipError_t e = dispatch(c, [&](auto L, auto S) {
        using LT = decltype(L);
        using ST = decltype(S);
        hipLaunchKernelGGL((k_refine_prolong<LT, ST, true, false>), dim3(blocks_of(r->g.Nf)), dim3(RTPB), 0,
                           c->stream, r->g, r->q, current<ST>(c), current<ST>(c), 1.0, current<ST>(f));
        return hipGetLastError();
    });
    if (e == hipSuccess && !f->geom.rows.empty()) {
        const size_t nb = f->geom.rows.size() * (f->D == 3 ? 3 : 1) * 8;
        e = hipMemsetAsync(f->d.h2off, 0, nb, f->stream);
        if (e == hipSuccess) e = hipMemsetAsync(f->d.h2off2, 0, nb, f->stream);
    }
    if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("refine prolong: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_refine_step(lbm_refine* r, int n) {
    if (!r) return LBM_E_INVAL;
    if (n < 0) return rfail(r, LBM_E_INVAL, "n < 0");
    if (r->parent) return rfail(r, LBM_E_INVAL, "a nested coupling is stepped through its outer coupling");
    if (int rc = check_bodies(r)) return rc;
    if (n == 0) return LBM_OK;
    int m = n - 1;                  // coupled steps before the last one
    if (n >= kNestGraphMinSteps) {
        // pairs replay the captured graph; an odd step and the last one run directly
        if (m % 2) {
            if (int rc = coupled_step(r)) return rc;
            --m;
        }
        if (int rc = ensure_nest_graph(r)) return rc;
        for (int i = 0; i < m / 2; ++i) {
            const hipError_t e = hipGraphLaunch(r->graph_exec, r->coarse->stream);
            if (e != hipSuccess) return rfail(r, LBM_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
        }
        for (lbm_handle* h : nest_handles(r)) h->stepped = h->any_step = 1;
    } else {
        for (int s = 0; s < m; ++s)
            if (int rc = coupled_step(r)) return rc;
    }
    if (int rc = coupled_step(r)) return rc;
    if (int rc = residual_handle(r->coarse)) return rfail(r, rc, std::string("coarse residual: ") + r->coarse->err);
    return LBM_OK;
}

int lbm_refine_nest(lbm_refine* outer, lbm_refine* inner) {
    if (!outer || !inner || outer == inner) return LBM_E_INVAL;
    if (inner->coarse != outer->fine)
        return rfail(outer, LBM_E_INVAL, "the inner coupling's coarse handle is not the outer one's fine handle");
    if (outer->child || inner->parent) return rfail(outer, LBM_E_INVAL, "already nested");
    for (const lbm_refine* p = outer; p; p = p->parent)
        if (p == inner) return rfail(outer, LBM_E_INVAL, "nesting would form a cycle");
    // the inner block and the coarse nodes its band reads stay clear of the middle level's band,
    // which holds wrapped values until the outer coupling refills it
    const RefineGeom &go = outer->g, &gi = inner->g;
    const int D = outer->fine->D;
    for (int a = 0; a < D; ++a)
        if (gi.org[a] < go.G || gi.org[a] + gi.nf[a] / 2 > go.nf[a] - 1 - go.G)
            return rfail(outer, LBM_E_INVAL, "inner block within the band of the middle level");
    outer->child = inner;
    inner->parent = outer;
    return LBM_OK;
}

void lbm_refine_destroy(lbm_refine* r) {
    if (!r) return;
    if (r->parent) {
        r->parent->child = nullptr;
        if (r->parent->graph_exec) {          // its graph stepped this coupling
            hipGraphExecDestroy(r->parent->graph_exec);
            r->parent->graph_exec = nullptr;
        }
    }
    if (r->child) r->child->parent = nullptr;
    if (r->graph_exec) hipGraphExecDestroy(r->graph_exec);
    if (r->cap_stream) hipStreamDestroy(r->cap_stream);
    if (r->side) hipStreamDestroy(r->side);
    if (r->ev_fork) hipEventDestroy(r->ev_fork);
    if (r->ev_join) hipEventDestroy(r->ev_join);
    delete r;
}

const char* lbm_refine_last_error(lbm_refine* r) { return r ? r->err.c_str() : g_refine_error.c_str(); }

}  // extern "C"
