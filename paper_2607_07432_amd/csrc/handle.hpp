// Host-side handle of one grid, shared by the single-grid API and the batch API.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbmib.h"
#include "kernels.hpp"
#include "precompute.hpp"

namespace lbmib {

// Device arrays carved out of the caller's workspace.
struct Dev {
    // state (storage precision), ping-pong
    void *fA, *eA, *hA, *fB, *eB, *hB;
    void* work;     // M [(D+2) N] followed by fcol [Q N], compute precision
    int* rowmap;
    double* partials;
    double* resid;  // [2]
    double* loads;  // [16]
    int* flag;
    // markers
    long long *supp_ptr, *supp_node, *proj_ptr, *proj_node, *tw_ptr, *tw_node;
    double *supp_w, *proj_w, *tw_w, *phi, *dbv, *W, *u_wall, *t_value, *G, *diag, *eps;
    double *Xm, *nm;   // marker positions and outward normals [m][D]
    int* t_kind;
    long long *rows, *row_ptr, *col_marker;
    double *col_s, *fib, *fE, *h2off, *h2off2;   // sparse history, ping-pong with the state
};

}  // namespace lbmib

struct lbm_handle {
    lbm_params p;
    int D = 0, Q = 0;
    long long N = 0;
    hipStream_t stream = nullptr;
    int device = -1;       // HIP device current at lbm_init_grid
    lbmib::Dev d{};
    int cur = 0;           // 0: state A is current, 1: state B
    lbmib::SweepArgs args{};
    lbmib::MarkersP mk{};
    lbmib::Geometry geom;
    std::vector<double> host_stage;
    int method = 0;
    int chunk = 0;         // planes per work item of the fused sweep (set by lbm_init_grid)
    int markers_set = 0;
    int stepped = 0;       // a step has run since the body was set
    int any_step = 0;
    int geom_version = 0;  // incremented by every ib_set_markers
    // Bounding box of the forced nodes {x min, x max, y min, y max, marching-axis min, max}
    // (y unused in 2D, where the marching axis is y); empty when min > max. Fused-sweep tiles whose
    // footprint misses it run without the forcing path.
    int fbox[6] = {1, 0, 1, 0, 1, 0};
    // Two steps without the residual, captured as a HIP graph from state index graph_cur for body
    // version graph_geom on a private stream, replayed on `stream` by long lbm_step calls.
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    int graph_cur = -1, graph_geom = -1;
    std::string err;
};

namespace lbmib {

template <class S>
StateP<S> stateA(lbm_handle* h) {
    return {(S*)h->d.fA, (S*)h->d.eA, (S*)h->d.hA};
}
template <class S>
StateP<S> stateB(lbm_handle* h) {
    return {(S*)h->d.fB, (S*)h->d.eB, (S*)h->d.hB};
}

// The current state (the last step's output) and the other one (its input).
template <class S>
StateP<S> current(lbm_handle* h) {
    return h->cur == 0 ? stateA<S>(h) : stateB<S>(h);
}
template <class S>
StateP<S> other(lbm_handle* h) {
    return h->cur == 0 ? stateB<S>(h) : stateA<S>(h);
}

// Call f(lattice tag, storage type tag) for the handle's lattice and precision.
template <class F>
hipError_t dispatch(lbm_handle* h, F&& f) {
    if (h->D == 2) {
        if (h->p.precision == LBM_F64) return f(D2Q9{}, double{});
        return f(D2Q9{}, float{});
    }
    if (h->p.precision == LBM_F64) return f(D3Q19{}, double{});
    return f(D3Q19{}, float{});
}

// Recompute the kernel argument blocks of a handle from its current state index and body.
void refresh_handle_args(lbm_handle* h);

// n steps of one handle as lbm_step; the last one forms the residual only if want_resid.
int step_handle(lbm_handle* h, int n, bool want_resid);

// The residual between the previous and the current state (as lbm_residual reports it), enqueued.
int residual_handle(lbm_handle* h);

}  // namespace lbmib
