// Launch interface between the C ABI (api.hip) and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "node_math.hpp"

namespace lbmib {

struct GridP {
    int nx, ny, nz;
    long long N;
    int bc_x;           // 0 periodic; 1 inflow/outflow closure along x; 2 the same inlet with the
                        // characteristic outlet (the sweep leaves columns nx-2, nx-1 to it)
};

// Ping-pong state (storage type S): f~[Q][N] (f - w), e[N] (rho E - e_ref), h2[D-1][N]
// (diagonal of the deviatoric force history; the last diagonal entry is minus the sum).
template <class S>
struct StateP {
    S* f;
    S* e;
    S* h2;
};

// Sparse data of the forced nodes (CSR rows), FP64.
struct RowsP {
    int nrows;
    const int* rowmap;      // [N] row index of a node, -1 if not forced
    const long long* rows;  // [nrows] node of each row
    double* fib;            // [D][nrows] momentum forcing
    double* fE;             // [nrows] energy forcing w + q
    const double* h2off;    // [NOFF][nrows] off-diagonal force history (xy[, xz, yz]), current step
    double* h2off_out;      // the same for the next step (ping-pong with h2off)
};

struct FreeStream {
    double fdev[19];        // f^eq_i - w_i at (rho_inf, u_inf, T_inf)
    double e_ref;           // rho_inf (|u_inf|^2/2 + Cv T_inf): reference of the energy deviation
    double eint_inf;        // rho_inf Cv T_inf: internal energy density, proportional to p_inf
    double rho_inf, u_inf[3], T_inf;
};

struct SweepArgs {
    GridP grid;
    Gas gas;
    FreeStream fs;
    RowsP rows;
};

// Marker data (FP64) uploaded by ib_set_markers.
struct MarkersP {
    int m, dim, method;
    const long long *supp_ptr, *supp_node;
    const double* supp_w;
    const long long *proj_ptr, *proj_node;
    const double* proj_w;
    const long long *tw_ptr, *tw_node;
    const double* tw_w;
    const double *phi, *dbv, *W;
    const double *u_wall, *t_value;
    const int* t_kind;
    const long long *row_ptr, *col_marker;
    const double* col_s;
    double* G;              // [m][D+2]: F (D), W^IB, Q^IB of the last step
    double* diag;           // [m][8]: rho*, T*, TP, uP (D), Tt  (last step)
    double* eps;            // [m][4]: eps_dir, eps_neu, eps_iso, kind mask
};

// Arguments of the fused sweep in its arithmetic type C (no conversions inside the kernel).
template <class C>
struct FusedK {
    int nx, ny, nz, bc_x;
    long long N;
    GasT<C> gas;
    C e_ref;
    C eint_inf;
    C fdev[19];
    RowsP rows;
};

template <class C>
inline FusedK<C> fused_args(const SweepArgs& a) {
    FusedK<C> k;
    k.nx = a.grid.nx;
    k.ny = a.grid.ny;
    k.nz = a.grid.nz;
    k.bc_x = a.grid.bc_x;
    k.N = a.grid.N;
    k.gas = gas_as<C>(a.gas);
    k.e_ref = C(a.fs.e_ref);
    k.eint_inf = C(a.fs.eint_inf);
    for (int i = 0; i < 19; ++i) k.fdev[i] = C(a.fs.fdev[i]);
    k.rows = a.rows;
    return k;
}

// One case of a batch of independent 2D grids (an entry of a device table). Index k of a[] and
// st[] belongs to the step parity at which state k is the current one; at batch step parity g
// the current state is (cur0 + g) & 1.
template <class S>
struct CaseDesc {
    SweepArgs a[2];         // a[k].rows.h2off / h2off_out: the history buffers when state k is current
    FusedK<S> k[2];         // the same for the fused sweep
    StateP<S> st[2];        // state A, state B of the case
    MarkersP mk;
    int cur0;               // current state at batch parity 0
    int tiles_x, chunk, small;
    int item0;              // first sweep work item of the case (items: tiles_x per chunk of rows)
    int fb[6];              // bounding box of the case's forced nodes (lbm_handle::fbox)
    int marker0, row0;      // first marker and first CSR row of the case in the batch numbering
    int part0, nparts, part_len;   // residual partial sums: first, count, nodes per partial
    double resid_scale;     // 1 / (|u_inf| sqrt(N))
    double* resid;          // [2] residual and non-finite flag of the case
};

// Split sweep (macros -> collide -> stream + fluxes + energy).
template <class L, class S, class C>
hipError_t launch_split_step(const SweepArgs& a, StateP<S> A, StateP<S> B, C* M, C* fcol, hipStream_t st);

// fbox: bounding box of the forced nodes (see lbm_handle::fbox). With rpart (capacity rcap
// pairs) the sweep also writes the step's residual partials, one (sum, non-finite flag) pair per
// workgroup, and sets *rparts to their count; *rparts = 0 when this grid cannot (run k_residual).
template <class L, class S>
hipError_t launch_fused_step(const SweepArgs& a, StateP<S> A, StateP<S> B, int chunk, const int* fbox,
                             hipStream_t st, double* rpart = nullptr, int rcap = 0, int* rparts = nullptr);

// Planes per work item of the fused sweep on this grid for a device of `cus` compute units
// (chosen from the number of work items each length gives against the workgroups the chip holds).
template <class L, class S>
int fused_auto_chunk(const GridP& g, int cus);

template <class L, class S>
hipError_t launch_init_state(const SweepArgs& a, StateP<S> A, hipStream_t st);
template <class L, class S>
hipError_t launch_set_fields(const SweepArgs& a, StateP<S> A, const double* rho, const double* u,
                             const double* T, hipStream_t st);
template <class L, class S, class O>
hipError_t launch_fields(const SweepArgs& a, StateP<S> A, O* rho, O* u, O* T, O* p, hipStream_t st);
template <class L, class S>
hipError_t launch_export(const SweepArgs& a, StateP<S> A, int comp, double* out, hipStream_t st);
template <class L, class S>
hipError_t launch_import(const SweepArgs& a, StateP<S> A, int comp, const double* in, int* bad, hipStream_t st);
template <class L, class S>
hipError_t launch_residual(const SweepArgs& a, StateP<S> Old, StateP<S> New, double* partials, int nparts,
                           double* out, hipStream_t st);
// Characteristic outlet (outlet.hip): columns nx-2, nx-1 of New from the LODI relations on Old.
template <class L, class S>
hipError_t launch_outlet_char(const SweepArgs& a, StateP<S> Old, StateP<S> New, double sigma_c, hipStream_t st);
// The final reduction alone, over nparts partial pairs written by a sweep.
template <class L>
hipError_t launch_residual_final(const SweepArgs& a, const double* partials, int nparts, double* out, hipStream_t st);

// Immersed boundary.
template <class L, class S>
hipError_t launch_markers(const SweepArgs& a, const MarkersP& mk, StateP<S> A, hipStream_t st);
hipError_t launch_spread(int dim, const MarkersP& mk, RowsP rows, hipStream_t st);
template <class L, class S>
hipError_t launch_eps(const SweepArgs& a, const MarkersP& mk, StateP<S> A, double u_ref, double T_inf,
                      double ref_len, hipStream_t st);
hipError_t launch_loads(int dim, const MarkersP& mk, double* out, hipStream_t st);
hipError_t launch_rowmap(const long long* rows, int nrows, int* rowmap, hipStream_t st);

int residual_parts(long long N);
// Capacity of the residual partials buffer, in (sum, flag) pairs: k_residual uses at most 1024,
// a fused sweep one per workgroup.
constexpr int RESID_PARTS_MAX = 8192;

// Batch of 2D grids. Sweep tile widths: 62, 126 or 254 nodes (64, 128, 256 threads).
template <class L, class S>
hipError_t launch_fused_batch(const CaseDesc<S>* cases, int ncases, int total_items, int tx, int grid, int g,
                              hipStream_t st);
template <class L, class S>
int fused_batch_occupancy(int tx);   // resident workgroups per CU, 0 if tx is not a batch tile width
template <class L, class S>
hipError_t launch_markers_batch(const CaseDesc<S>* cases, int ncases, int total_markers, int g, hipStream_t st);
template <class S>
hipError_t launch_spread_batch(const CaseDesc<S>* cases, int ncases, int total_rows, int dim, hipStream_t st);
template <class L, class S>
hipError_t launch_residual_batch(const CaseDesc<S>* cases, int ncases, int total_parts, double* partials, int g,
                                 hipStream_t st);

}  // namespace lbmib
