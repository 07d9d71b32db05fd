/*
 * lbmib.h -- C ABI of the MI355X (gfx950) FODIBM-R + hybrid lattice Boltzmann library.
 *
 * One time step (Sec. 2.5 of Mao, Zhao, Boivin, Favier, arXiv 2607.07432):
 *   1. predicted density, momentum, velocity and temperature at the Lagrangian
 *      markers by one-sided interpolation over the interior nodes (Eq. (14));
 *   2. velocity and temperature at the projection points by two-sided
 *      interpolation with the d = 1 kernel (Eq. (12));
 *   3. Lagrangian forces with the reconstructed targets (Eqs. (27), (29)-(32))
 *      or the plain targets (Eqs. (20)-(22));
 *   4. one-sided spreading (Eq. (15)) through a node -> marker CSR;
 *   5. the hybrid LBM collide-and-stream (Eq. (6)) with the MUSCL-Hancock
 *      total-energy update (Eqs. (10)-(11), Appendix A).
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, R = c_s^2 = 1/3, temperatures in units of T_ref.
 *   - Return value 0 (LBM_OK) on success, a negative LBM_E_* code otherwise;
 *     lbm_last_error() gives a message. Nothing throws across this boundary.
 *   - Fields are structure-of-arrays over nodes, node = x + nx*(y + ny*z) (x fastest).
 *   - Every call is ordered on the HIP stream given to lbm_init_grid. A handle is
 *     bound to one stream and one device and is not thread-safe.
 *   - The device workspace is owned by the caller (it must outlive the handle);
 *     the library never allocates device memory. Host arrays passed in are copied.
 */
#ifndef LBMIB_H
#define LBMIB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,      /* invalid argument or parameter */
    LBM_E_NOMEM = -2,      /* workspace too small for the request */
    LBM_E_HIP = -3,        /* a HIP runtime call failed */
    LBM_E_STATE = -4,      /* call not valid in the current state (e.g. loads before a step) */
    LBM_E_NONFINITE = -5   /* a non-finite value was detected by the step check */
};

enum { LBM_BC_PERIODIC = 0, LBM_BC_INFLOW_OUTFLOW = 1, LBM_BC_CHARACTERISTIC = 2 };
enum { LBM_IB_DIBM = 0, LBM_IB_FODIBM = 1, LBM_IB_FODIBM_R = 2 };
enum { LBM_KERNEL_COS = 0, LBM_KERNEL_ROMA3 = 1 };
enum { LBM_T_NONE = 0, LBM_T_DIRICHLET = 1, LBM_T_NEUMANN = 2 };
enum { LBM_F32 = 32, LBM_F64 = 64 };
enum { LBM_SWEEP_FUSED = 0, LBM_SWEEP_THREE_PASS = 1 };

/* Problem parameters (lattice units). Sec. 2.1 (gas), Sec. 2.2 (solver), Sec. 3.4 (gamma). */
typedef struct lbm_params {
    int dim;            /* 2 (D2Q9) or 3 (D3Q19, Appendix A) */
    int nx, ny, nz;     /* grid size: nx >= 5, ny >= 2, nz >= 2 in 3D and nz = 1 in 2D */
    int precision;      /* LBM_F32 or LBM_F64: storage and arithmetic of the sweep */
    int bc_x;           /* LBM_BC_PERIODIC, LBM_BC_INFLOW_OUTFLOW or LBM_BC_CHARACTERISTIC
                           along x (y, z periodic). Inflow/outflow: columns 0, 1 are reset to the
                           free stream every step; columns nx-2, nx-1 take column nx-3 scaled
                           by p_inf / p (populations and rho E; history copied), i.e. pressure
                           held at p_inf, zero gradient of u and T. Characteristic: the same
                           inlet; columns nx-2, nx-1 advance by the locally one-dimensional
                           characteristic relations (Sec. 2.4 names Poinsot and Lele's
                           conditions for the far field), outgoing waves leaving freely and the
                           incoming one relaxed to p_inf with sigma_c; populations are the
                           equilibrium of Eq. (A.3) at the new fields plus the non-equilibrium
                           part of column nx-3. Batches take the first two only. */
    int kernel;         /* marker kernel: LBM_KERNEL_COS (Eq. (19), d = 2) or LBM_KERNEL_ROMA3 */
    int max_markers;    /* marker capacity reserved in the workspace */
    int with_aC;        /* 1: lattice third-order correction a^C in Eq. (A.9); 0: a^C = 0 */
    int sweep;          /* LBM_SWEEP_FUSED (single pass, default) or LBM_SWEEP_THREE_PASS */
    double gamma;       /* ratio of specific heats */
    double mu;          /* dynamic viscosity (constant) */
    double lambda_;     /* thermal conductivity */
    double sigma;       /* HRR weight of Eq. (A.7) (0.98 in the paper) */
    double rho_inf;     /* free stream density */
    double u_inf[3];    /* free stream velocity */
    double T_inf;       /* free stream temperature (units of T_ref) */
    double ref_len;     /* reference length for Re, Cd and Nu */
    double ref_area;    /* reference area for Cd, Cl (a length in 2D) */
    double surface;     /* wetted surface for Nu (a perimeter in 2D) */
    double T_wall;      /* wall temperature used in Nu */
    double sigma_c;     /* characteristic outlet: relaxation of the incoming wave,
                           L1 = sigma_c (1 - Ma^2) c / nx (p - p_inf); 0 = non-reflecting
                           (0.25 is usual); finite and >= 0; unused by the other closures */
} lbm_params;

/* Loads of the last step (FP64). F = -sum_l F_l W_l (force on the body), Q_heat = sum_l Q_l W_l,
 * Cd = F_x / (rho u^2 A / 2), Cl = F_y / (rho u^2 A / 2), Nu = Q_heat L / (lambda (T_w - T_inf) S).
 * eps_* are the mean boundary-condition errors of Eqs. (35), (36), (38) over active markers,
 * with the "s" values interpolated two-sidedly (Eq. (12), d = 2) from the current fields. */
typedef struct lbm_loads {
    double F[3];
    double Q_heat;
    double Cd, Cl, Nu;
    double eps_dir, eps_neu, eps_iso;
    int n_inactive;     /* markers whose interior support is empty (phi = 0) */
    int n_markers;
} lbm_loads;

typedef struct lbm_handle lbm_handle;

/* Device workspace bytes the library needs for p (0 if p is invalid). Pure function. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a handle on the current HIP device. dev_workspace: caller-owned device memory of at
 * least lbm_workspace_bytes(p) bytes, 256-byte aligned. hip_stream: a hipStream_t (NULL = the
 * default stream). The state is set to the free-stream equilibrium f = f^eq(rho_inf, u_inf, T_inf)
 * (Eq. (A.3)), rho E = rho_inf (|u_inf|^2/2 + Cv T_inf), zero force history. The fused sweep's
 * planes per work item are chosen here for the grid and the device's compute units; the
 * environment variable LBMIB_FUSED_CHUNK, if set to a positive integer, overrides the choice.
 * Errors: LBM_E_INVAL (dim, sizes, tau-bar <= 1/2, rest population of Eq. (A.3) negative at
 * T_inf, non-finite values), LBM_E_NOMEM (bytes too small), LBM_E_HIP. */
int lbm_init_grid(const lbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                  lbm_handle** out);

/* Immersed body: m markers with positions X[m*dim] and outward unit normals normal[m*dim]
 * (host, row-major per marker). area_w (nullable) is the input weight dq dr ds of Eq. (13),
 * unused by the one-sided methods. u_wall[m*dim] is the wall velocity u^Bt, t_kind[m] one of
 * LBM_T_*, t_value[m] the wall temperature (Dirichlet) or dT/dn (Neumann). method: LBM_IB_*.
 * Runs the per-geometry precompute on the host in FP64 (supports, interior set, phi of Eq. (16),
 * X* of Eq. (25), d_BV, projection points, W of Eq. (17), node -> marker CSR) and uploads it.
 * Replaces any previous body and clears the force history held at forced nodes.
 * Errors: LBM_E_INVAL (non-finite input, |n| != 1 within 1e-12, a marker within 4 cells of an
 * x boundary under the inflow/outflow or characteristic closure or within 3 cells of any edge, m > max_markers),
 * LBM_E_NOMEM (precomputed lists exceed the workspace), LBM_E_HIP. m = 0 removes the body. */
int ib_set_markers(lbm_handle* h, int m, const double* X, const double* normal,
                   const double* area_w, const double* u_wall, const int* t_kind,
                   const double* t_value, int method);

/* Enqueue n time steps on the handle's stream (Sec. 2.5). Asynchronous; the last step also
 * accumulates the FP64 velocity residual r = ||u^{n+1} - u^n|| / (|u_inf| sqrt(N)) over the
 * stored states and a non-finite check (read with lbm_residual): inside the fused sweep, or by a
 * separate pass for the three-pass sweep and the characteristic outlet. Calls of 5 or more steps
 * replay pairs of steps as a HIP graph, captured on the first such call and again after
 * ib_set_markers (results equal to stepping one at a time). Errors: LBM_E_INVAL (n < 0),
 * LBM_E_HIP. */
int lbm_step(lbm_handle* h, int n);

/* As lbm_step, and also times the launches of every step with HIP events recorded on the
 * handle's stream: kernel_ms[0] = marker interpolation + forces, kernel_ms[1] = spreading,
 * kernel_ms[2] = the grid sweep (collision, streaming, fluxes, energy update), each the
 * average per step in milliseconds. Synchronises. Errors: LBM_E_INVAL (n <= 0), LBM_E_HIP. */
int lbm_step_timed(lbm_handle* h, int n, double* kernel_ms);

/* Loads of the last step (see lbm_loads). Synchronises the stream.
 * Errors: LBM_E_STATE (no body or no step taken since the body was set), LBM_E_HIP. */
int ib_wall_loads(lbm_handle* h, lbm_loads* out);

/* Marker capacity of ib_wall_loads_noalloc's static scratch (32 bytes per marker, 2 MiB per GPU). */
#define LBM_NOALLOC_MAX_MARKERS 65536

/* For callers that cannot allocate device memory or use a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): ib_wall_loads with its
 * per-marker boundary-error buffer and its reduced-loads buffer taken from a static device array
 * of the library instead of the handle's workspace. Same inputs, outputs, results and errors as
 * ib_wall_loads, plus LBM_E_INVAL when the body has more than LBM_NOALLOC_MAX_MARKERS markers and
 * LBM_E_HIP when the array's device address could not be resolved at lbm_init_grid. Calls no
 * allocating routine. The array is one per GPU and holds the last call's contents until the
 * process ends; every call rewrites what it reads. Calls that overlap on one GPU (from several
 * threads or streams, any handles) race on the array and must be serialised by the caller.
 * Synchronises the handle's stream. */
int ib_wall_loads_noalloc(lbm_handle* h, lbm_loads* out);

/* Fields of the current state: rho = sum f, u = sum c f / rho (force-free), T from
 * rho E = rho (|u|^2/2 + Cv T), p = rho R T. dtype LBM_F32 or LBM_F64; on_device = 1 for device
 * pointers (stream-ordered), 0 for host pointers (the call synchronises). u has dim components
 * stored as u[a*N + node]. Any pointer may be NULL. Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_fields(lbm_handle* h, int dtype, int on_device, void* rho, void* u, void* T, void* p);

/* Set the state to the equilibrium of given FP64 fields rho[N], u[dim*N], T[N] (host or device),
 * with zero force history (a warm or cold start). Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_set_fields(lbm_handle* h, int on_device, const double* rho, const double* u,
                   const double* T);

/* Canonical FP64 state (host arrays): f[Q*N] (populations f-bar, population-major), rhoE[N],
 * H2[dim*dim*N] (the deviatoric sum_i (c c - delta c^2/D) F_i of the previous step, tensor
 * component (a,b) at H2[(a*dim+b)*N + node]). set: off-diagonal H2 must vanish away from the
 * forced nodes of the current body. Both synchronise. Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_get_state(lbm_handle* h, double* f, double* rhoE, double* H2);
int lbm_set_state(lbm_handle* h, const double* f, const double* rhoE, const double* H2);

/* FP64 residual and non-finite flag of the last step of the last lbm_step call.
 * Returns LBM_E_NONFINITE if the state held a non-finite value; LBM_E_STATE before any step. */
int lbm_residual(lbm_handle* h, double* r);

/* Precomputed geometry, for inspection (host outputs, any may be NULL).
 * counts[6] = {m, n_rows, n_entries, n_support_entries, n_interior, n_active}.
 * supp_ptr[m+1], supp_node[], supp_w[] (delta_il); phi[m], xstar[m*dim], dbv[m], W[m];
 * rows[n_rows] (node indices), row_ptr[n_rows+1], col_marker[], col_s[] (phi_k delta_ik W_k). */
int ib_geometry_counts(lbm_handle* h, long long* counts);
int ib_geometry(lbm_handle* h, long long* supp_ptr, long long* supp_node, double* supp_w,
                double* phi, double* xstar, double* dbv, double* W, long long* rows,
                long long* row_ptr, long long* col_marker, double* col_s, long long* interior);

/* Per-marker results of the last step (host, any may be NULL): F[m*dim], Wib[m], Qib[m],
 * rho[m], T[m] (interpolated predicted values), uP[m*dim], TP[m] (projection point). Synchronises. */
int ib_marker_state(lbm_handle* h, double* F, double* Wib, double* Qib, double* rho, double* T,
                    double* uP, double* TP);

/* ---- Batches of independent 2D grids -------------------------------------------------------
 * Many D2Q9 cases of uneven size (each its own handle, body and parameters) advanced together:
 * per step one launch computes the marker forces of every case, one spreads them, and one
 * persistent launch runs the fused sweep (the same per-node update as lbm_step, Sec. 2.5 and
 * Appendix A) over a queue of tiles of all cases; the steps are replayed from captured HIP graphs.
 * The handles keep their own state: lbm_fields, ib_wall_loads, lbm_residual etc. work on each
 * case after batch steps exactly as after lbm_step. Results per case are identical to lbm_step
 * except the residual, which is reduced in a different (fixed) order.
 * Requirements: every case is 2D, all share the precision and the HIP stream; a handle appears
 * once; the handles and the workspace outlive the batch. A case may be changed between batch
 * calls (ib_set_markers, lbm_step, lbm_set_fields, lbm_set_state); the batch notices and
 * rebuilds its tables. Not thread-safe. */
typedef struct lbm_batch lbm_batch;

/* Device workspace bytes for a batch of these n cases (0 if invalid). */
size_t lbm_batch_workspace_bytes(lbm_handle* const* cases, int n);

/* Create a batch. dev_workspace: caller-owned device memory of at least
 * lbm_batch_workspace_bytes bytes, 256-byte aligned. autotune = 1 times the sweep for each tile
 * width (62, 126, 254 nodes) and chunk length (16, 32, 64, 128 rows) on the current states and
 * keeps the fastest (the states are left unchanged); 0 takes width 62 and chunks of 32 rows, or
 * of 16 rows when 32-row chunks would give fewer than eight work items per workgroup of the
 * persistent launch.
 * Errors: LBM_E_INVAL (see requirements), LBM_E_NOMEM, LBM_E_HIP. */
int lbm_batch_create(lbm_handle* const* cases, int n, void* dev_workspace, size_t bytes, int autotune,
                     lbm_batch** out);

/* Enqueue n steps of every case (graph replays) on the shared stream; the last step also
 * computes each case's residual (lbm_residual). Asynchronous. Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_batch_step(lbm_batch* b, int n);

/* As lbm_batch_step but launched without graphs and timed with HIP events: kernel_ms[0] marker
 * forces, [1] spreading, [2] sweep, each the average per step over all cases. Synchronises. */
int lbm_batch_step_timed(lbm_batch* b, int n, double* kernel_ms);

/* Residual of every case after its last step (as lbm_residual; NaN for a case whose state held
 * a non-finite value), out[n] on the host, in the order of creation. Synchronises.
 * Errors: LBM_E_STATE (a case has taken no step), LBM_E_HIP. */
int lbm_batch_residuals(lbm_batch* b, double* out);

/* Use tile width tile_x (62, 126 or 254 nodes) and chunks of `chunk` rows (>= 1) for the sweep.
 * Errors: LBM_E_INVAL (other values), LBM_E_HIP. */
int lbm_batch_set_tile(lbm_batch* b, int tile_x, int chunk);

/* cfg[6] = {tile width, chunk rows, persistent grid size, sweep work items, markers, CSR rows}. */
int lbm_batch_config(lbm_batch* b, int* cfg);

/* Release the batch (not the handles or the workspace). */
void lbm_batch_destroy(lbm_batch* b);

/* Message of the last error of this batch (of the last failed lbm_batch_create if b is NULL). */
const char* lbm_batch_last_error(lbm_batch* b);

/* ---- Two-level grid refinement ---------------------------------------------------------------
 * The paper computes every case on locally refined meshes without stating the scheme; this pair
 * of handles is the one adopted here (ratio 2, acoustic scaling). A fine handle covers a block of
 * the coarse grid: fine node 2k on axis a coincides with coarse node origin[a] + k, so the block
 * spans nf_a / 2 coarse cells. Lattice velocities, density and temperature are shared; the fine
 * handle is created with twice the coarse mu and lambda_ (lattice units of half the spacing and
 * half the step) and periodic closure (its edges are overwritten). One coupled step:
 *   1. the coarse grid takes one step (lbm_step);
 *   2. the fine grid takes two steps; after each, its outer band of `band` nodes is refilled from
 *      the coarse grid: coarse values linear in time (weight 1/2, then 1) between the states before
 *      and after step 1, multilinear in space;
 *   3. every coarse node whose fine counterpart lies at least `margin` fine nodes inside the block
 *      on every axis takes the fine values (restriction).
 * A transferred population keeps the equilibrium of its own density, velocity and temperature
 * (Eq. (A.3)) and scales its non-equilibrium part by s = taubar_f / (2 taubar_c) coarse to fine and
 * 1/s fine to coarse, taubar = mu / (rho cs^2) + 1/2 of each level (Eq. (6)); rho E is transferred
 * unchanged; the diagonal force history (a per-step quantity) by 1/2 and 2. The off-diagonal force
 * history exists only at a level's own forced nodes and is not transferred. The coupling is not
 * conservative. All arithmetic of the transfers is FP64; the stored state keeps each handle's
 * precision. Kernels run on the handles' common stream; no device memory is allocated.
 * Requirements (checked at creation, and the body ones before every step):
 *   - both handles of one dimension, precision, device and stream; equal gamma, sigma, rho_inf,
 *     u_inf, T_inf, with_aC; fine mu and lambda_ twice the coarse ones (relative 1e-12);
 *   - fine bc_x = LBM_BC_PERIODIC; fine node counts even, each > 2 band; 2 <= band <= margin;
 *   - the block inside the coarse grid without wrapping (origin[a] >= 0, origin[a] + nf_a / 2 <=
 *     nc_a - 1), and along x clear of the closure columns when the coarse bc_x is not periodic
 *     (origin[0] >= 2, origin[0] + nf_x / 2 <= nx_c - 3);
 *   - no body on the coarse handle; the fine body's forced nodes at least `margin` nodes from
 *     every edge of the fine grid. */
typedef struct lbm_refine lbm_refine;

/* Couple two handles; origin[dim] in coarse nodes. The handles outlive the coupling.
 * Errors: LBM_E_INVAL (see requirements), LBM_E_NOMEM (host). */
int lbm_refine_create(lbm_handle* coarse, lbm_handle* fine, const int* origin, int band, int margin,
                      lbm_refine** out);

/* Set every fine node from the current coarse state (interpolated and rescaled as the band),
 * with zero off-diagonal force history; the coarse state is not changed. Asynchronous.
 * Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_refine_prolong(lbm_refine* r);

/* Enqueue n coupled steps (with every nested level, see lbm_refine_nest). The last one leaves in
 * the coarse handle the residual (lbm_residual) between the coarse states before and after it,
 * restriction included. Asynchronous. From three steps on, pairs of coupled steps replay a HIP
 * graph captured on the first such call (again after a state index or a body changed). Within a
 * coupled step the coarse step runs on a second stream of the coupling beside the first fine
 * step; events join it before the band refill, so all work stays ordered on the handles' stream.
 * The graph, the streams and the events belong to the coupling and are freed by
 * lbm_refine_destroy.
 * Errors: LBM_E_INVAL (n < 0, a body requirement broken, a nested coupling), LBM_E_HIP. */
int lbm_refine_step(lbm_refine* r, int n);

/* Nest two couplings: inner couples a finer block to outer's fine handle (inner's coarse handle
 * must be outer's fine handle). Stepping outer then advances the fine level through inner: each
 * of its two steps is one coupled step of inner (so level k of a nest takes 2^k steps per step of
 * the outermost coarse level), and inner itself may hold a further nesting. The body, if any, is
 * on the finest handle; the middle handles hold none. Only the outermost coupling is stepped
 * (lbm_refine_step on a nested coupling returns LBM_E_INVAL). Requirement: the inner block lies at
 * least `band` nodes of the middle level inside that level's edges (its band holds wrapped values
 * until the outer coupling refills it). Errors: LBM_E_INVAL (handles do not match, already nested,
 * a cycle, the placement). */
int lbm_refine_nest(lbm_refine* outer, lbm_refine* inner);

/* Release the coupling (not the handles); a nesting it takes part in is undone. */
void lbm_refine_destroy(lbm_refine* r);

/* Message of the last error of this coupling (of the last failed lbm_refine_create if r is NULL). */
const char* lbm_refine_last_error(lbm_refine* r);

/* ---- Learned warm start helpers (2D handles; the network is declared in lbmib_nn.h) --------
 * Ma = |u_inf| / sqrt(gamma R T_inf). Arrays are device FP32 [N][4], node = x + nx y. */

/* Network input planes of the case: {SDF / sdf_scale, ma_n, re_n, body indicator}. SDF is the
 * distance to the nearest marker, negative where (x - X_l) . n_l < 0 for that marker (inside).
 * ma_n and re_n are the caller's normalised Mach and Reynolds numbers. Asynchronous.
 * Errors: LBM_E_INVAL (3D handle, sdf_scale <= 0), LBM_E_HIP. */
int lbm_learn_input(lbm_handle* h, double sdf_scale, double ma_n, double re_n, float* d_out);

/* Normalised fields of the current state (force-free rho, u, T as lbm_fields):
 * {(rho - rho_inf)/(rho_inf Ma^2), u_x/|u_inf|, u_y/|u_inf|, (T - T_inf)/(T_inf Ma^2)}.
 * Uses the working area (not during steps). Asynchronous. */
int lbm_learn_target(lbm_handle* h, float* d_out);

/* Warm start: the state is set, as lbm_set_fields, to the equilibrium of the denormalised
 * prediction d_pred (the inverse of lbm_learn_target's normalisation), zero force history, and
 * the populations get the second-order non-equilibrium part w_i H_i : Pi / (2 c_s^4) with
 * Pi = -rho c_s^2 tau_bar (grad u + grad u^T - div u I) (periodic central differences), the
 * stress the finite-difference branch of Eq. (A.7) gives the predicted velocity; mass, momentum
 * and energy are those of the prediction. Synchronises. Errors: LBM_E_INVAL, LBM_E_HIP. */
int lbm_learn_warm_start(lbm_handle* h, const float* d_pred);

/* Release the handle (not the caller's workspace). */
void lbm_destroy(lbm_handle* h);

/* Measurement helper: copy `bytes` bytes (a multiple of 16; both pointers 16-byte aligned) from
 * device memory src to device memory dst with a plain streaming kernel on hip_stream
 * (asynchronous). It is the yardstick the sweep's bandwidth is compared with (read + write).
 * Errors: LBM_E_INVAL (size or alignment), LBM_E_HIP. */
int lbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Message of the last error on this handle (or of the last failed lbm_init_grid if h is NULL). */
const char* lbm_last_error(lbm_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* LBMIB_H */
