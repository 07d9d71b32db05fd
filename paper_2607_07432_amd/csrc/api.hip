// C ABI of the library (declarations and contracts in include/lbmib.h).
//
// The handle carves every device array out of the caller's workspace; the library
// allocates no device memory. All device work is ordered on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"

using namespace lbmib;

namespace {

thread_local std::string g_init_error;

// ---- Static scratch of ib_wall_loads_noalloc ----------------------------------------------------
// Per-marker boundary errors [LBM_NOALLOC_MAX_MARKERS][4] followed by the 16 reduced loads. Every
// GPU the library runs on holds its own copy until the process ends. In host code `scratch` names
// a host-side stand-in, never the device memory: the device address of each GPU's copy is taken
// once per device with hipGetSymbolAddress (scratch_on_device) and only that address is passed on.
constexpr size_t kScratchLoads = 16;
constexpr size_t kScratchDoubles = size_t(LBM_NOALLOC_MAX_MARKERS) * 4 + kScratchLoads;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of the scratch copy of device dev; resolved on the first call for dev, which must
// run with dev current (lbm_init_grid calls it for the device the handle is created on).
double* scratch_on_device(int dev, hipError_t* err) {
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev] && g_scratch_err[dev] == hipSuccess) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess && ptr)
            g_scratch_ptr[dev] = static_cast<double*>(ptr);
        else
            g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Bump layout over the workspace: the same routine computes the size and the pointers.
struct Layout {
    char* base;
    size_t off = 0;
    explicit Layout(char* b) : base(b) {}
    template <class T>
    T* take(size_t count) {
        off = align_up(off);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int lattice_q(int dim) { return dim == 2 ? 9 : 19; }

size_t layout(const lbm_params& p, char* base, Dev* d) {
    Dev tmp;
    Dev& o = d ? *d : tmp;
    Layout L(base);
    const int D = p.dim, Q = lattice_q(D);
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const size_t s = p.precision == LBM_F64 ? 8 : 4;
    o.fA = L.take<char>(Q * N * s);
    o.eA = L.take<char>(N * s);
    o.hA = L.take<char>((D - 1) * N * s);
    o.fB = L.take<char>(Q * N * s);
    o.eB = L.take<char>(N * s);
    o.hB = L.take<char>((D - 1) * N * s);
    o.work = L.take<char>((D + 2 + Q) * N * s);
    o.rowmap = L.take<int>(N);
    o.partials = L.take<double>(2 * RESID_PARTS_MAX);
    o.resid = L.take<double>(2);
    o.loads = L.take<double>(16);
    o.flag = L.take<int>(4);
    const size_t mc = (size_t)(p.max_markers > 0 ? p.max_markers : 0);
    const size_t sc = mc * (D == 3 ? 64 : 16);        // at most 4 nodes per axis (strict |r| < 2)
    const size_t pc = mc * (D == 3 ? 8 : 4);          // at most 2 nodes per axis (strict |r| < 1)
    o.supp_ptr = L.take<long long>(mc + 1);
    o.supp_node = L.take<long long>(sc);
    o.supp_w = L.take<double>(sc);
    o.proj_ptr = L.take<long long>(mc + 1);
    o.proj_node = L.take<long long>(pc);
    o.proj_w = L.take<double>(pc);
    o.tw_ptr = L.take<long long>(mc + 1);
    o.tw_node = L.take<long long>(sc);
    o.tw_w = L.take<double>(sc);
    o.phi = L.take<double>(mc);
    o.dbv = L.take<double>(mc);
    o.W = L.take<double>(mc);
    o.u_wall = L.take<double>(mc * D);
    o.t_value = L.take<double>(mc);
    o.t_kind = L.take<int>(mc);
    o.Xm = L.take<double>(mc * D);
    o.nm = L.take<double>(mc * D);
    o.G = L.take<double>(mc * (D + 2));
    o.diag = L.take<double>(mc * 8);
    o.eps = L.take<double>(mc * 4);
    o.rows = L.take<long long>(sc);
    o.row_ptr = L.take<long long>(sc + 1);
    o.col_marker = L.take<long long>(sc);
    o.col_s = L.take<double>(sc);
    o.fib = L.take<double>(sc * D);
    o.fE = L.take<double>(sc);
    o.h2off = L.take<double>(sc * (D == 3 ? 3 : 1));
    o.h2off2 = L.take<double>(sc * (D == 3 ? 3 : 1));
    return align_up(L.off);
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

namespace {

int fail(lbm_handle* h, int code, const std::string& msg) {
    if (h)
        h->err = msg;
    else
        g_init_error = msg;
    return code;
}

#define HIPCHK(h, call)                                                                                 \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail((h), LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)


void refresh_args(lbm_handle* h) {
    h->args.rows.nrows = (int)h->geom.rows.size();
    h->args.rows.rowmap = h->d.rowmap;
    h->args.rows.rows = h->d.rows;
    h->args.rows.fib = h->d.fib;
    h->args.rows.fE = h->d.fE;
    h->args.rows.h2off = h->cur == 0 ? h->d.h2off : h->d.h2off2;
    h->args.rows.h2off_out = h->cur == 0 ? h->d.h2off2 : h->d.h2off;
    MarkersP& m = h->mk;
    m.m = h->geom.m;
    m.dim = h->D;
    m.method = h->method;
    m.supp_ptr = h->d.supp_ptr;
    m.supp_node = h->d.supp_node;
    m.supp_w = h->d.supp_w;
    m.proj_ptr = h->d.proj_ptr;
    m.proj_node = h->d.proj_node;
    m.proj_w = h->d.proj_w;
    m.tw_ptr = h->d.tw_ptr;
    m.tw_node = h->d.tw_node;
    m.tw_w = h->d.tw_w;
    m.phi = h->d.phi;
    m.dbv = h->d.dbv;
    m.W = h->d.W;
    m.u_wall = h->d.u_wall;
    m.t_value = h->d.t_value;
    m.t_kind = h->d.t_kind;
    m.row_ptr = h->d.row_ptr;
    m.col_marker = h->d.col_marker;
    m.col_s = h->d.col_s;
    m.G = h->d.G;
    m.diag = h->d.diag;
    m.eps = h->d.eps;
}

}  // namespace

void lbmib::refresh_handle_args(lbm_handle* h) { refresh_args(h); }

namespace {

int validate_params(const lbm_params* p, std::string& why) {
    if (!p) return why = "params is NULL", LBM_E_INVAL;
    if (p->dim != 2 && p->dim != 3) return why = "dim must be 2 or 3", LBM_E_INVAL;
    // Stencils reach two nodes along every axis and the periodic wraps add or subtract the axis
    // length once, so every active axis holds at least two nodes; x also holds the two inflow
    // and two outflow columns of the domain closure plus one interior column.
    if (p->nx < 5 || p->ny < 2 || p->nz < 1 || (p->dim == 3 && p->nz < 2))
        return why = "grid too small (nx >= 5, ny >= 2, and nz >= 2 in 3D)", LBM_E_INVAL;
    if (p->dim == 2 && p->nz != 1) return why = "nz must be 1 in 2D", LBM_E_INVAL;
    if (p->precision != LBM_F32 && p->precision != LBM_F64) return why = "precision must be 32 or 64", LBM_E_INVAL;
    if (p->bc_x != LBM_BC_PERIODIC && p->bc_x != LBM_BC_INFLOW_OUTFLOW && p->bc_x != LBM_BC_CHARACTERISTIC)
        return why = "bad bc_x", LBM_E_INVAL;
    if (p->bc_x == LBM_BC_CHARACTERISTIC && !(is_fin(p->sigma_c) && p->sigma_c >= 0.0))
        return why = "sigma_c must be finite and >= 0", LBM_E_INVAL;
    if (p->kernel != LBM_KERNEL_COS && p->kernel != LBM_KERNEL_ROMA3) return why = "bad kernel", LBM_E_INVAL;
    if (p->max_markers < 0) return why = "max_markers < 0", LBM_E_INVAL;
    const double vals[] = {p->gamma, p->mu, p->lambda_, p->sigma, p->rho_inf, p->u_inf[0], p->u_inf[1],
                           p->u_inf[2], p->T_inf, p->ref_len, p->ref_area, p->surface, p->T_wall};
    for (double v : vals)
        if (!is_fin(v)) return why = "non-finite parameter", LBM_E_INVAL;
    if (p->gamma <= 1.0 || p->mu <= 0.0 || p->lambda_ < 0.0 || p->rho_inf <= 0.0 || p->T_inf <= 0.0)
        return why = "need gamma > 1, mu > 0, lambda >= 0, rho_inf > 0, T_inf > 0", LBM_E_INVAL;
    if (p->sigma < 0.0 || p->sigma > 1.0) return why = "sigma must lie in [0, 1]", LBM_E_INVAL;
    if (p->sweep != LBM_SWEEP_FUSED && p->sweep != LBM_SWEEP_THREE_PASS) return why = "bad sweep", LBM_E_INVAL;
    if (p->dim == 2 && p->u_inf[2] != 0.0) return why = "u_inf[2] must be 0 in 2D", LBM_E_INVAL;
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) {
    std::string why;
    if (validate_params(p, why) != LBM_OK) return 0;
    return layout(*p, nullptr, nullptr);
}

int lbm_init_grid(const lbm_params* p, void* ws, size_t bytes, void* stream, lbm_handle** out) {
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (validate_params(p, why) != LBM_OK) return fail(nullptr, LBM_E_INVAL, why);
    const size_t need = layout(*p, nullptr, nullptr);
    if (!ws || bytes < need)
        return fail(nullptr, LBM_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(nullptr, LBM_E_INVAL, "workspace not 256-byte aligned");

    const int D = p->dim;
    const double Cv = (1.0 / 3.0) / (p->gamma - 1.0);
    // The rest population of the free-stream equilibrium (Eq. (A.3)), whose temperature term
    // rho (w_0 - 1)(theta - 1) turns it negative when T_inf is too large for T_ref, must be positive.
    // The moving populations are not checked: with a low T_ref (small theta) the upstream ones go
    // negative at moderate Mach numbers, which the regularised scheme tolerates (the paper's
    // supersonic cases need it).
    double u[3] = {p->u_inf[0], p->u_inf[1], p->u_inf[2]};
    double fd[19];
    if (D == 2)
        feq_dev<D2Q9, double>(p->rho_inf, u, p->T_inf, fd);
    else
        feq_dev<D3Q19, double>(p->rho_inf, u, p->T_inf, fd);
    const int Q = lattice_q(D);
    if (!(fd[0] + (D == 2 ? D2Q9::w[0] : D3Q19::w[0]) > 0.0))
        return fail(nullptr, LBM_E_INVAL, "free-stream rest population is not positive (T_inf too large for T_ref)");

    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    h->p = *p;
    h->D = D;
    h->Q = Q;
    h->N = (long long)p->nx * p->ny * p->nz;
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    {
        hipError_t se = hipSuccess;
        (void)scratch_on_device(h->device, &se);   // once per device, with the handle's device current
    }
    if (const char* ch = std::getenv("LBMIB_FUSED_CHUNK")) h->chunk = std::atoi(ch);
    layout(*p, (char*)ws, &h->d);

    SweepArgs& a = h->args;
    a.grid = {p->nx, p->ny, p->nz, h->N, p->bc_x};
    if (h->chunk <= 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) cus = 0;
        if (D == 2)
            h->chunk = p->precision == LBM_F64 ? fused_auto_chunk<D2Q9, double>(a.grid, cus)
                                               : fused_auto_chunk<D2Q9, float>(a.grid, cus);
        else
            h->chunk = p->precision == LBM_F64 ? fused_auto_chunk<D3Q19, double>(a.grid, cus)
                                               : fused_auto_chunk<D3Q19, float>(a.grid, cus);
    }
    a.gas = {p->mu, p->lambda_, p->gamma, p->sigma, Cv, Cv + 1.0 / 3.0, p->with_aC, 1.0 / Cv};
    for (int i = 0; i < 19; ++i) a.fs.fdev[i] = i < Q ? fd[i] : 0.0;
    double uu = 0;
    for (int b = 0; b < 3; ++b) uu += u[b] * u[b];
    a.fs.e_ref = p->rho_inf * (0.5 * uu + Cv * p->T_inf);
    a.fs.eint_inf = p->rho_inf * Cv * p->T_inf;
    a.fs.rho_inf = p->rho_inf;
    for (int b = 0; b < 3; ++b) a.fs.u_inf[b] = u[b];
    a.fs.T_inf = p->T_inf;
    refresh_args(h);

    hipError_t e = hipMemsetAsync(h->d.rowmap, 0xFF, sizeof(int) * h->N, h->stream);
    if (e == hipSuccess)
        e = dispatch(h, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            return launch_init_state<LT, ST>(h->args, stateA<ST>(h), h->stream);
        });
    if (e != hipSuccess) {
        std::string m = std::string("init: ") + hipGetErrorString(e);
        delete h;
        return fail(nullptr, LBM_E_HIP, m);
    }
    *out = h;
    return LBM_OK;
}

int ib_set_markers(lbm_handle* h, int m, const double* X, const double* normal, const double* area_w,
                   const double* u_wall, const int* t_kind, const double* t_value, int method) {
    (void)area_w;
    if (!h) return LBM_E_INVAL;
    const int D = h->D;
    if (m < 0 || m > h->p.max_markers) return fail(h, LBM_E_INVAL, "marker count outside [0, max_markers]");
    if (method < LBM_IB_DIBM || method > LBM_IB_FODIBM_R) return fail(h, LBM_E_INVAL, "bad method");
    if (m > 0 && (!X || !normal || !u_wall || !t_kind || !t_value)) return fail(h, LBM_E_INVAL, "NULL marker array");
    const long long dims[3] = {h->p.nx, h->p.ny, h->p.nz};
    for (int l = 0; l < m; ++l) {
        double nn = 0;
        for (int a = 0; a < D; ++a) {
            const double x = X[l * D + a], nv = normal[l * D + a];
            if (!is_fin(x) || !is_fin(nv) || !is_fin(u_wall[l * D + a]))
                return fail(h, LBM_E_INVAL, "non-finite marker data at marker " + std::to_string(l));
            nn += nv * nv;
            const double margin = (a == 0 && h->p.bc_x != LBM_BC_PERIODIC) ? 4.0 : 3.0;
            if (x < margin || x > (double)(dims[a] - 1) - margin)
                return fail(h, LBM_E_INVAL, "marker " + std::to_string(l) + " too close to the domain edge");
        }
        if (std::fabs(std::sqrt(nn) - 1.0) > 1e-12) return fail(h, LBM_E_INVAL, "normal not of unit length");
        if (!is_fin(t_value[l]) || t_kind[l] < 0 || t_kind[l] > 2)
            return fail(h, LBM_E_INVAL, "bad thermal condition at marker " + std::to_string(l));
    }
    GeomInput in{D, {dims[0], dims[1], dims[2]}, m, X, normal, method, h->p.kernel};
    std::string why;
    Geometry g;
    build_geometry(in, g, why);
    const size_t mc = (size_t)h->p.max_markers;
    const size_t sc = mc * (D == 3 ? 64 : 16);
    if (g.supp_node.size() > sc || g.tw_node.size() > sc || g.rows.size() > sc || g.col_marker.size() > sc)
        return fail(h, LBM_E_NOMEM, "precomputed lists exceed the workspace");

    // Clear the previous body's row map and forcing, then upload.
    hipStream_t st = h->stream;
    HIPCHK(h, hipStreamSynchronize(st));
    HIPCHK(h, hipMemsetAsync(h->d.rowmap, 0xFF, sizeof(int) * h->N, st));
    h->geom = std::move(g);
    {
        // bounding box of the forced nodes; the whole grid if any lies within 2 nodes of an edge
        // (a tile footprint reaches 2 nodes past the tile and wraps periodically)
        int* fb = h->fbox;
        const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
        const int nm = D == 3 ? nz : ny;
        fb[0] = nx; fb[1] = -1; fb[2] = ny; fb[3] = -1; fb[4] = nm; fb[5] = -1;
        for (long long n : h->geom.rows) {
            const int x = (int)(n % nx);
            const long long q = n / nx;
            const int y = D == 3 ? (int)(q % ny) : 0;
            const int mm = D == 3 ? (int)(q / ny) : (int)q;
            fb[0] = std::min(fb[0], x); fb[1] = std::max(fb[1], x);
            fb[2] = std::min(fb[2], y); fb[3] = std::max(fb[3], y);
            fb[4] = std::min(fb[4], mm); fb[5] = std::max(fb[5], mm);
        }
        if (fb[0] <= fb[1] && (fb[0] < 2 || fb[1] > nx - 3 || fb[4] < 2 || fb[5] > nm - 3 ||
                               (D == 3 && (fb[2] < 2 || fb[3] > ny - 3)))) {
            fb[0] = 0; fb[1] = nx - 1; fb[2] = 0; fb[3] = ny - 1; fb[4] = 0; fb[5] = nm - 1;
        }
        if (D == 2 && fb[0] <= fb[1]) { fb[2] = 0; fb[3] = 0; }
    }
    h->method = method;
    const Geometry& G = h->geom;
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    std::vector<long long> zero_ptr(1, 0);
    const std::vector<long long>& sp = m ? G.supp_ptr : zero_ptr;
    const std::vector<long long>& pp = m ? G.proj_ptr : zero_ptr;
    const std::vector<long long>& tp = m ? G.tw_ptr : zero_ptr;
    const std::vector<long long>& rp = G.row_ptr.empty() ? zero_ptr : G.row_ptr;
    HIPCHK(h, up(h->d.supp_ptr, sp.data(), sp.size() * 8));
    HIPCHK(h, up(h->d.supp_node, G.supp_node.data(), G.supp_node.size() * 8));
    HIPCHK(h, up(h->d.supp_w, G.supp_w.data(), G.supp_w.size() * 8));
    HIPCHK(h, up(h->d.proj_ptr, pp.data(), pp.size() * 8));
    HIPCHK(h, up(h->d.proj_node, G.proj_node.data(), G.proj_node.size() * 8));
    HIPCHK(h, up(h->d.proj_w, G.proj_w.data(), G.proj_w.size() * 8));
    HIPCHK(h, up(h->d.tw_ptr, tp.data(), tp.size() * 8));
    HIPCHK(h, up(h->d.tw_node, G.tw_node.data(), G.tw_node.size() * 8));
    HIPCHK(h, up(h->d.tw_w, G.tw_w.data(), G.tw_w.size() * 8));
    HIPCHK(h, up(h->d.phi, G.phi.data(), G.phi.size() * 8));
    HIPCHK(h, up(h->d.dbv, G.dbv.data(), G.dbv.size() * 8));
    HIPCHK(h, up(h->d.W, G.W.data(), G.W.size() * 8));
    HIPCHK(h, up(h->d.u_wall, u_wall, (size_t)m * D * 8));
    HIPCHK(h, up(h->d.t_value, t_value, (size_t)m * 8));
    HIPCHK(h, up(h->d.t_kind, t_kind, (size_t)m * 4));
    HIPCHK(h, up(h->d.Xm, X, (size_t)m * D * 8));
    HIPCHK(h, up(h->d.nm, normal, (size_t)m * D * 8));
    HIPCHK(h, up(h->d.rows, G.rows.data(), G.rows.size() * 8));
    HIPCHK(h, up(h->d.row_ptr, rp.data(), rp.size() * 8));
    HIPCHK(h, up(h->d.col_marker, G.col_marker.data(), G.col_marker.size() * 8));
    HIPCHK(h, up(h->d.col_s, G.col_s.data(), G.col_s.size() * 8));
    const size_t nr = G.rows.size();
    if (nr) {
        HIPCHK(h, hipMemsetAsync(h->d.fib, 0, nr * D * 8, st));
        HIPCHK(h, hipMemsetAsync(h->d.fE, 0, nr * 8, st));
        HIPCHK(h, hipMemsetAsync(h->d.h2off, 0, nr * (D == 3 ? 3 : 1) * 8, st));
        HIPCHK(h, hipMemsetAsync(h->d.h2off2, 0, nr * (D == 3 ? 3 : 1) * 8, st));
    }
    if (m) {
        HIPCHK(h, hipMemsetAsync(h->d.G, 0, (size_t)m * (D + 2) * 8, st));
        HIPCHK(h, hipMemsetAsync(h->d.diag, 0, (size_t)m * 8 * 8, st));
    }
    refresh_args(h);
    HIPCHK(h, launch_rowmap(h->d.rows, (int)nr, h->d.rowmap, st));
    HIPCHK(h, hipStreamSynchronize(st));   // host vectors above must outlive the copies
    h->markers_set = m > 0;
    h->stepped = 0;
    h->geom_version++;
    return LBM_OK;
}

namespace {

// n steps; with ev (4 events per step) the marker, spread and sweep launches are bracketed. The
// last step forms the residual unless want_resid is false.
int run_steps(lbm_handle* h, int n, hipEvent_t* ev, bool want_resid = true) {
    for (int s = 0; s < n; ++s) {
        const bool last = want_resid && s == n - 1;
        hipEvent_t* e4 = ev ? ev + 4 * s : nullptr;
        hipError_t e = dispatch(h, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            StateP<ST> A = current<ST>(h), B = other<ST>(h);
            hipError_t r = hipSuccess;
            if (e4) r = hipEventRecord(e4[0], h->stream);
            if (h->markers_set && r == hipSuccess) {
                r = launch_markers<LT, ST>(h->args, h->mk, A, h->stream);
                if (r == hipSuccess && e4) r = hipEventRecord(e4[1], h->stream);
                if (r == hipSuccess) r = launch_spread(h->D, h->mk, h->args.rows, h->stream);
            } else if (e4 && r == hipSuccess) {
                r = hipEventRecord(e4[1], h->stream);
            }
            if (r == hipSuccess && e4) r = hipEventRecord(e4[2], h->stream);
            ST* M = (ST*)h->d.work;
            ST* fcol = M + (size_t)(h->D + 2) * h->N;
            // the last step's residual: formed by the fused sweep where it can, else k_residual
            int rparts = 0;
            if (r == hipSuccess) {
                if (h->p.sweep == LBM_SWEEP_THREE_PASS)
                    r = launch_split_step<LT, ST, ST>(h->args, A, B, M, fcol, h->stream);
                else
                    r = launch_fused_step<LT, ST>(h->args, A, B, h->chunk, h->fbox, h->stream,
                                                  last ? h->d.partials : nullptr, RESID_PARTS_MAX, &rparts);
            }
            if (r == hipSuccess && h->p.bc_x == LBM_BC_CHARACTERISTIC)
                r = launch_outlet_char<LT, ST>(h->args, A, B, h->p.sigma_c, h->stream);
            if (r == hipSuccess && e4) r = hipEventRecord(e4[3], h->stream);
            if (r == hipSuccess && last) {
                if (rparts > 0)
                    r = launch_residual_final<LT>(h->args, h->d.partials, rparts, h->d.resid, h->stream);
                else
                    r = launch_residual<LT, ST>(h->args, A, B, h->d.partials, residual_parts(h->N), h->d.resid,
                                                h->stream);
            }
            return r;
        });
        if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("lbm_step: ") + hipGetErrorString(e));
        h->cur ^= 1;
        refresh_args(h);
    }
    if (n > 0) {
        h->stepped = 1;
        h->any_step = 1;
    }
    return LBM_OK;
}

// Calls of at least this many steps replay the two-step graph.
constexpr int kGraphMinSteps = 5;

// Capture (once per state index and body) the two steps from the current state. Nothing runs
// during the capture, and the state index ends where it started.
int ensure_graph(lbm_handle* h) {
    if (h->graph_exec && h->graph_cur == h->cur && h->graph_geom == h->geom_version) return LBM_OK;
    if (h->graph_exec) {
        hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
    }
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const int cur0 = h->cur, stepped = h->stepped, any = h->any_step;
    hipStream_t user = h->stream;
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    h->stream = h->cap_stream;
    const int rc = run_steps(h, 2, nullptr, false);
    h->stream = user;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap_stream, &g);
    h->stepped = stepped;
    h->any_step = any;
    if (h->cur != cur0) {   // a failed capture may stop after one step
        h->cur = cur0;
        refresh_args(h);
    }
    if (rc != LBM_OK || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return rc != LBM_OK ? rc : fail(h, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph_exec = nullptr;
        return fail(h, LBM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    h->graph_cur = h->cur;
    h->graph_geom = h->geom_version;
    return LBM_OK;
}

}  // namespace

int lbm_step(lbm_handle* h, int n) {
    if (!h) return LBM_E_INVAL;
    if (n < 0) return fail(h, LBM_E_INVAL, "n < 0");
    if (n < kGraphMinSteps) return run_steps(h, n, nullptr);
    // pairs of steps replay the captured graph; an odd step and the last one (which forms the
    // residual) run directly
    int m = n - 1;
    if (m % 2) {
        if (int rc = run_steps(h, 1, nullptr, false)) return rc;
        --m;
    }
    if (int rc = ensure_graph(h)) return rc;
    for (int i = 0; i < m / 2; ++i) HIPCHK(h, hipGraphLaunch(h->graph_exec, h->stream));
    return run_steps(h, 1, nullptr, true);
}

int lbm_step_timed(lbm_handle* h, int n, double* kernel_ms) {
    if (!h || !kernel_ms) return LBM_E_INVAL;
    if (n <= 0) return fail(h, LBM_E_INVAL, "n must be positive");
    std::vector<hipEvent_t> ev((size_t)4 * n);
    for (auto& e : ev) HIPCHK(h, hipEventCreate(&e));
    int rc = run_steps(h, n, ev.data());
    if (rc == LBM_OK) {
        hipError_t e = hipEventSynchronize(ev.back());
        double acc[3] = {0, 0, 0};
        for (int s = 0; s < n && e == hipSuccess; ++s)
            for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                float ms = 0;
                e = hipEventElapsedTime(&ms, ev[4 * s + k], ev[4 * s + k + 1]);
                acc[k] += ms;
            }
        if (e != hipSuccess) rc = fail(h, LBM_E_HIP, std::string("event timing: ") + hipGetErrorString(e));
        for (int k = 0; k < 3; ++k) kernel_ms[k] = acc[k] / n;
    }
    for (auto& e : ev) hipEventDestroy(e);
    return rc;
}

int lbm_residual(lbm_handle* h, double* r) {
    if (!h || !r) return LBM_E_INVAL;
    if (!h->any_step) return fail(h, LBM_E_STATE, "no step taken");
    double out[2];
    HIPCHK(h, hipMemcpyAsync(out, h->d.resid, sizeof(out), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *r = out[0];
    if (out[1] != 0.0) return fail(h, LBM_E_NONFINITE, "non-finite value in the state");
    return LBM_OK;
}

namespace {

// Loads of the last step with the per-marker error buffer eps ([m][4]) and the reduced-loads buffer
// loads (16 doubles) given by the caller of this helper: the handle's workspace or the static scratch.
int wall_loads_with(lbm_handle* h, lbm_loads* out, double* eps, double* loads) {
    const lbm_params& p = h->p;
    double ur = std::sqrt(p.u_inf[0] * p.u_inf[0] + p.u_inf[1] * p.u_inf[1] + p.u_inf[2] * p.u_inf[2]);
    const double u_ref = ur > 0 ? ur : 1.0;
    MarkersP mk = h->mk;
    mk.eps = eps;
    hipError_t e = dispatch(h, [&](auto L, auto S) {
        using LT = decltype(L);
        using ST = decltype(S);
        return launch_eps<LT, ST>(h->args, mk, current<ST>(h), u_ref, p.T_inf, p.ref_len, h->stream);
    });
    if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("eps: ") + hipGetErrorString(e));
    HIPCHK(h, launch_loads(h->D, mk, loads, h->stream));
    double v[11];
    HIPCHK(h, hipMemcpyAsync(v, loads, sizeof(v), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof(*out));
    for (int b = 0; b < h->D; ++b) out->F[b] = v[b];
    out->Q_heat = v[3];
    const double q = 0.5 * p.rho_inf * u_ref * u_ref * p.ref_area;
    out->Cd = out->F[0] / q;
    out->Cl = out->F[1] / q;
    out->Nu = (p.T_wall != p.T_inf) ? out->Q_heat * p.ref_len / (p.lambda_ * (p.T_wall - p.T_inf) * p.surface) : 0.0;
    out->eps_dir = v[5] > 0 ? v[4] / v[5] : 0.0;
    out->eps_neu = v[7] > 0 ? v[6] / v[7] : 0.0;
    out->eps_iso = v[9] > 0 ? v[8] / v[9] : 0.0;
    out->n_inactive = (int)v[10];
    out->n_markers = h->geom.m;
    return LBM_OK;
}

}  // namespace

int ib_wall_loads(lbm_handle* h, lbm_loads* out) {
    if (!h || !out) return LBM_E_INVAL;
    if (!h->markers_set || !h->stepped) return fail(h, LBM_E_STATE, "no body or no step since it was set");
    return wall_loads_with(h, out, h->mk.eps, h->d.loads);
}

int ib_wall_loads_noalloc(lbm_handle* h, lbm_loads* out) {
    if (!h || !out) return LBM_E_INVAL;
    if (!h->markers_set || !h->stepped) return fail(h, LBM_E_STATE, "no body or no step since it was set");
    if (h->geom.m > LBM_NOALLOC_MAX_MARKERS)
        return fail(h, LBM_E_INVAL, "ib_wall_loads_noalloc: " + std::to_string(h->geom.m) + " markers exceed the " +
                                        std::to_string(LBM_NOALLOC_MAX_MARKERS) + " of the static scratch");
    hipError_t se = hipSuccess;
    double* buf = scratch_on_device(h->device, &se);
    if (!buf) return fail(h, LBM_E_HIP, std::string("static scratch: ") + hipGetErrorString(se));
    // Every marker's error row is rewritten by the eps kernel and every load by the reduction, so
    // nothing left from an earlier call (of any handle on this device) is read.
    return wall_loads_with(h, out, buf, buf + size_t(LBM_NOALLOC_MAX_MARKERS) * 4);
}

int lbm_fields(lbm_handle* h, int dtype, int on_device, void* rho, void* u, void* T, void* p) {
    if (!h) return LBM_E_INVAL;
    if (dtype != LBM_F32 && dtype != LBM_F64) return fail(h, LBM_E_INVAL, "dtype must be 32 or 64");
    const size_t N = (size_t)h->N;
    const size_t esz = dtype == LBM_F64 ? 8 : 4;
    auto run = [&](void* r_, void* u_, void* T_, void* p_) -> hipError_t {
        return dispatch(h, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            if (dtype == LBM_F64)
                return launch_fields<LT, ST, double>(h->args, current<ST>(h), (double*)r_, (double*)u_, (double*)T_,
                                                     (double*)p_, h->stream);
            return launch_fields<LT, ST, float>(h->args, current<ST>(h), (float*)r_, (float*)u_, (float*)T_,
                                                (float*)p_, h->stream);
        });
    };
    if (on_device) {
        HIPCHK(h, run(rho, u, T, p));
        return LBM_OK;
    }
    // Host outputs: one field at a time through the working area (free between steps).
    char* scratch = (char*)h->d.work;
    void* outs[4] = {rho, u, T, p};
    const size_t comps[4] = {1, (size_t)h->D, 1, 1};
    for (int k = 0; k < 4; ++k) {
        if (!outs[k]) continue;
        void* ptrs[4] = {nullptr, nullptr, nullptr, nullptr};
        ptrs[k] = scratch;
        HIPCHK(h, run(ptrs[0], ptrs[1], ptrs[2], ptrs[3]));
        HIPCHK(h, hipMemcpyAsync(outs[k], scratch, comps[k] * N * esz, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return LBM_OK;
}

int lbm_set_fields(lbm_handle* h, int on_device, const double* rho, const double* u, const double* T) {
    if (!h || !rho || !u || !T) return LBM_E_INVAL;
    const size_t N = (size_t)h->N;
    const double *dr = rho, *du = u, *dT = T;
    if (!on_device) {
        double* s = (double*)h->d.work;   // (D + 2) N doubles fit in the working area
        HIPCHK(h, hipMemcpyAsync(s, rho, N * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(s + N, u, (size_t)h->D * N * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(s + (1 + h->D) * N, T, N * 8, hipMemcpyHostToDevice, h->stream));
        dr = s;
        du = s + N;
        dT = s + (1 + h->D) * N;
    }
    hipError_t e = dispatch(h, [&](auto L, auto S) {
        using LT = decltype(L);
        using ST = decltype(S);
        return launch_set_fields<LT, ST>(h->args, current<ST>(h), dr, du, dT, h->stream);
    });
    if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("set_fields: ") + hipGetErrorString(e));
    const size_t nr = h->geom.rows.size();
    if (nr) {
        HIPCHK(h, hipMemsetAsync(h->d.h2off, 0, nr * (h->D == 3 ? 3 : 1) * 8, h->stream));
        HIPCHK(h, hipMemsetAsync(h->d.h2off2, 0, nr * (h->D == 3 ? 3 : 1) * 8, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// The canonical state moves one component (N doubles) at a time through the working area.
int lbm_get_state(lbm_handle* h, double* f, double* rhoE, double* H2) {
    if (!h || !f || !rhoE || !H2) return LBM_E_INVAL;
    const size_t N = (size_t)h->N;
    const int D = h->D, Q = h->Q;
    double* s = (double*)h->d.work;
    for (int c = 0; c < Q + 1 + D * D; ++c) {
        hipError_t e = dispatch(h, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            return launch_export<LT, ST>(h->args, current<ST>(h), c, s, h->stream);
        });
        if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("get_state: ") + hipGetErrorString(e));
        double* dst = c < Q ? f + (size_t)c * N : (c == Q ? rhoE : H2 + (size_t)(c - Q - 1) * N);
        HIPCHK(h, hipMemcpyAsync(dst, s, N * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    return LBM_OK;
}

int lbm_set_state(lbm_handle* h, const double* f, const double* rhoE, const double* H2) {
    if (!h || !f || !rhoE || !H2) return LBM_E_INVAL;
    const size_t N = (size_t)h->N;
    const int D = h->D, Q = h->Q;
    double* s = (double*)h->d.work;
    HIPCHK(h, hipMemsetAsync(h->d.flag, 0, sizeof(int), h->stream));
    for (int c = 0; c < Q + 1 + D * D; ++c) {
        const double* src = c < Q ? f + (size_t)c * N : (c == Q ? rhoE : H2 + (size_t)(c - Q - 1) * N);
        HIPCHK(h, hipMemcpyAsync(s, src, N * 8, hipMemcpyHostToDevice, h->stream));
        hipError_t e = dispatch(h, [&](auto L, auto S) {
            using LT = decltype(L);
            using ST = decltype(S);
            SweepArgs ia = h->args;
            ia.rows.h2off_out = const_cast<double*>(ia.rows.h2off);   // import writes the current buffer
            return launch_import<LT, ST>(ia, current<ST>(h), c, s, h->d.flag, h->stream);
        });
        if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("set_state: ") + hipGetErrorString(e));
        HIPCHK(h, hipStreamSynchronize(h->stream));   // the host source must stay valid until copied
    }
    int bad = 0;
    HIPCHK(h, hipMemcpyAsync(&bad, h->d.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (bad) return fail(h, LBM_E_INVAL, "off-diagonal force history away from the forced nodes");
    return LBM_OK;
}

int ib_geometry_counts(lbm_handle* h, long long* c) {
    if (!h || !c) return LBM_E_INVAL;
    const Geometry& g = h->geom;
    c[0] = g.m;
    c[1] = (long long)g.rows.size();
    c[2] = (long long)g.col_marker.size();
    c[3] = (long long)g.supp_node.size();
    c[4] = (long long)g.interior.size();
    c[5] = g.n_active;
    return LBM_OK;
}

int ib_geometry(lbm_handle* h, long long* supp_ptr, long long* supp_node, double* supp_w, double* phi,
                double* xstar, double* dbv, double* W, long long* rows, long long* row_ptr, long long* col_marker,
                double* col_s, long long* interior) {
    if (!h) return LBM_E_INVAL;
    const Geometry& g = h->geom;
    auto cp = [](auto* dst, const auto& v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(supp_ptr, g.supp_ptr);
    cp(supp_node, g.supp_node);
    cp(supp_w, g.supp_w);
    cp(phi, g.phi);
    cp(xstar, g.xstar);
    cp(dbv, g.dbv);
    cp(W, g.W);
    cp(rows, g.rows);
    cp(row_ptr, g.row_ptr);
    cp(col_marker, g.col_marker);
    cp(col_s, g.col_s);
    cp(interior, g.interior);
    return LBM_OK;
}

int ib_marker_state(lbm_handle* h, double* F, double* Wib, double* Qib, double* rho, double* T, double* uP,
                    double* TP) {
    if (!h) return LBM_E_INVAL;
    const int m = h->geom.m, D = h->D;
    if (m == 0) return fail(h, LBM_E_STATE, "no body");
    std::vector<double> G((size_t)m * (D + 2)), dg((size_t)m * 8);
    HIPCHK(h, hipMemcpyAsync(G.data(), h->d.G, G.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(dg.data(), h->d.diag, dg.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int l = 0; l < m; ++l) {
        for (int b = 0; b < D; ++b) {
            if (F) F[l * D + b] = G[(size_t)l * (D + 2) + b];
            if (uP) uP[l * D + b] = dg[(size_t)l * 8 + 3 + b];
        }
        if (Wib) Wib[l] = G[(size_t)l * (D + 2) + D];
        if (Qib) Qib[l] = G[(size_t)l * (D + 2) + D + 1];
        if (rho) rho[l] = dg[(size_t)l * 8 + 0];
        if (T) T[l] = dg[(size_t)l * 8 + 1];
        if (TP) TP[l] = dg[(size_t)l * 8 + 2];
    }
    return LBM_OK;
}

void lbm_destroy(lbm_handle* h) {
    if (!h) return;
    if (h->graph_exec) hipGraphExecDestroy(h->graph_exec);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    delete h;
}

namespace {

// Plain streaming copy: every thread moves four 16-byte vectors, consecutive threads consecutive
// vectors (the yardstick of the achievable read + write bandwidth).
__global__ void __launch_bounds__(256) k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    long long n4) {
    const long long base = (long long)blockIdx.x * (256 * 4) + threadIdx.x;
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + k * 256;
        if (i < n4) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + k * 256;
        if (i < n4) dst[i] = v[k];
    }
}

}  // namespace

int lbm_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return LBM_E_INVAL;
    const long long n4 = (long long)(bytes / 16);
    if (n4 == 0) return LBM_OK;
    const long long blocks = (n4 + 1023) / 1024;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

const char* lbm_last_error(lbm_handle* h) { return h ? h->err.c_str() : g_init_error.c_str(); }

}  // extern "C"

int lbmib::step_handle(lbm_handle* h, int n, bool want_resid) { return run_steps(h, n, nullptr, want_resid); }

int lbmib::residual_handle(lbm_handle* h) {
    hipError_t e = dispatch(h, [&](auto L, auto S) {
        using LT = decltype(L);
        using ST = decltype(S);
        return launch_residual<LT, ST>(h->args, other<ST>(h), current<ST>(h), h->d.partials, residual_parts(h->N),
                                       h->d.resid, h->stream);
    });
    if (e != hipSuccess) return fail(h, LBM_E_HIP, std::string("residual: ") + hipGetErrorString(e));
    return LBM_OK;
}
