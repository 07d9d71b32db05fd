// Batch of independent 2D grids stepped together: one launch per kernel for all cases
// (marker forces, spreading, persistent fused sweep), replayed from captured HIP graphs.
// Each case keeps its own handle (state, body, loads); the batch only adds a device table
// of case descriptors and the residual partial sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"

using namespace lbmib;

namespace lbmib {

namespace {

constexpr int RTPB = 256;
constexpr int PART_LEN = 16 * RTPB;   // nodes per residual partial sum

template <class S, class Key>
__device__ __forceinline__ int find_case(const CaseDesc<S>* __restrict__ cases, int ncases, int w, Key key) {
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (key(cases[mid]) <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Partial sums of |u^{n+1} - u^n|^2 and the non-finite flag over PART_LEN nodes of one case.
// g is the parity of the step just taken: its input state is the old one.
template <class L, class S>
__global__ void __launch_bounds__(RTPB) k_residual_batch(const CaseDesc<S>* __restrict__ cases, int ncases, int g,
                                                         double* partials) {
    const int p = blockIdx.x;
    const int c = find_case(cases, ncases, p, [](const CaseDesc<S>& d) { return d.part0; });
    const CaseDesc<S>& cd = cases[c];
    const int cur = (cd.cur0 + g) & 1;
    const StateP<S> Old = cd.st[cur], New = cd.st[cur ^ 1];
    const long long N = cd.a[0].grid.N;
    const long long n0 = (long long)(p - cd.part0) * cd.part_len;
    const long long n1 = n0 + cd.part_len < N ? n0 + cd.part_len : N;
    __shared__ double red[RTPB];
    __shared__ int nf[RTPB];
    double acc = 0;
    int bad = 0;
    for (long long n = n0 + threadIdx.x; n < n1; n += RTPB) {
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
        double d2 = 0;
        for (int b = 0; b < L::D; ++b) {
            const double d = j1[b] / r1 - j0[b] / r0;
            d2 += d * d;
        }
        acc += d2;
        if (!isfinite(d2) || !isfinite(double(New.e[n])) || !isfinite(r1)) bad = 1;
    }
    red[threadIdx.x] = acc;
    nf[threadIdx.x] = bad;
    __syncthreads();
    for (int s = RTPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x] += red[threadIdx.x + s];
            nf[threadIdx.x] |= nf[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * p] = red[0];
        partials[2 * p + 1] = nf[0] ? 1.0 : 0.0;
    }
}

// One workgroup per case: fixed-order sum of its partials into the case's residual slot.
template <class S>
__global__ void __launch_bounds__(RTPB) k_residual_batch_final(const CaseDesc<S>* __restrict__ cases,
                                                               const double* partials) {
    const CaseDesc<S>& cd = cases[blockIdx.x];
    __shared__ double red[RTPB];
    __shared__ double nf[RTPB];
    double acc = 0, bad = 0;
    for (int k = threadIdx.x; k < cd.nparts; k += RTPB) {
        acc += partials[2 * (cd.part0 + k)];
        bad = fmax(bad, partials[2 * (cd.part0 + k) + 1]);
    }
    red[threadIdx.x] = acc;
    nf[threadIdx.x] = bad;
    __syncthreads();
    for (int s = RTPB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x] += red[threadIdx.x + s];
            nf[threadIdx.x] = fmax(nf[threadIdx.x], nf[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cd.resid[0] = sqrt(red[0]) * cd.resid_scale;
        cd.resid[1] = (nf[0] > 0.0 || !isfinite(red[0])) ? 1.0 : 0.0;
    }
}

// out[c] = residual of case c, NaN if its state held a non-finite value.
template <class S>
__global__ void k_gather_resid(const CaseDesc<S>* __restrict__ cases, int ncases, double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncases) return;
    const double* r = cases[c].resid;
    out[c] = r[1] != 0.0 ? __builtin_nan("") : r[0];
}

}  // namespace

template <class S>
hipError_t launch_gather_resid(const CaseDesc<S>* cases, int ncases, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_gather_resid<S>), dim3((ncases + 255) / 256), dim3(256), 0, st, cases, ncases, out);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_residual_batch(const CaseDesc<S>* cases, int ncases, int total_parts, double* partials, int g,
                                 hipStream_t st) {
    if (total_parts <= 0 || ncases <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_residual_batch<L, S>), dim3(total_parts), dim3(RTPB), 0, st, cases, ncases, g, partials);
    hipLaunchKernelGGL((k_residual_batch_final<S>), dim3(ncases), dim3(RTPB), 0, st, cases, (const double*)partials);
    return hipGetLastError();
}

template hipError_t launch_residual_batch<D2Q9, float>(const CaseDesc<float>*, int, int, double*, int, hipStream_t);
template hipError_t launch_residual_batch<D2Q9, double>(const CaseDesc<double>*, int, int, double*, int, hipStream_t);

}  // namespace lbmib

struct lbm_batch {
    std::vector<lbm_handle*> hs;
    int precision = 0;
    hipStream_t stream = nullptr;      // the stream of every case handle
    hipStream_t cap = nullptr;         // private stream the graphs are captured on
    char* desc = nullptr;              // device table of CaseDesc
    double* partials = nullptr;
    double* resid = nullptr;           // [ncases] gathered residuals
    int total_items = 0, total_markers = 0, total_rows = 0, total_parts = 0;
    int tx = 62, chunk = 32, grid = 0;
    int gpar = 0;                      // parity of the next batch step
    std::vector<int> cur0, version;
    hipGraphExec_t step_exec[2] = {nullptr, nullptr};   // one step at parity g
    hipGraphExec_t pair_exec[2] = {nullptr, nullptr};   // steps at parities g, g ^ 1
    std::vector<char> host_desc;
    std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(lbm_batch* b, int code, const std::string& msg) {
    if (b)
        b->err = msg;
    else
        g_batch_error = msg;
    return code;
}

#define BCHK(b, call)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return bfail((b), LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

size_t desc_bytes() { return sizeof(CaseDesc<double>) > sizeof(CaseDesc<float>) ? sizeof(CaseDesc<double>) : sizeof(CaseDesc<float>); }

int parts_of(long long N) { return (int)((N + PART_LEN - 1) / PART_LEN); }

int validate_cases(lbm_handle* const* hs, int n, std::string& why) {
    if (!hs || n <= 0) return why = "need at least one case", LBM_E_INVAL;
    for (int c = 0; c < n; ++c) {
        const lbm_handle* h = hs[c];
        if (!h) return why = "case " + std::to_string(c) + " is NULL", LBM_E_INVAL;
        if (h->D != 2) return why = "batches hold 2D (D2Q9) grids only", LBM_E_INVAL;
        if (h->p.bc_x == LBM_BC_CHARACTERISTIC)
            return why = "batches support the periodic and inflow/outflow closures only", LBM_E_INVAL;
        if (h->p.precision != hs[0]->p.precision) return why = "all cases must share the precision", LBM_E_INVAL;
        if (h->stream != hs[0]->stream) return why = "all cases must share one stream", LBM_E_INVAL;
        for (int k = 0; k < c; ++k)
            if (hs[k] == h) return why = "a handle appears twice", LBM_E_INVAL;
    }
    return LBM_OK;
}

// Fill the host descriptor table for tile width tx and chunk rows, and the batch totals.
template <class S>
void fill_desc(lbm_batch* b, int tx, int chunk) {
    const int n = (int)b->hs.size();
    b->host_desc.assign((size_t)n * desc_bytes(), 0);
    CaseDesc<S>* t = reinterpret_cast<CaseDesc<S>*>(b->host_desc.data());
    int items = 0, markers = 0, rows = 0, parts = 0;
    b->cur0.resize(n);
    b->version.resize(n);
    for (int c = 0; c < n; ++c) {
        lbm_handle* h = b->hs[c];
        refresh_handle_args(h);
        CaseDesc<S> d;
        std::memset(&d, 0, sizeof(d));
        d.a[0] = h->args;
        d.a[0].rows.h2off = h->d.h2off;
        d.a[0].rows.h2off_out = h->d.h2off2;
        d.a[1] = h->args;
        d.a[1].rows.h2off = h->d.h2off2;
        d.a[1].rows.h2off_out = h->d.h2off;
        d.k[0] = fused_args<S>(d.a[0]);
        d.k[1] = fused_args<S>(d.a[1]);
        d.st[0] = stateA<S>(h);
        d.st[1] = stateB<S>(h);
        d.mk = h->mk;
        const int m = h->markers_set ? h->geom.m : 0;
        const int nr = h->markers_set ? (int)h->geom.rows.size() : 0;
        d.mk.m = m;
        d.cur0 = h->cur;
        d.tiles_x = (h->p.nx + tx - 1) / tx;
        d.chunk = chunk;
        d.small = (h->p.nx <= tx || h->p.ny < 4) ? 1 : 0;
        d.item0 = items;
        for (int i = 0; i < 6; ++i) d.fb[i] = h->fbox[i];
        items += d.tiles_x * ((h->p.ny + chunk - 1) / chunk);
        d.marker0 = markers;
        markers += m;
        d.row0 = rows;
        rows += nr;
        d.part_len = PART_LEN;
        d.nparts = parts_of(h->N);
        d.part0 = parts;
        parts += d.nparts;
        const double ur = std::sqrt(h->p.u_inf[0] * h->p.u_inf[0] + h->p.u_inf[1] * h->p.u_inf[1]);
        d.resid_scale = ur > 0 ? 1.0 / (ur * std::sqrt((double)h->N)) : 1.0 / std::sqrt((double)h->N);
        d.resid = h->d.resid;
        t[c] = d;
        b->cur0[c] = h->cur;
        b->version[c] = h->geom_version;
    }
    b->total_items = items;
    b->total_markers = markers;
    b->total_rows = rows;
    b->total_parts = parts;
    b->tx = tx;
    b->chunk = chunk;
    b->gpar = 0;
}

template <class S>
const CaseDesc<S>* dtab(lbm_batch* b) {
    return reinterpret_cast<const CaseDesc<S>*>(b->desc);
}

template <class S>
int persistent_grid(int tx, int items) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    int occ = fused_batch_occupancy<D2Q9, S>(tx);
    if (occ <= 0) occ = 1;
    long long g = (long long)occ * cus;
    const long long need = ((long long)items + 7) / 8 * 8;
    if (g > need) g = need;
    g = g / 8 * 8;
    return (int)(g < 8 ? 8 : g);
}

template <class S>
hipError_t enqueue_step(lbm_batch* b, int g, hipStream_t st) {
    const int n = (int)b->hs.size();
    hipError_t e = launch_markers_batch<D2Q9, S>(dtab<S>(b), n, b->total_markers, g, st);
    if (e == hipSuccess) e = launch_spread_batch<S>(dtab<S>(b), n, b->total_rows, 2, st);
    if (e == hipSuccess) e = launch_fused_batch<D2Q9, S>(dtab<S>(b), n, b->total_items, b->tx, b->grid, g, st);
    return e;
}

void drop_graphs(lbm_batch* b) {
    for (int g = 0; g < 2; ++g) {
        if (b->step_exec[g]) (void)hipGraphExecDestroy(b->step_exec[g]);
        if (b->pair_exec[g]) (void)hipGraphExecDestroy(b->pair_exec[g]);
        b->step_exec[g] = b->pair_exec[g] = nullptr;
    }
}

template <class S>
int capture(lbm_batch* b, int g, int steps, hipGraphExec_t* out) {
    BCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < steps && e == hipSuccess; ++s) e = enqueue_step<S>(b, (g + s) & 1, b->cap);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bfail(b, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return bfail(b, LBM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
    return LBM_OK;
}

// Upload the table for (tx, chunk) and capture the step graphs.
template <class S>
int rebuild(lbm_batch* b, int tx, int chunk) {
    BCHK(b, hipStreamSynchronize(b->stream));
    fill_desc<S>(b, tx, chunk);
    b->grid = persistent_grid<S>(tx, b->total_items);
    BCHK(b, hipMemcpy(b->desc, b->host_desc.data(), b->host_desc.size(), hipMemcpyHostToDevice));
    drop_graphs(b);
    for (int g = 0; g < 2; ++g) {
        int rc = capture<S>(b, g, 1, &b->step_exec[g]);
        if (rc != LBM_OK) return rc;
        rc = capture<S>(b, g, 2, &b->pair_exec[g]);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

// Chunk length of an untuned batch at tile width 62: 32 rows, or 16 where 32-row chunks would
// leave fewer than eight work items per workgroup of the persistent grid (a small batch, such as
// the tail of cases still marching to steady state), where the shorter items balance better.
template <class S>
int untuned_chunk(lbm_batch* b) {
    fill_desc<S>(b, 62, 32);
    const long long slots = persistent_grid<S>(62, 1 << 30);
    return b->total_items >= 8 * slots ? 32 : 16;
}

template <class S>
int in_sync(lbm_batch* b) {
    for (size_t c = 0; c < b->hs.size(); ++c) {
        const lbm_handle* h = b->hs[c];
        if (h->geom_version != b->version[c] || h->cur != ((b->cur0[c] + b->gpar) & 1)) return 0;
    }
    return 1;
}

// Time the sweep alone for each tile width and chunk; it reads the current state and writes
// the other one, so repeating it leaves the state unchanged.
template <class S>
int autotune(lbm_batch* b) {
    static const int txs[] = {62, 126, 254};
    static const int chunks[] = {16, 32, 64, 128};
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    float best = 1e30f;
    int btx = b->tx, bch = b->chunk;
    int rc = LBM_OK;
    for (int tx : txs)
        for (int ch : chunks) {
            if (rc != LBM_OK) break;
            fill_desc<S>(b, tx, ch);
            const int grid = persistent_grid<S>(tx, b->total_items);
            hipError_t e = hipMemcpy(b->desc, b->host_desc.data(), b->host_desc.size(), hipMemcpyHostToDevice);
            const int n = (int)b->hs.size();
            if (e == hipSuccess)
                e = launch_fused_batch<D2Q9, S>(dtab<S>(b), n, b->total_items, tx, grid, 0, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int r = 0; r < 3 && e == hipSuccess; ++r)
                e = launch_fused_batch<D2Q9, S>(dtab<S>(b), n, b->total_items, tx, grid, 0, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = bfail(b, LBM_E_HIP, std::string("autotune: ") + hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                btx = tx;
                bch = ch;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    return rebuild<S>(b, btx, bch);
}

template <class F>
int by_precision(lbm_batch* b, F&& f) {
    if (b->precision == LBM_F64) return f(double{});
    return f(float{});
}

void after_steps(lbm_batch* b) {
    for (size_t c = 0; c < b->hs.size(); ++c) {
        lbm_handle* h = b->hs[c];
        h->cur = (b->cur0[c] + b->gpar) & 1;
        refresh_handle_args(h);
        h->stepped = 1;
        h->any_step = 1;
    }
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(lbm_handle* const* cases, int n) {
    std::string why;
    if (validate_cases(cases, n, why) != LBM_OK) return 0;
    size_t parts = 0;
    for (int c = 0; c < n; ++c) parts += (size_t)parts_of(cases[c]->N);
    return align_up((size_t)n * desc_bytes()) + align_up(2 * parts * sizeof(double)) + align_up((size_t)n * sizeof(double));
}

int lbm_batch_create(lbm_handle* const* cases, int n, void* ws, size_t bytes, int tune, lbm_batch** out) {
    if (!out) return bfail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (validate_cases(cases, n, why) != LBM_OK) return bfail(nullptr, LBM_E_INVAL, why);
    const size_t need = lbm_batch_workspace_bytes(cases, n);
    if (!ws || bytes < need)
        return bfail(nullptr, LBM_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return bfail(nullptr, LBM_E_INVAL, "workspace not 256-byte aligned");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    b->hs.assign(cases, cases + n);
    b->precision = cases[0]->p.precision;
    b->stream = cases[0]->stream;
    b->desc = (char*)ws;
    b->partials = (double*)((char*)ws + align_up((size_t)n * desc_bytes()));
    size_t parts = 0;
    for (int c = 0; c < n; ++c) parts += (size_t)parts_of(cases[c]->N);
    b->resid = (double*)((char*)b->partials + align_up(2 * parts * sizeof(double)));
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return bfail(nullptr, LBM_E_HIP, std::string("stream: ") + hipGetErrorString(e));
    }
    int rc = by_precision(b, [&](auto S) {
        using ST = decltype(S);
        return tune ? autotune<ST>(b) : rebuild<ST>(b, 62, untuned_chunk<ST>(b));
    });
    if (rc != LBM_OK) {
        g_batch_error = b->err;
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n) {
    if (!b) return LBM_E_INVAL;
    if (n < 0) return bfail(b, LBM_E_INVAL, "n < 0");
    if (n == 0) return LBM_OK;
    return by_precision(b, [&](auto S) {
        using ST = decltype(S);
        if (!in_sync<ST>(b)) {
            const int rc = rebuild<ST>(b, b->tx, b->chunk);
            if (rc != LBM_OK) return rc;
        }
        int left = n;
        while (left >= 2) {
            BCHK(b, hipGraphLaunch(b->pair_exec[b->gpar], b->stream));
            left -= 2;
        }
        if (left == 1) {
            BCHK(b, hipGraphLaunch(b->step_exec[b->gpar], b->stream));
            b->gpar ^= 1;
        }
        const hipError_t er = launch_residual_batch<D2Q9, ST>(dtab<ST>(b), (int)b->hs.size(), b->total_parts,
                                                              b->partials, b->gpar ^ 1, b->stream);
        BCHK(b, er);
        after_steps(b);
        return (int)LBM_OK;
    });
}

int lbm_batch_step_timed(lbm_batch* b, int n, double* kernel_ms) {
    if (!b || !kernel_ms) return LBM_E_INVAL;
    if (n <= 0) return bfail(b, LBM_E_INVAL, "n must be positive");
    return by_precision(b, [&](auto S) {
        using ST = decltype(S);
        if (!in_sync<ST>(b)) {
            const int rc = rebuild<ST>(b, b->tx, b->chunk);
            if (rc != LBM_OK) return rc;
        }
        const int nc = (int)b->hs.size();
        std::vector<hipEvent_t> ev((size_t)4 * n, nullptr);
        int rc = LBM_OK;
        for (auto& x : ev)
            if (hipEventCreate(&x) != hipSuccess) rc = bfail(b, LBM_E_HIP, "event create");
        hipError_t e = hipSuccess;
        for (int s = 0; s < n && rc == LBM_OK && e == hipSuccess; ++s) {
            hipEvent_t* e4 = &ev[4 * (size_t)s];
            const int g = b->gpar;
            e = hipEventRecord(e4[0], b->stream);
            if (e == hipSuccess) e = launch_markers_batch<D2Q9, ST>(dtab<ST>(b), nc, b->total_markers, g, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e4[1], b->stream);
            if (e == hipSuccess) e = launch_spread_batch<ST>(dtab<ST>(b), nc, b->total_rows, 2, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e4[2], b->stream);
            if (e == hipSuccess)
                e = launch_fused_batch<D2Q9, ST>(dtab<ST>(b), nc, b->total_items, b->tx, b->grid, g, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e4[3], b->stream);
            if (e == hipSuccess) b->gpar ^= 1;
        }
        if (rc == LBM_OK && e == hipSuccess)
            e = launch_residual_batch<D2Q9, ST>(dtab<ST>(b), nc, b->total_parts, b->partials, b->gpar ^ 1, b->stream);
        if (rc == LBM_OK && e == hipSuccess) e = hipEventSynchronize(ev.back());
        double acc[3] = {0, 0, 0};
        for (int s = 0; s < n && rc == LBM_OK && e == hipSuccess; ++s)
            for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                float ms = 0;
                e = hipEventElapsedTime(&ms, ev[4 * (size_t)s + k], ev[4 * (size_t)s + k + 1]);
                acc[k] += ms;
            }
        for (auto& x : ev)
            if (x) (void)hipEventDestroy(x);
        if (rc == LBM_OK && e != hipSuccess) rc = bfail(b, LBM_E_HIP, std::string("batch step: ") + hipGetErrorString(e));
        if (rc == LBM_OK) {
            for (int k = 0; k < 3; ++k) kernel_ms[k] = acc[k] / n;
            after_steps(b);
        }
        return rc;
    });
}

int lbm_batch_set_tile(lbm_batch* b, int tile_x, int chunk) {
    if (!b) return LBM_E_INVAL;
    if (tile_x != 62 && tile_x != 126 && tile_x != 254) return bfail(b, LBM_E_INVAL, "tile width must be 62, 126 or 254");
    if (chunk < 1) return bfail(b, LBM_E_INVAL, "chunk must be positive");
    return by_precision(b, [&](auto S) {
        using ST = decltype(S);
        return rebuild<ST>(b, tile_x, chunk);
    });
}

int lbm_batch_residuals(lbm_batch* b, double* out) {
    if (!b || !out) return LBM_E_INVAL;
    for (lbm_handle* h : b->hs)
        if (!h->any_step) return bfail(b, LBM_E_STATE, "a case has taken no step");
    const int n = (int)b->hs.size();
    return by_precision(b, [&](auto S) {
        using ST = decltype(S);
        if (!in_sync<ST>(b)) {
            const int rc = rebuild<ST>(b, b->tx, b->chunk);
            if (rc != LBM_OK) return rc;
        }
        BCHK(b, launch_gather_resid<ST>(dtab<ST>(b), n, b->resid, b->stream));
        BCHK(b, hipMemcpyAsync(out, b->resid, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        BCHK(b, hipStreamSynchronize(b->stream));
        return (int)LBM_OK;
    });
}

int lbm_batch_config(lbm_batch* b, int* cfg) {
    if (!b || !cfg) return LBM_E_INVAL;
    cfg[0] = b->tx;
    cfg[1] = b->chunk;
    cfg[2] = b->grid;
    cfg[3] = b->total_items;
    cfg[4] = b->total_markers;
    cfg[5] = b->total_rows;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

const char* lbm_batch_last_error(lbm_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
