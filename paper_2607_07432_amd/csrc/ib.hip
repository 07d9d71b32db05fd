// Immersed-boundary kernels: marker interpolation + target reconstruction + forces,
// atomic-free spreading through the node -> marker CSR, boundary errors and loads.
// All marker arithmetic is FP64 whatever the storage precision of the populations.
#include "kernels.hpp"

namespace lbmib {

namespace {

constexpr int WAVE = 64;
constexpr double D_PB = 1.5;   // d_n = d_PB = 1.5 dx (Sec. 2.3)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

// Predicted (force-free) variables at a node: rho, j, u* = j/rho, T* from rho E (Sec. 2.5 step 1).
template <class L, class S>
__device__ __forceinline__ void predicted(const SweepArgs& a, StateP<S> A, long long n, double& rho, double* j,
                                          double* u, double& T) {
    const long long N = a.grid.N;
    double drho = 0;
    j[0] = j[1] = j[2] = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double f = double(A.f[i * N + n]);
        drho += f;
#pragma unroll
        for (int b = 0; b < L::D; ++b)
            if (L::c[i][b]) j[b] += L::c[i][b] * f;
    }
    rho = 1.0 + drho;
    double uu = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        u[b] = j[b] / rho;
        uu += u[b] * u[b];
    }
    T = ((double(A.e[n]) + a.fs.e_ref) / rho - 0.5 * uu) / a.gas.Cv;
}

}  // namespace

// One wavefront per marker: Eqs. (14)/(12) interpolation, Eqs. (27)/(29) reconstruction,
// Eqs. (20)-(22)/(30)-(32) forces.
template <class L, class S>
__device__ __forceinline__ void marker_forces(const SweepArgs& a, const MarkersP& mk, StateP<S> A, int l, int lane) {
    constexpr int D = L::D;
    const double phi = mk.phi[l];
    double* G = mk.G + (long long)l * (D + 2);
    double* dg = mk.diag + (long long)l * 8;
    if (phi <= 0.0) {
        if (lane < D + 2) G[lane] = 0.0;
        if (lane < 8) dg[lane] = 0.0;
        return;
    }
    // One-sided (or two-sided for DIBM, phi = 1) interpolation of rho, j, u*, T*.
    double sr = 0, sj[3] = {0, 0, 0}, su[3] = {0, 0, 0}, sT = 0;
    for (long long e = mk.supp_ptr[l] + lane; e < mk.supp_ptr[l + 1]; e += WAVE) {
        double r, j[3], u[3], T;
        predicted<L, S>(a, A, mk.supp_node[e], r, j, u, T);
        const double w = mk.supp_w[e];
        sr += w * r;
        sT += w * T;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            sj[b] += w * j[b];
            su[b] += w * u[b];
        }
    }
    // Projection point: two-sided, d = 1.
    double pu[3] = {0, 0, 0}, pT = 0;
    for (long long e = mk.proj_ptr[l] + lane; e < mk.proj_ptr[l + 1]; e += WAVE) {
        double r, j[3], u[3], T;
        predicted<L, S>(a, A, mk.proj_node[e], r, j, u, T);
        const double w = mk.proj_w[e];
        pT += w * T;
#pragma unroll
        for (int b = 0; b < D; ++b) pu[b] += w * u[b];
    }
    sr = wave_sum(sr);
    sT = wave_sum(sT);
    pT = wave_sum(pT);
#pragma unroll
    for (int b = 0; b < D; ++b) {
        sj[b] = wave_sum(sj[b]);
        su[b] = wave_sum(su[b]);
        pu[b] = wave_sum(pu[b]);
    }
    if (lane != 0) return;
    const double rl = phi * sr, Tl = phi * sT;
    double jl[3], ul[3], ut[3], ub[3];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        jl[b] = phi * sj[b];
        ul[b] = phi * su[b];
        ub[b] = mk.u_wall[(long long)l * D + b];
    }
    const int kind = mk.t_kind[l];
    const double tv = mk.t_value[l];
    double Tt;
    if (mk.method == 2) {
        const double ratio = mk.dbv[l] / D_PB;
#pragma unroll
        for (int b = 0; b < D; ++b) ut[b] = ub[b] - ratio * (pu[b] - ub[b]);          // Eq. (27)
        if (kind == 1)
            Tt = tv - ratio * (pT - tv);                                                 // Eq. (27)
        else if (kind == 2)
            Tt = pT - tv * (D_PB + mk.dbv[l]);                                           // Eq. (29)
        else
            Tt = Tl;
    } else {
#pragma unroll
        for (int b = 0; b < D; ++b) ut[b] = ub[b];
        Tt = kind == 1 ? tv : (kind == 2 ? pT - tv * D_PB : Tl);
    }
    double ut2 = 0, ul2 = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        G[b] = 2.0 * (rl * ut[b] - jl[b]);                                               // Eqs. (20)/(30)
        ut2 += ut[b] * ut[b];
        ul2 += ul[b] * ul[b];
    }
    G[D] = rl * (ut2 - ul2) / 2.0;                                                       // Eqs. (21)/(31)
    G[D + 1] = kind != 0 ? a.gas.Cv * rl * (Tt - Tl) : 0.0;                              // Eqs. (22)/(32)
    dg[0] = rl;
    dg[1] = Tl;
    dg[2] = pT;
#pragma unroll
    for (int b = 0; b < 3; ++b) dg[3 + b] = b < D ? pu[b] : 0.0;
    dg[6] = Tt;
    dg[7] = 0.0;
}

template <class L, class S>
__global__ void __launch_bounds__(WAVE) k_markers(SweepArgs a, MarkersP mk, StateP<S> A) {
    marker_forces<L, S>(a, mk, A, blockIdx.x, threadIdx.x);
}

// Batch: one wavefront per marker of any case; the case is found from the marker numbering.
template <class L, class S>
__global__ void __launch_bounds__(WAVE) k_markers_batch(const CaseDesc<S>* __restrict__ cases, int ncases, int g) {
    const int l = blockIdx.x;
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (cases[mid].marker0 <= l) lo = mid; else hi = mid - 1;
    }
    const CaseDesc<S>& cd = cases[lo];
    const int cur = (cd.cur0 + g) & 1;
    marker_forces<L, S>(cd.a[cur], cd.mk, cd.st[cur], l - cd.marker0, threadIdx.x);
}

// Eq. (15): g_i = sum_k s_ik G_k over the CSR row r of node i. A group of SPREAD_LANES
// consecutive lanes shares a row (rows hold ~13 entries on the sphere, at most 24): lane j sums
// the entries j, j + SPREAD_LANES, ... in order, then the group adds its partial sums in a fixed
// butterfly, so the result does not depend on scheduling. Every lane of the group takes part in
// the exchange (valid = false for lanes past the last row); lane 0 stores.
constexpr int SPREAD_LANES = 8;

__device__ __forceinline__ void spread_row(int dim, const MarkersP& mk, const RowsP& rows, int r, int j, bool valid) {
    double f[3] = {0, 0, 0}, e = 0;
    if (valid) {
        for (long long k = mk.row_ptr[r] + j; k < mk.row_ptr[r + 1]; k += SPREAD_LANES) {
            const double s = mk.col_s[k];
            const double* G = mk.G + mk.col_marker[k] * (dim + 2);
            for (int b = 0; b < dim; ++b) f[b] += s * G[b];
            e += s * (G[dim] + G[dim + 1]);
        }
    }
#pragma unroll
    for (int m = SPREAD_LANES / 2; m > 0; m >>= 1) {
#pragma unroll
        for (int b = 0; b < 3; ++b) f[b] += __shfl_xor(f[b], m, SPREAD_LANES);
        e += __shfl_xor(e, m, SPREAD_LANES);
    }
    if (valid && j == 0) {
        for (int b = 0; b < dim; ++b) rows.fib[(long long)b * rows.nrows + r] = f[b];
        rows.fE[r] = e;
    }
}

// SPREAD_LANES lanes per forced node.
__global__ void __launch_bounds__(256) k_spread(int dim, MarkersP mk, RowsP rows) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int r = (int)(t / SPREAD_LANES);
    spread_row(dim, mk, rows, r, (int)(t % SPREAD_LANES), r < rows.nrows);
}

template <class S>
__global__ void __launch_bounds__(256) k_spread_batch(const CaseDesc<S>* __restrict__ cases, int ncases, int total,
                                                      int dim) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int r = (int)(t / SPREAD_LANES);
    const bool valid = r < total;
    int lo = 0, hi = ncases - 1;
    const int rs = valid ? r : total - 1;             // lanes past the end search a real row
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (cases[mid].row0 <= rs) lo = mid; else hi = mid - 1;
    }
    const CaseDesc<S>& cd = cases[lo];
    spread_row(dim, cd.mk, cd.a[0].rows, rs - cd.row0, (int)(t % SPREAD_LANES), valid);
}

// Boundary errors of Eqs. (35), (36), (38) at each marker from the current fields.
template <class L, class S>
__global__ void __launch_bounds__(WAVE) k_eps(SweepArgs a, MarkersP mk, StateP<S> A, double u_ref, double T_inf,
                                              double ref_len) {
    constexpr int D = L::D;
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    double* ep = mk.eps + (long long)l * 4;
    if (mk.phi[l] <= 0.0) {
        if (lane < 4) ep[lane] = 0.0;
        return;
    }
    double su[3] = {0, 0, 0}, sT = 0, pT = 0;
    for (long long e = mk.tw_ptr[l] + lane; e < mk.tw_ptr[l + 1]; e += WAVE) {
        double r, j[3], u[3], T;
        predicted<L, S>(a, A, mk.tw_node[e], r, j, u, T);
        const double w = mk.tw_w[e];
        sT += w * T;
#pragma unroll
        for (int b = 0; b < D; ++b) su[b] += w * u[b];
    }
    for (long long e = mk.proj_ptr[l] + lane; e < mk.proj_ptr[l + 1]; e += WAVE) {
        double r, j[3], u[3], T;
        predicted<L, S>(a, A, mk.proj_node[e], r, j, u, T);
        pT += mk.proj_w[e] * T;
    }
    sT = wave_sum(sT);
    pT = wave_sum(pT);
#pragma unroll
    for (int b = 0; b < D; ++b) su[b] = wave_sum(su[b]);
    if (lane != 0) return;
    double d2 = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const double d = su[b] - mk.u_wall[(long long)l * D + b];
        d2 += d * d;
    }
    const int kind = mk.t_kind[l];
    const double tv = mk.t_value[l];
    ep[0] = sqrt(d2) / u_ref;
    ep[1] = kind == 2 ? fabs((pT - sT) / D_PB - tv) / (T_inf / ref_len) : 0.0;
    ep[2] = kind == 1 ? fabs(sT - tv) / tv : 0.0;
    ep[3] = kind == 1 ? 5.0 : (kind == 2 ? 3.0 : 1.0);   // bit 0 dir, bit 1 neu, bit 2 iso
}

// Deterministic FP64 block reduction of the loads over markers (fixed tree order).
// out: F[3], Q, sum_dir, n_dir, sum_neu, n_neu, sum_iso, n_iso, n_inactive.
__global__ void __launch_bounds__(256) k_loads(int dim, MarkersP mk, double* out) {
    __shared__ double red[11][256];
    double acc[11];
    for (int q = 0; q < 11; ++q) acc[q] = 0.0;
    for (int l = threadIdx.x; l < mk.m; l += 256) {
        const double W = mk.W[l];
        if (mk.phi[l] <= 0.0) {
            acc[10] += 1.0;
            continue;
        }
        const double* G = mk.G + (long long)l * (dim + 2);
        for (int b = 0; b < dim; ++b) acc[b] -= G[b] * W;
        acc[3] += G[dim + 1] * W;
        const double* ep = mk.eps + (long long)l * 4;
        const int mask = (int)ep[3];
        if (mask & 1) {
            acc[4] += ep[0];
            acc[5] += 1.0;
        }
        if (mask & 2) {
            acc[6] += ep[1];
            acc[7] += 1.0;
        }
        if (mask & 4) {
            acc[8] += ep[2];
            acc[9] += 1.0;
        }
    }
    for (int q = 0; q < 11; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 11; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 11) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_rowmap(const long long* rows, int nrows, int* rowmap) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < nrows) rowmap[rows[r]] = r;
}

hipError_t launch_rowmap(const long long* rows, int nrows, int* rowmap, hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowmap, dim3((nrows + 255) / 256), dim3(256), 0, st, rows, nrows, rowmap);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_markers(const SweepArgs& a, const MarkersP& mk, StateP<S> A, hipStream_t st) {
    if (mk.m <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_markers<L, S>), dim3(mk.m), dim3(WAVE), 0, st, a, mk, A);
    return hipGetLastError();
}

hipError_t launch_spread(int dim, const MarkersP& mk, RowsP rows, hipStream_t st) {
    if (rows.nrows <= 0) return hipSuccess;
    const long long lanes = (long long)rows.nrows * SPREAD_LANES;
    hipLaunchKernelGGL(k_spread, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, dim, mk, rows);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_eps(const SweepArgs& a, const MarkersP& mk, StateP<S> A, double u_ref, double T_inf,
                      double ref_len, hipStream_t st) {
    if (mk.m <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_eps<L, S>), dim3(mk.m), dim3(WAVE), 0, st, a, mk, A, u_ref, T_inf, ref_len);
    return hipGetLastError();
}

hipError_t launch_loads(int dim, const MarkersP& mk, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_loads, dim3(1), dim3(256), 0, st, dim, mk, out);
    return hipGetLastError();
}

template <class L, class S>
hipError_t launch_markers_batch(const CaseDesc<S>* cases, int ncases, int total_markers, int g, hipStream_t st) {
    if (total_markers <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_markers_batch<L, S>), dim3(total_markers), dim3(WAVE), 0, st, cases, ncases, g);
    return hipGetLastError();
}

template <class S>
hipError_t launch_spread_batch(const CaseDesc<S>* cases, int ncases, int total_rows, int dim, hipStream_t st) {
    if (total_rows <= 0) return hipSuccess;
    const long long lanes = (long long)total_rows * SPREAD_LANES;
    hipLaunchKernelGGL((k_spread_batch<S>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, cases, ncases,
                       total_rows, dim);
    return hipGetLastError();
}

template hipError_t launch_markers_batch<D2Q9, float>(const CaseDesc<float>*, int, int, int, hipStream_t);
template hipError_t launch_markers_batch<D2Q9, double>(const CaseDesc<double>*, int, int, int, hipStream_t);
template hipError_t launch_spread_batch<float>(const CaseDesc<float>*, int, int, int, hipStream_t);
template hipError_t launch_spread_batch<double>(const CaseDesc<double>*, int, int, int, hipStream_t);

#define LBMIB_INST_IB(L, S)                                                                                    \
    template hipError_t launch_markers<L, S>(const SweepArgs&, const MarkersP&, StateP<S>, hipStream_t);       \
    template hipError_t launch_eps<L, S>(const SweepArgs&, const MarkersP&, StateP<S>, double, double, double, \
                                         hipStream_t);

LBMIB_INST_IB(D2Q9, float)
LBMIB_INST_IB(D2Q9, double)
LBMIB_INST_IB(D3Q19, float)
LBMIB_INST_IB(D3Q19, double)

}  // namespace lbmib
