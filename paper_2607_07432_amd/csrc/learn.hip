// Grid-side pieces of the learned warm start (2D): the network input planes of a case (signed
// distance to the body, flow parameters, body indicator), the normalised steady fields used as
// training targets, and the warm start itself: the equilibrium of the denormalised prediction
// (Eq. (A.3)) plus the second-order non-equilibrium part that the finite-difference branch of
// Eq. (A.7) assigns to its velocity field, Pi = -rho c_s^2 tau_bar (grad u + grad u^T - div u I),
// so that the first collision sees the viscous stress of the prediction.
//
// Normalisation, with Ma = |u_inf| / sqrt(gamma R T_inf):
//   t0 = (rho - rho_inf) / (rho_inf Ma^2), t1 = u_x / |u_inf|, t2 = u_y / |u_inf|,
//   t3 = (T - T_inf) / (T_inf Ma^2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "handle.hpp"

using namespace lbmib;

namespace {

constexpr int TPB = 256;

// Signed distance from node n to the polygon of markers, taken as the distance to the nearest
// marker, positive on the side its outward normal points to (the nearest-marker normal test
// that also defines the interior nodes of the geometry precompute).
__global__ void __launch_bounds__(TPB) k_learn_input(int nx, int ny, int m, const double* __restrict__ X,
                                                     const double* __restrict__ nrm, double sdf_scale, double ma_n,
                                                     double re_n, float* __restrict__ out) {
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= (long long)nx * ny) return;
    const double x = (double)(n % nx), y = (double)(n / nx);
    double best = 1e300;
    int lb = -1;
    for (int l = 0; l < m; ++l) {
        const double dx = x - X[2 * l], dy = y - X[2 * l + 1];
        const double d2 = dx * dx + dy * dy;
        if (d2 < best) {
            best = d2;
            lb = l;
        }
    }
    double sdf = 0.0;
    int inside = 0;
    if (lb >= 0) {
        const double s = (x - X[2 * lb]) * nrm[2 * lb] + (y - X[2 * lb + 1]) * nrm[2 * lb + 1];
        inside = s < 0.0;
        sdf = inside ? -sqrt(best) : sqrt(best);
    }
    out[4 * n + 0] = (float)(sdf / sdf_scale);
    out[4 * n + 1] = (float)ma_n;
    out[4 * n + 2] = (float)re_n;
    out[4 * n + 3] = inside ? 1.f : 0.f;
}

__global__ void __launch_bounds__(TPB) k_learn_norm(long long N, const double* __restrict__ rho, const double* __restrict__ u,
                                                    const double* __restrict__ T, double rho_inf, double u_ref, double T_inf,
                                                    double ma2, float* __restrict__ out) {
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    out[4 * n + 0] = (float)((rho[n] - rho_inf) / (rho_inf * ma2));
    out[4 * n + 1] = (float)(u[n] / u_ref);
    out[4 * n + 2] = (float)(u[N + n] / u_ref);
    out[4 * n + 3] = (float)((T[n] - T_inf) / (T_inf * ma2));
}

__global__ void __launch_bounds__(TPB) k_learn_denorm(long long N, const float* __restrict__ pred, double rho_inf,
                                                      double u_ref, double T_inf, double ma2, double* __restrict__ rho,
                                                      double* __restrict__ u, double* __restrict__ T) {
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    rho[n] = rho_inf * (1.0 + ma2 * (double)pred[4 * n + 0]);
    u[n] = u_ref * (double)pred[4 * n + 1];
    u[N + n] = u_ref * (double)pred[4 * n + 2];
    T[n] = T_inf * (1.0 + ma2 * (double)pred[4 * n + 3]);
}

// f_i += w_i H_i : Pi / (2 c_s^4) with Pi = -rho c_s^2 tau_bar S (D2Q9, periodic central differences).
template <class S>
__global__ void __launch_bounds__(TPB) k_learn_neq(int nx, int ny, const double* __restrict__ rho,
                                                   const double* __restrict__ u, double mu, S* __restrict__ f) {
    const long long N = (long long)nx * ny;
    const long long n = (long long)blockIdx.x * TPB + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx), y = (int)(n / nx);
    const int xp = x + 1 < nx ? x + 1 : 0, xm = x > 0 ? x - 1 : nx - 1;
    const int yp = y + 1 < ny ? y + 1 : 0, ym = y > 0 ? y - 1 : ny - 1;
    const double* ux = u;
    const double* uy = u + N;
    const long long e = (long long)y * nx + xp, w = (long long)y * nx + xm;
    const long long nn = (long long)yp * nx + x, s = (long long)ym * nx + x;
    const double dxx = 0.5 * (ux[e] - ux[w]), dxy = 0.5 * (ux[nn] - ux[s]);   // d u_x / d x, d u_x / d y
    const double dyx = 0.5 * (uy[e] - uy[w]), dyy = 0.5 * (uy[nn] - uy[s]);
    const double div = dxx + dyy;
    const double cs2 = 1.0 / 3.0;
    const double r = rho[n];
    const double coef = r * cs2 * (mu / (r * cs2) + 0.5);
    const double P00 = -coef * (2.0 * dxx - div), P11 = -coef * (2.0 * dyy - div), P01 = -coef * (dxy + dyx);
#pragma unroll
    for (int i = 0; i < D2Q9::Q; ++i) {
        const double cx = D2Q9::c[i][0], cy = D2Q9::c[i][1];
        const double h = (cx * cx - cs2) * P00 + 2.0 * cx * cy * P01 + (cy * cy - cs2) * P11;
        f[i * N + n] = S((double)f[i * N + n] + D2Q9::w[i] * h / (2.0 * cs2 * cs2));
    }
}

int lfail(lbm_handle* h, int code, const std::string& m) {
    h->err = m;
    return code;
}

double u_ref_of(const lbm_handle* h) { return std::sqrt(h->p.u_inf[0] * h->p.u_inf[0] + h->p.u_inf[1] * h->p.u_inf[1]); }

double mach2_of(const lbm_handle* h) {
    const double c2 = h->p.gamma * (1.0 / 3.0) * h->p.T_inf;
    const double u = u_ref_of(h);
    return u * u / c2;
}

}  // namespace

extern "C" {

int lbm_learn_input(lbm_handle* h, double sdf_scale, double ma_n, double re_n, float* d_out) {
    if (!h || !d_out) return LBM_E_INVAL;
    if (h->D != 2) return lfail(h, LBM_E_INVAL, "the learned warm start is 2D");
    if (!(sdf_scale > 0.0)) return lfail(h, LBM_E_INVAL, "sdf_scale must be positive");
    const int m = h->markers_set ? h->geom.m : 0;
    hipLaunchKernelGGL(k_learn_input, dim3((unsigned)((h->N + TPB - 1) / TPB)), dim3(TPB), 0, h->stream, h->p.nx, h->p.ny,
                       m, (const double*)h->d.Xm, (const double*)h->d.nm, sdf_scale, ma_n, re_n, d_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lfail(h, LBM_E_HIP, std::string("learn_input: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_learn_target(lbm_handle* h, float* d_out) {
    if (!h || !d_out) return LBM_E_INVAL;
    if (h->D != 2) return lfail(h, LBM_E_INVAL, "the learned warm start is 2D");
    const double ur = u_ref_of(h);
    if (!(ur > 0.0)) return lfail(h, LBM_E_INVAL, "needs a nonzero free stream");
    const long long N = h->N;
    double* rho = (double*)h->d.work;      // 4 N doubles fit in the working area
    double* u = rho + N;
    double* T = u + 2 * N;
    const int rc = lbm_fields(h, LBM_F64, 1, rho, u, T, nullptr);
    if (rc != LBM_OK) return rc;
    hipLaunchKernelGGL(k_learn_norm, dim3((unsigned)((N + TPB - 1) / TPB)), dim3(TPB), 0, h->stream, N,
                       (const double*)rho, (const double*)u, (const double*)T, h->p.rho_inf, ur, h->p.T_inf, mach2_of(h),
                       d_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lfail(h, LBM_E_HIP, std::string("learn_target: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_learn_warm_start(lbm_handle* h, const float* d_pred) {
    if (!h || !d_pred) return LBM_E_INVAL;
    if (h->D != 2) return lfail(h, LBM_E_INVAL, "the learned warm start is 2D");
    const double ur = u_ref_of(h);
    if (!(ur > 0.0)) return lfail(h, LBM_E_INVAL, "needs a nonzero free stream");
    const long long N = h->N;
    double* rho = (double*)h->d.work;
    double* u = rho + N;
    double* T = u + 2 * N;
    hipLaunchKernelGGL(k_learn_denorm, dim3((unsigned)((N + TPB - 1) / TPB)), dim3(TPB), 0, h->stream, N, d_pred,
                       h->p.rho_inf, ur, h->p.T_inf, mach2_of(h), rho, u, T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lfail(h, LBM_E_HIP, std::string("learn_warm_start: ") + hipGetErrorString(e));
    const int rc = lbm_set_fields(h, 1, rho, u, T);
    if (rc != LBM_OK) return rc;
    // the current state is A when cur == 0
    void* fcur = h->cur == 0 ? h->d.fA : h->d.fB;
    const unsigned g = (unsigned)((N + TPB - 1) / TPB);
    if (h->p.precision == LBM_F64)
        hipLaunchKernelGGL(k_learn_neq<double>, dim3(g), dim3(TPB), 0, h->stream, h->p.nx, h->p.ny, (const double*)rho,
                           (const double*)u, h->p.mu, (double*)fcur);
    else
        hipLaunchKernelGGL(k_learn_neq<float>, dim3(g), dim3(TPB), 0, h->stream, h->p.nx, h->p.ny, (const double*)rho,
                           (const double*)u, h->p.mu, (float*)fcur);
    const hipError_t e2 = hipGetLastError();
    if (e2 == hipSuccess) {
        const hipError_t e3 = hipStreamSynchronize(h->stream);
        if (e3 != hipSuccess) return lfail(h, LBM_E_HIP, std::string("learn_warm_start: ") + hipGetErrorString(e3));
        return LBM_OK;
    }
    return lfail(h, LBM_E_HIP, std::string("learn_warm_start: ") + hipGetErrorString(e2));
}

}  // extern "C"
