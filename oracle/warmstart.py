"""FP64 reference of the grid-side pieces of the learned warm start (2D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * signed distance of node (x, y) to the body: the distance to the nearest marker (lowest index
    on ties), negative when (x - X_l) . n_l < 0 for that marker, the same nearest-marker normal
    test that defines the closed interior of the geometry precompute (Sec. 2.3 as read);
  * network input planes {SDF / sdf_scale, ma_n, re_n, body indicator};
  * normalised fields with Ma = |u_inf| / sqrt(gamma R T_inf):
    {(rho - rho_inf)/(rho_inf Ma^2), u_x/|u_inf|, u_y/|u_inf|, (T - T_inf)/(T_inf Ma^2)}
    and the inverse map used for the warm start;
  * the warm-start state: equilibrium populations of the denormalised fields (Eq. (A.3)) plus
    w_i H_i : Pi / (2 c_s^4) with Pi = -rho c_s^2 tau_bar S(u), S the deviatoric strain of the
    finite-difference branch of Eq. (A.7) (tau_bar = mu / (rho c_s^2) + 1/2).
The paper has no warm start; parity is pinned by closed forms (circle distance, free stream)
and round trips in the tests.
"""
import numpy as np

R_GAS = 1.0 / 3.0


def signed_distance(nx, ny, X, n):
    """[ny, nx] signed distance and body indicator from markers X, normals n ([m, 2])."""
    ys, xs = np.mgrid[0:ny, 0:nx].astype(np.float64)
    best = np.full((ny, nx), np.inf)
    arg = np.zeros((ny, nx), dtype=np.int64)
    for l in range(len(X)):
        d2 = (xs - X[l, 0]) ** 2 + (ys - X[l, 1]) ** 2
        better = d2 < best
        best = np.where(better, d2, best)
        arg = np.where(better, l, arg)
    s = (xs - X[arg, 0]) * n[arg, 0] + (ys - X[arg, 1]) * n[arg, 1]
    inside = s < 0.0
    sdf = np.where(inside, -np.sqrt(best), np.sqrt(best))
    return sdf, inside


def input_planes(nx, ny, X, n, sdf_scale, ma_n, re_n):
    sdf, inside = signed_distance(nx, ny, X, n)
    out = np.zeros((ny, nx, 4))
    out[..., 0] = sdf / sdf_scale
    out[..., 1] = ma_n
    out[..., 2] = re_n
    out[..., 3] = inside
    return out


def mach2(u_inf, T_inf, gamma):
    u2 = float(np.dot(u_inf, u_inf))
    return u2 / (gamma * R_GAS * T_inf)


def normalise(rho, u, T, rho_inf, u_inf, T_inf, gamma):
    """rho, T [ny, nx], u [2, ny, nx] -> [ny, nx, 4]."""
    ur = float(np.linalg.norm(u_inf))
    m2 = mach2(u_inf, T_inf, gamma)
    out = np.zeros(rho.shape + (4,))
    out[..., 0] = (rho - rho_inf) / (rho_inf * m2)
    out[..., 1] = u[0] / ur
    out[..., 2] = u[1] / ur
    out[..., 3] = (T - T_inf) / (T_inf * m2)
    return out


def denormalise(pred, rho_inf, u_inf, T_inf, gamma):
    """[ny, nx, 4] -> rho, u [2, ny, nx], T."""
    ur = float(np.linalg.norm(u_inf))
    m2 = mach2(u_inf, T_inf, gamma)
    rho = rho_inf * (1.0 + m2 * pred[..., 0])
    u = np.stack([ur * pred[..., 1], ur * pred[..., 2]])
    T = T_inf * (1.0 + m2 * pred[..., 3])
    return rho, u, T


def warm_state(lat, prm, rho, u, T):
    """Populations f-bar of the warm start (2D): Eq. (A.3) plus the second-order part."""
    from oracle import lbm as olbm
    D, cs2 = lat.D, lat.cs2
    feq = olbm.equilibrium(lat, rho, u, T)
    du = olbm.central_gradient(u, D)
    div = sum(du[a, a] for a in range(D))
    eye = np.eye(D).reshape((D, D) + (1,) * rho.ndim)
    strain = du + du.transpose((1, 0) + tuple(range(2, du.ndim))) - (2.0 / D) * eye * div
    taubar = prm.mu / (rho * cs2) + 0.5
    Pi = -rho * cs2 * taubar * strain
    w = lat.w.reshape((-1,) + (1,) * rho.ndim)
    return feq + w * np.einsum('iab,ab...->i...', lat.h2, Pi) / (2 * cs2 ** 2)
