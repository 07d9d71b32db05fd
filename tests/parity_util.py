"""Shared helpers of the GPU-vs-oracle parity tests (oracle side in FP64 on the CPU)."""
import numpy as np

from oracle import ib as oib
from oracle import lbm as olbm
from oracle.lattice import for_dim
from paper_2607_07432_amd import workloads as wl


def oracle_params(case, with_aC=True):
    u = tuple(case.u_inf) + (0.0,) * (3 - len(case.u_inf))
    return olbm.Params(mu=case.mu, lam=case.lam, gamma=case.gamma, sigma=case.sigma, rho_inf=case.rho_inf,
                       u_inf=u[:case.dim], T_inf=case.T_inf, bc=case.bc, with_aC=with_aC, sigma_c=case.sigma_c)


def oracle_geometry(case):
    return oib.build_geometry(case.dims, case.X, case.n, case.method, case.kernel)


def oracle_markers(case):
    return oib.Markers(u_wall=case.u_wall, t_kind=case.t_kind, t_value=case.t_value)


def oracle_step(case, st, geom=None, mk=None, with_aC=True):
    lat = for_dim(case.dim)
    prm = oracle_params(case, with_aC)
    mf = None
    if geom is not None:
        fib, fE, mf = oib.ib_step_forcing(lat, prm, geom, mk, st)
    else:
        fib = fE = None
    return olbm.lbm_step(lat, prm, st, fib, fE), mf


def random_state(case, geom, seed, neq=1e-3, hist=1e-4):
    """Smooth random fields around the free stream with off-equilibrium content and history.

    Off-diagonal force history is placed only on the forced nodes, as the scheme produces it.
    """
    lat = for_dim(case.dim)
    prm = oracle_params(case)
    rho, u, T = wl.random_state_perturbation(case, seed)
    st = olbm.state_from_fields(lat, prm, rho, u, T)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    D = case.dim
    grid = rho.shape
    st.f = st.f + neq * rng.standard_normal(st.f.shape) * lat.w.reshape((-1,) + (1,) * D)
    H2 = hist * rng.standard_normal((D, D) + grid)
    H2 = 0.5 * (H2 + H2.transpose((1, 0) + tuple(range(2, H2.ndim))))
    H2 -= np.eye(D).reshape((D, D) + (1,) * D) * sum(H2[a, a] for a in range(D)) / D
    mask = np.zeros(int(np.prod(grid)), dtype=bool)
    if geom is not None and len(geom.rows):
        mask[geom.rows] = True
    mask = mask.reshape(grid)
    for a in range(D):
        for b in range(D):
            if a != b:
                H2[a, b] = np.where(mask, H2[a, b], 0.0)
    st.H2 = H2
    return st


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def small_sphere_case(method=wl.METHOD_FODIBM_R, T_wall_ratio=None, dims=(28, 22, 20), D=8.0, reynolds=50.0,
                      mach=0.3, markers=None, omega_star=0.0):
    nx, ny, nz = dims
    return wl.sphere_case(nx=nx, ny=ny, nz=nz, diameter=D, center=(0.4 * nx + 0.23, ny / 2 + 0.17, nz / 2 - 0.11),
                          mach=mach, reynolds=reynolds, T_wall_ratio=T_wall_ratio, method=method, steps=1,
                          markers=markers, omega_star=omega_star)
