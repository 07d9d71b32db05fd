"""Seeded synthetic inputs: marker geometries and flow parameters of the benchmark workloads.

This module holds input generation only (body shapes, marker placement, the
conversion of Mach/Reynolds numbers to lattice units, seeds). It contains none
of the time step's arithmetic. Both the HIP path and the CPU checker are fed
from it.

Lattice units: dx = dt = 1, R = c_s^2 = 1/3, temperatures in units of T_ref.
The paper fixes Delta x / Delta s = 1 (markers about one cell apart, Sec. 2.4),
gamma = 1.4 (Sec. 3.4); the Prandtl number is not given and is taken as 0.71.
"""
from dataclasses import dataclass, field
import math

import numpy as np

R_GAS = 1.0 / 3.0
GAMMA = 1.4
PRANDTL = 0.71

METHOD_DIBM, METHOD_FODIBM, METHOD_FODIBM_R = 0, 1, 2
KERNEL_COS, KERNEL_ROMA3 = 0, 1
T_NONE, T_DIRICHLET, T_NEUMANN = 0, 1, 2


def cylinder_markers(center, radius, m):
    """X_l = c + R (cos 2 pi l/m, sin 2 pi l/m) with outward normals."""
    t = 2.0 * np.pi * np.arange(m) / m
    n = np.stack([np.cos(t), np.sin(t)], axis=1)
    return np.asarray(center, dtype=np.float64)[None, :] + radius * n, n


def sphere_markers(center, radius, m):
    """Fibonacci lattice on the sphere: z_l = 1 - (2l+1)/m, azimuth l * golden angle."""
    l = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * l + 1.0) / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ga = np.pi * (3.0 - np.sqrt(5.0))
    phi = ga * l
    n = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    return np.asarray(center, dtype=np.float64)[None, :] + radius * n, n


def ellipse_markers(center, a, b, angle, m, dense=20000):
    """m markers at equal arc length on an ellipse (semi-axes a, b, rotated by angle)."""
    t = np.linspace(0.0, 2.0 * np.pi, dense + 1)
    px, py = a * np.cos(t), b * np.sin(t)
    seg = np.hypot(np.diff(px), np.diff(py))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    target = s[-1] * np.arange(m) / m
    tm = np.interp(target, s, t)
    x, y = a * np.cos(tm), b * np.sin(tm)
    nx_, ny_ = b * np.cos(tm), a * np.sin(tm)          # outward normal of the unrotated ellipse
    nn = np.hypot(nx_, ny_)
    nx_, ny_ = nx_ / nn, ny_ / nn
    ca, sa = math.cos(angle), math.sin(angle)
    X = np.stack([center[0] + ca * x - sa * y, center[1] + sa * x + ca * y], axis=1)
    n = np.stack([ca * nx_ - sa * ny_, sa * nx_ + ca * ny_], axis=1)
    return X, n


def ellipse_perimeter(a, b, dense=20000):
    t = np.linspace(0.0, 2.0 * np.pi, dense + 1)
    return float(np.hypot(np.diff(a * np.cos(t)), np.diff(b * np.sin(t))).sum())


def star_markers(center, r0, dr, m):
    """Five-point star of Eq. (39): r = r0 + dr cos(5 t), normals from the tangent."""
    t = 2.0 * np.pi * np.arange(m) / m
    r = r0 + dr * np.cos(5 * t)
    drdt = -5 * dr * np.sin(5 * t)
    x, y = r * np.cos(t), r * np.sin(t)
    tx, ty = drdt * np.cos(t) - r * np.sin(t), drdt * np.sin(t) + r * np.cos(t)
    nn = np.hypot(tx, ty)
    n = np.stack([ty / nn, -tx / nn], axis=1)
    return np.stack([center[0] + x, center[1] + y], axis=1), n


def flow_units(mach, reynolds, ref_len, T_inf, rho_inf=1.0, gamma=GAMMA, prandtl=PRANDTL):
    """Free-stream speed, viscosity and conductivity in lattice units.

    u = Ma sqrt(gamma R T_inf); mu = rho u L / Re; lambda = mu Cp / Pr.
    """
    u = mach * math.sqrt(gamma * R_GAS * T_inf)
    mu = rho_inf * u * ref_len / reynolds
    cp = gamma * R_GAS / (gamma - 1.0)
    return u, mu, mu * cp / prandtl


# Choice of the reference temperature T_ref (theta = T / T_ref), which the paper leaves free to set
# the CFL number of the scheme. Three bounds on theta_inf = T_inf / T_ref:
#   * the rest population of Eq. (A.3) stays positive with margin where the gas is hottest (the
#     wall, or the stagnation temperature): theta <= THETA_HOT;
#   * the free-stream lattice speed u_inf = Ma sqrt(gamma theta_inf / 3) stays below U_LIMIT: the
#     linearised hybrid step becomes unstable near |u| = 0.31-0.35 whatever theta, sigma or the
#     readings of Eq. (A.9) (von Neumann analysis of the step; a short-wave energy mode along the
#     stream), and flow round a body is faster than the free stream;
#   * the conduction number kappa = lambda / (rho Cv) = gamma u_inf L / (Pr Re) stays below
#     KAPPA_LIMIT (explicit conduction in the energy update).
# theta_inf is the largest value that meets all three, and at most 1. A floor comes from the
# equilibrium itself: its upstream populations stay positive only while theta exceeds about
# 3 |u| (about 4.2 Ma^2 with u = Ma sqrt(gamma theta / 3)), and runs below it diverged from the
# impulsive start; theta_inf must stay above THETA_FLOOR_MA2 Ma^2, or the flow is refused
# (ValueError). With the velocity bound this leaves no theta for Ma above about 0.45.
THETA_HOT = 1.2
U_LIMIT = 0.21
KAPPA_LIMIT = 0.1
THETA_FLOOR_MA2 = 5.0


def lattice_temperature(mach, reynolds, ref_len, T_wall_ratio=None, gamma=GAMMA, prandtl=PRANDTL,
                        u_limit=None, kappa_limit=None):
    """theta_inf = T_inf / T_ref for the flow (see the bounds above); T_wall_ratio None means an
    adiabatic wall, whose hottest point is the stagnation temperature."""
    u_limit = U_LIMIT if u_limit is None else u_limit
    kappa_limit = KAPPA_LIMIT if kappa_limit is None else kappa_limit
    hot = 1.0 + 0.5 * (gamma - 1.0) * mach * mach
    if T_wall_ratio is not None:
        hot = max(hot, T_wall_ratio)
    theta = min(1.0, THETA_HOT / hot)
    cs_unit = math.sqrt(gamma * R_GAS)                       # sound speed at theta = 1
    u_cap = u_limit
    u_cap = min(u_cap, kappa_limit * prandtl * reynolds / (gamma * ref_len))
    theta = min(theta, (u_cap / (mach * cs_unit)) ** 2)
    if theta < THETA_FLOOR_MA2 * mach * mach:
        raise ValueError(f'no reference temperature for Ma {mach:.3f}, Re {reynolds:.1f}, L {ref_len:.1f}: '
                         f'theta_inf {theta:.3f} below the floor {THETA_FLOOR_MA2 * mach * mach:.3f}')
    return theta


def reference_temperatures(T_wall_ratio, mach=None, reynolds=None, ref_len=None):
    """(T_inf, T_w) in units of T_ref. With the flow given, T_ref follows lattice_temperature; the
    older rule T_ref = (T_inf + T_w)/2 is kept when it is not."""
    if mach is None:
        t_inf = 2.0 / (1.0 + T_wall_ratio)
    else:
        t_inf = lattice_temperature(mach, reynolds, ref_len, T_wall_ratio)
    return t_inf, T_wall_ratio * t_inf


@dataclass
class Case:
    """One flow problem: grid, gas, free stream and the immersed body."""
    name: str
    dim: int
    dims: tuple
    mu: float
    lam: float
    u_inf: tuple
    T_inf: float
    rho_inf: float = 1.0
    gamma: float = GAMMA
    sigma: float = 0.98
    bc: str = 'inflow_outflow'          # 'periodic', 'inflow_outflow' or 'characteristic' (x closure)
    sigma_c: float = 0.25               # characteristic outlet: relaxation of the incoming wave
    X: np.ndarray = None
    n: np.ndarray = None
    u_wall: np.ndarray = None
    t_kind: np.ndarray = None
    t_value: np.ndarray = None
    method: int = METHOD_FODIBM_R
    kernel: int = KERNEL_COS
    ref_len: float = 1.0
    ref_area: float = 1.0
    surface: float = 1.0
    T_wall: float = 1.0
    steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(np.prod(self.dims))

    @property
    def u_ref(self):
        return float(np.linalg.norm(self.u_inf))


def _markers_common(X, n, t_kind, t_value):
    m = len(X)
    return dict(X=X, n=n, u_wall=np.zeros_like(X), t_kind=np.full(m, t_kind, dtype=np.int32),
                t_value=np.full(m, t_value, dtype=np.float64))


def rotation_wall_velocity(X, center, omega):
    """Wall velocity of a body turning at angular velocity omega about the z axis through
    center: u = omega e_z x (X - c), the first two components in 2D."""
    X = np.asarray(X, dtype=np.float64)
    u = np.zeros_like(X)
    u[:, 0] = -omega * (X[:, 1] - center[1])
    u[:, 1] = omega * (X[:, 0] - center[0])
    return u


def cylinder_case(nx=200, ny=100, center=(60.0, 50.0), diameter=20.0, markers=63, mach=0.2,
                  reynolds=40.0, T_wall_ratio=1.2, method=METHOD_FODIBM_R, kernel=KERNEL_COS, steps=1000,
                  omega_star=0.0):
    """2D cylinder, no-slip: D2Q9, 200 x 100, D = 20 at (60, 50), 63 markers. Isothermal wall
    (T_w = T_wall_ratio T_inf) or, with T_wall_ratio None, adiabatic (theta_inf = 1). With
    omega_star the cylinder turns counter-clockwise at omega = 2 omega_star |u_inf| / D, i.e. its
    surface moves at omega_star |u_inf|."""
    if T_wall_ratio is None:
        T_inf = lattice_temperature(mach, reynolds, diameter)
        T_w, kind, tv = T_inf, T_NEUMANN, 0.0
    else:
        T_inf, T_w = reference_temperatures(T_wall_ratio, mach, reynolds, diameter)
        kind, tv = T_DIRICHLET, T_w
    u, mu, lam = flow_units(mach, reynolds, diameter, T_inf)
    X, n = cylinder_markers(center, diameter / 2.0, markers)
    mk = _markers_common(X, n, kind, tv)
    if omega_star:
        mk['u_wall'] = rotation_wall_velocity(X, center, 2.0 * omega_star * u / diameter)
    return Case(name='cylinder2d', dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u, 0.0), T_inf=T_inf,
                method=method, kernel=kernel, ref_len=diameter, ref_area=diameter,
                surface=math.pi * diameter, T_wall=T_w, steps=steps,
                extra={'omega_star': omega_star}, **mk)


def sphere_case(nx=384, ny=192, nz=192, diameter=32.0, center=None, mach=0.3, reynolds=100.0,
                T_wall_ratio=None, method=METHOD_FODIBM_R, steps=5000, markers=None, omega_star=0.0):
    """3D sphere: adiabatic (T_wall_ratio None, theta_inf = 1) or isothermal wall. With
    omega_star it turns about the z axis at omega = 2 omega_star |u_inf| / D (Sec. 4, rotating
    sphere: the equator moves at omega_star |u_inf|)."""
    if center is None:
        center = (0.3 * nx, ny / 2.0, nz / 2.0)
    if T_wall_ratio is None:
        T_inf = lattice_temperature(mach, reynolds, diameter)
        T_w, kind, tv = T_inf, T_NEUMANN, 0.0
    else:
        T_inf, T_w = reference_temperatures(T_wall_ratio, mach, reynolds, diameter)
        kind, tv = T_DIRICHLET, T_w
    u, mu, lam = flow_units(mach, reynolds, diameter, T_inf)
    m = markers if markers is not None else int(round(math.pi * diameter * diameter))
    X, n = sphere_markers(center, diameter / 2.0, m)
    mk = _markers_common(X, n, kind, tv)
    if omega_star:
        mk['u_wall'] = rotation_wall_velocity(X, center, 2.0 * omega_star * u / diameter)
    return Case(name='sphere3d', dim=3, dims=(nx, ny, nz), mu=mu, lam=lam, u_inf=(u, 0.0, 0.0),
                T_inf=T_inf, method=method, ref_len=diameter, ref_area=math.pi * diameter ** 2 / 4,
                surface=math.pi * diameter ** 2, T_wall=T_w, steps=steps,
                extra={'omega_star': omega_star}, **mk)


def taylor_couette_case(scale=1, method=METHOD_FODIBM_R, speed=0.04, nu=0.048, r_in=8.0, r_out=20.0):
    """Circular Couette flow between an inner cylinder of radius r_in*scale turning at surface
    speed `speed` and a fixed outer cylinder of radius r_out*scale (fluid in the gap), both walls
    isothermal at T_inf = 1, periodic box at rest, no free stream. Markers one per unit of arc;
    inner normals point outward, outer normals inward (into the fluid). The steady solution is
    u_theta = A r + B / r with u_theta(r1) = speed, u_theta(r2) = 0."""
    r1, r2 = r_in * scale, r_out * scale
    n = int(2 * math.ceil(r2 + 6.0))
    c = (n / 2.0 + 0.31, n / 2.0 - 0.23)
    m1, m2 = int(round(2 * math.pi * r1)), int(round(2 * math.pi * r2))
    X1, n1 = cylinder_markers(c, r1, m1)
    X2, n2o = cylinder_markers(c, r2, m2)
    X = np.concatenate([X1, X2])
    nrm = np.concatenate([n1, -n2o])
    mk = _markers_common(X, nrm, T_DIRICHLET, 1.0)
    mk['u_wall'] = np.concatenate([rotation_wall_velocity(X1, c, speed / r1), np.zeros_like(X2)])
    gamma = GAMMA
    lam = nu * (R_GAS * gamma / (gamma - 1.0)) / PRANDTL
    case = Case(name='taylor_couette', dim=2, dims=(n, n), mu=nu, lam=lam, u_inf=(0.0, 0.0), T_inf=1.0,
                bc='periodic', method=method, ref_len=2.0 * r1, ref_area=2.0 * r1, surface=2 * math.pi * r1,
                T_wall=1.0, steps=1, extra=dict(center=c, r1=r1, r2=r2, speed=speed, n_inner=m1), **mk)
    return case


def couette_profile(case, r):
    """Analytic u_theta(r) of taylor_couette_case."""
    r1, r2, U = case.extra['r1'], case.extra['r2'], case.extra['speed']
    A = -U * r1 / (r2 * r2 - r1 * r1)
    B = U * r1 * r2 * r2 / (r2 * r2 - r1 * r1)
    return A * r + B / r


def config1(**kw):
    """200 x 100 D2Q9 cylinder D = 20 at (60, 50), 63 markers, Ma 0.2, Re 40, T_w = 1.2 T_inf."""
    return cylinder_case(**kw)


def config2(reynolds=100.0, **kw):
    """384 x 192 x 192 D3Q19, sphere D = 32, 3217 markers, adiabatic, Ma 0.3, Re 100-300."""
    return sphere_case(reynolds=reynolds, **kw)


def config3(**kw):
    """512 x 256 x 256 D3Q19, sphere D = 32, isothermal T_w = 1.5 T_inf, Ma 0.5, Re 300."""
    kw.setdefault('nx', 512)
    kw.setdefault('ny', 256)
    kw.setdefault('nz', 256)
    return sphere_case(mach=0.5, reynolds=300.0, T_wall_ratio=1.5, **kw)


def precision_case(nx=512, ny=256, nz=256, center=None):
    """The precision study as run: the 512 x 256 x 256 sphere (D = 32) with an isothermal wall at
    T_w = 1.2 T_inf, Ma 0.2, Re 300 (the recipe's Ma 0.5 / T_w = 1.5 T_inf diverges within 50
    steps from the impulsive start in this scheme, on the oracle as on the GPU)."""
    return sphere_case(nx=nx, ny=ny, nz=nz, center=center, mach=0.2, reynolds=300.0, T_wall_ratio=1.2)


def _refined_temperatures(mach, reynolds, fine_len, T_wall_ratio):
    """(T_inf, T_w, thermal kind, value) with the temperature rule applied on the fine level, where
    the body spans twice the coarse nodes and the conduction number is twice the coarse one."""
    if T_wall_ratio is None:
        T_inf = lattice_temperature(mach, reynolds, fine_len)
        return T_inf, T_inf, T_NEUMANN, 0.0
    T_inf, T_w = reference_temperatures(T_wall_ratio, mach, reynolds, fine_len)
    return T_inf, T_w, T_DIRICHLET, T_w


def refined_cylinder(nx=120, ny=64, origin=(24, 12), block=(40, 40), diameter=10.0, center=None, mach=0.2,
                     reynolds=40.0, T_wall_ratio=None, bc='inflow_outflow', method=METHOD_FODIBM_R, steps=1):
    """2D cylinder of `diameter` coarse cells inside a refined block: the coarse grid nx x ny
    (no body; closure bc along x), and a block of block[a] coarse cells at coarse node `origin`
    whose fine grid has twice the resolution and holds the body (2 diameter nodes across, about one
    marker per fine node of perimeter). Re on the diameter; the free-stream temperature is chosen
    for the fine level. Returns (coarse case, fine case, origin); the fine case has doubled mu and
    lambda, periodic closure, and marker positions in fine lattice units."""
    if center is None:
        center = (origin[0] + 0.35 * block[0] + 0.23, origin[1] + 0.5 * block[1] + 0.17)
    Df = 2.0 * diameter
    T_inf, T_w, kind, tv = _refined_temperatures(mach, reynolds, Df, T_wall_ratio)
    u, mu, lam = flow_units(mach, reynolds, diameter, T_inf)
    coarse = Case(name='refined_cylinder_coarse', dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u, 0.0),
                  T_inf=T_inf, bc=bc, method=method, ref_len=diameter, ref_area=diameter,
                  surface=math.pi * diameter, T_wall=T_w, steps=steps)
    cf = (2.0 * (center[0] - origin[0]), 2.0 * (center[1] - origin[1]))
    X, n = cylinder_markers(cf, Df / 2.0, int(round(math.pi * Df)))
    fine = Case(name='refined_cylinder_fine', dim=2, dims=(2 * block[0], 2 * block[1]), mu=2.0 * mu,
                lam=2.0 * lam, u_inf=(u, 0.0), T_inf=T_inf, bc='periodic', method=method, ref_len=Df,
                ref_area=Df, surface=math.pi * Df, T_wall=T_w, steps=steps, **_markers_common(X, n, kind, tv))
    return coarse, fine, tuple(origin)


def refined_sphere(nx=48, ny=32, nz=32, origin=(10, 6, 6), block=(20, 20, 20), diameter=6.0, center=None,
                   mach=0.2, reynolds=50.0, T_wall_ratio=None, bc='inflow_outflow', method=METHOD_FODIBM_R,
                   markers=None, steps=1):
    """3D analogue of refined_cylinder: a sphere of `diameter` coarse cells in a refined block
    (markers: about pi (2 diameter)^2 unless given)."""
    if center is None:
        center = (origin[0] + 0.4 * block[0] + 0.23, origin[1] + 0.5 * block[1] + 0.17,
                  origin[2] + 0.5 * block[2] - 0.11)
    Df = 2.0 * diameter
    T_inf, T_w, kind, tv = _refined_temperatures(mach, reynolds, Df, T_wall_ratio)
    u, mu, lam = flow_units(mach, reynolds, diameter, T_inf)
    coarse = Case(name='refined_sphere_coarse', dim=3, dims=(nx, ny, nz), mu=mu, lam=lam, u_inf=(u, 0.0, 0.0),
                  T_inf=T_inf, bc=bc, method=method, ref_len=diameter, ref_area=math.pi * diameter ** 2 / 4,
                  surface=math.pi * diameter ** 2, T_wall=T_w, steps=steps)
    cf = tuple(2.0 * (center[a] - origin[a]) for a in range(3))
    m = markers if markers is not None else int(round(math.pi * Df * Df))
    X, n = sphere_markers(cf, Df / 2.0, m)
    fine = Case(name='refined_sphere_fine', dim=3, dims=tuple(2 * b for b in block), mu=2.0 * mu, lam=2.0 * lam,
                u_inf=(u, 0.0, 0.0), T_inf=T_inf, bc='periodic', method=method, ref_len=Df,
                ref_area=math.pi * Df ** 2 / 4, surface=math.pi * Df ** 2, T_wall=T_w, steps=steps,
                **_markers_common(X, n, kind, tv))
    return coarse, fine, tuple(origin)


def nested_cylinder(nx=64, ny=40, origins=((14, 8), (6, 6)), blocks=((28, 24), (22, 18)), diameter=2.5,
                    center=(14 + (6 + 11.15) / 2.0, 8 + (6 + 9.1) / 2.0), mach=0.2, reynolds=40.0,
                    T_wall_ratio=None, bc='inflow_outflow', method=METHOD_FODIBM_R, steps=1):
    """2D cylinder of `diameter` level-0 cells at level-0 position `center` inside nested refined
    blocks: block k (k = 1 .. L) has blocks[k-1] cells of level k-1 at level k-1 node
    origins[k-1] and twice its resolution; the body is on the finest level (2^L diameter nodes
    across, about one marker per node of perimeter). Re on the diameter; the free-stream
    temperature is chosen for the finest level. Returns (cases, origins): cases[0] is the coarse
    grid without body, cases[k] level k (mu and lambda 2^k times the coarse ones, periodic), the
    markers of the last in its own lattice units."""
    L = len(blocks)
    scale = 2 ** L
    T_inf, T_w, kind, tv = _refined_temperatures(mach, reynolds, scale * diameter, T_wall_ratio)
    u, mu, lam = flow_units(mach, reynolds, diameter, T_inf)
    cases = [Case(name='nested_cylinder_0', dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u, 0.0), T_inf=T_inf,
                  bc=bc, method=method, ref_len=diameter, ref_area=diameter, surface=math.pi * diameter,
                  T_wall=T_w, steps=steps)]
    c = tuple(center)
    for k in range(1, L + 1):
        c = tuple(2.0 * (c[a] - origins[k - 1][a]) for a in range(2))
        f = 2 ** k
        dk = f * diameter
        case = Case(name=f'nested_cylinder_{k}', dim=2, dims=(2 * blocks[k - 1][0], 2 * blocks[k - 1][1]), mu=f * mu,
                    lam=f * lam, u_inf=(u, 0.0), T_inf=T_inf, bc='periodic', method=method, ref_len=dk, ref_area=dk,
                    surface=math.pi * dk, T_wall=T_w, steps=steps)
        if k == L:
            X, n = cylinder_markers(c, dk / 2.0, int(round(math.pi * dk)))
            for key, v in _markers_common(X, n, kind, tv).items():
                setattr(case, key, v)
        cases.append(case)
    return cases, tuple(tuple(o) for o in origins)


def acoustic_pulse(nx=160, ny=4, u_inf=0.1, amp=1e-3, x0=60.0, width=6.0, mu=0.005, bc='characteristic',
                   sigma_c=0.0):
    """A plane right-running isentropic pressure pulse on a stream along x (2D, no body, periodic
    in y): p' = amp exp(-(x - x0)^2 / (2 width^2)), u' = p'/(rho c), rho' = p'/c^2 about
    (rho, T) = (1, 1), c^2 = gamma R T. Returns the case and its fields rho [ny, nx],
    u [2, ny, nx], T [ny, nx]; it tests how much of an outgoing wave an outlet closure reflects."""
    c = math.sqrt(GAMMA * R_GAS)
    x = np.arange(nx, dtype=np.float64)
    dp = amp * np.exp(-0.5 * ((x - x0) / width) ** 2)
    rho1 = 1.0 + dp / c ** 2
    u1 = u_inf + dp / c
    T1 = (R_GAS + dp) / (rho1 * R_GAS)
    lam = mu * (GAMMA * R_GAS / (GAMMA - 1.0)) / PRANDTL
    case = Case(name='pulse', dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u_inf, 0.0), T_inf=1.0, bc=bc,
                sigma_c=sigma_c, ref_len=1.0, steps=1)
    rho = np.tile(rho1, (ny, 1))
    u = np.stack([np.tile(u1, (ny, 1)), np.zeros((ny, nx))])
    T = np.tile(T1, (ny, 1))
    return case, rho, u, T


def conduction_number(case):
    """kappa = lambda / (rho C_v) in lattice units: the explicit conduction update of the energy
    equation needs kappa well below 1/(2D)."""
    cv = R_GAS / (case.gamma - 1.0)
    return case.lam / (case.rho_inf * cv)


def batched_cases(count=64, seed0=1000, steps=2000, m_lo=64, m_hi=256, kappa_max=0.11, isothermal=False):
    """Uneven 2D ellipse cases: M ~ U{m_lo..m_hi} (64..256), nx = 4M, ny = nx/2, aspect U[1,4],
    angle U[0,90 deg], Ma U[0.1,0.5], Re U[20,200] on L = 2a, adiabatic no-slip wall (isothermal:
    T_w U[1,1.5] T_inf, drawn in either case). T_ref follows lattice_temperature; (Ma, Re) pairs
    it refuses (no admissible T_ref, Ma above about 0.45) or whose conduction number exceeds
    kappa_max are drawn again."""
    cases = []
    for s in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + s))
        m = int(rng.integers(m_lo, m_hi + 1))
        aspect = rng.uniform(1.0, 4.0)
        angle = math.radians(rng.uniform(0.0, 90.0))
        tw = rng.uniform(1.0, 1.5)
        while True:
            mach = rng.uniform(0.1, 0.5)
            re = rng.uniform(20.0, 200.0)
            try:
                c = ellipse_case(m, aspect, angle, mach, re, tw if isothermal else None, steps=steps,
                                 name=f'batch{s}')
            except ValueError:
                continue
            if conduction_number(c) <= kappa_max:
                break
        cases.append(c)
    return cases


def learned_cases(count, seed0=0, nx=256, ny=128, m=64, mach=(0.05, 0.15), reynolds=(15.0, 35.0),
                  kappa_max=0.11, shape='ellipse'):
    """Cases of the learned warm start: one body of perimeter m on nx x ny, seed s drawn from
    PCG64(seed0 + s), adiabatic no-slip wall, T_inf = T_ref, Ma and Re uniform in the given ranges
    (redrawn while the conduction number exceeds kappa_max).
      shape 'ellipse': aspect U[1,4], angle U[0,90 deg];
      shape 'star': 5-point star of Eq. (39) with dr/D U[0,0.1], angle U[0,72 deg];
      shape 'mixed': even seeds ellipses, odd seeds stars."""
    cases = []
    for s in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + s))
        kind = shape if shape != 'mixed' else ('ellipse' if (seed0 + s) % 2 == 0 else 'star')
        if kind == 'ellipse':
            aspect = rng.uniform(1.0, 4.0)
            angle = math.radians(rng.uniform(0.0, 90.0))
        elif kind == 'star':
            dr_D = rng.uniform(0.0, 0.1)
            angle = math.radians(rng.uniform(0.0, 72.0))
        else:
            raise ValueError(f'unknown shape {shape}')
        while True:
            ma = rng.uniform(*mach)
            re = rng.uniform(*reynolds)
            if kind == 'ellipse':
                c = ellipse_case(m, aspect, angle, ma, re, None, nx=nx, ny=ny, name=f'learn{seed0 + s}', t_ref='unit')
            else:
                c = star_case(m, dr_D, angle, ma, re, None, nx=nx, ny=ny, name=f'star{seed0 + s}', t_ref='unit')
            if conduction_number(c) <= kappa_max:
                break
        cases.append(c)
    return cases


def star_perimeter(r0, dr, dense=20000):
    t = 2.0 * np.pi * np.arange(dense) / dense
    r = r0 + dr * np.cos(5 * t)
    drdt = -5 * dr * np.sin(5 * t)
    return float(np.sum(np.hypot(r, drdt)) * 2.0 * np.pi / dense)


def star_case(m, dr_over_D, angle, mach, reynolds, T_wall_ratio=None, steps=2000, name='star', nx=None, ny=None,
              t_ref='rule'):
    """Five-point star of Eq. (39) (r = r0 + dr cos 5t, D = 2 r0, dr = dr_over_D D) of perimeter
    m dx with m markers, turned by angle, centre (0.3 nx, 0.5 ny), no-slip wall; walls as in
    ellipse_case. Re and Ma are based on D."""
    nx = nx if nx is not None else 4 * m
    ny = ny if ny is not None else nx // 2
    r0 = m / star_perimeter(1.0, 2.0 * dr_over_D)       # perimeter scales with r0
    dr = 2.0 * dr_over_D * r0
    D = 2.0 * r0
    if T_wall_ratio is None:
        T_inf = T_w = lattice_temperature(mach, reynolds, D) if t_ref == 'rule' else 1.0
        kind, value = T_NEUMANN, 0.0
    else:
        T_inf, T_w = reference_temperatures(T_wall_ratio, mach, reynolds, D)
        kind, value = T_DIRICHLET, T_w
    u, mu, lam = flow_units(mach, reynolds, D, T_inf)
    c0 = (0.3 * nx, 0.5 * ny)
    X0, n0 = star_markers((0.0, 0.0), r0, dr, m)
    ca, sa = math.cos(angle), math.sin(angle)
    rot = np.array([[ca, -sa], [sa, ca]])
    X = X0 @ rot.T + np.array(c0)
    n = n0 @ rot.T
    return Case(name=name, dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u, 0.0), T_inf=T_inf,
                ref_len=D, ref_area=D, surface=m, T_wall=T_w, steps=steps,
                extra=dict(r0=r0, dr=dr, angle=angle, mach=mach, reynolds=reynolds, center=c0, shape='star'),
                **_markers_common(X, n, kind, value))


def ellipse_case(m, aspect, angle, mach, reynolds, T_wall_ratio=None, steps=2000, name='ellipse',
                 nx=None, ny=None, t_ref='rule'):
    """Ellipse of perimeter m dx (one marker per cell), centre (0.3 nx, 0.5 ny), no-slip wall.
    T_wall_ratio None: adiabatic wall (dT/dn = 0) and T_inf = 1; otherwise an isothermal wall at
    T_wall_ratio T_inf with T_ref = (T_inf + T_w)/2."""
    nx = nx if nx is not None else 4 * m
    ny = ny if ny is not None else nx // 2
    # perimeter(a, a/aspect) = m  ->  scale a unit-major ellipse
    per1 = ellipse_perimeter(1.0, 1.0 / aspect)
    a = m / per1
    b = a / aspect
    if T_wall_ratio is None:
        T_inf = T_w = lattice_temperature(mach, reynolds, 2.0 * a) if t_ref == 'rule' else 1.0
        kind, value = T_NEUMANN, 0.0
    else:
        T_inf, T_w = reference_temperatures(T_wall_ratio, mach, reynolds, 2.0 * a)
        kind, value = T_DIRICHLET, T_w
    u, mu, lam = flow_units(mach, reynolds, 2.0 * a, T_inf)
    X, n = ellipse_markers((0.3 * nx, 0.5 * ny), a, b, angle, m)
    return Case(name=name, dim=2, dims=(nx, ny), mu=mu, lam=lam, u_inf=(u, 0.0), T_inf=T_inf,
                ref_len=2.0 * a, ref_area=2.0 * a, surface=m, T_wall=T_w, steps=steps,
                extra=dict(a=a, b=b, angle=angle, mach=mach, reynolds=reynolds, center=(0.3 * nx, 0.5 * ny)),
                **_markers_common(X, n, kind, value))


def random_state_perturbation(case, seed, amp_rho=1e-3, amp_u=None, amp_T=1e-3):
    """Smooth seeded perturbation fields (rho, u, T) around the free stream, for parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = tuple(case.dims[::-1])
    D = case.dim
    amp_u = amp_u if amp_u is not None else 0.05 * max(case.u_ref, 0.01)

    def smooth():
        a = rng.standard_normal(grid)
        for ax in range(D):
            a = (np.roll(a, 1, ax) + 2 * a + np.roll(a, -1, ax)) / 4.0
        return a / max(np.abs(a).max(), 1e-300)

    rho = case.rho_inf * (1.0 + amp_rho * smooth())
    u = np.stack([case.u_inf[a] + amp_u * smooth() for a in range(D)])
    T = case.T_inf * (1.0 + amp_T * smooth())
    return rho, u, T


def init_params(shapes, seed):
    """Seeded initial parameters of a convolutional network, flat in layer order: per layer
    (cin, cout, taps) the weights [cout][taps][cin] drawn N(0, 2 / (taps cin)) (N(0, 1 / cin) for
    the last layer) and zero biases [cout]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for k, (ci, co, t) in enumerate(shapes):
        std = math.sqrt((1.0 if k == len(shapes) - 1 else 2.0) / (t * ci))
        parts.append(rng.standard_normal(co * t * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)
