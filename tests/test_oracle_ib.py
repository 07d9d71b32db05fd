"""Pins of the oracle's immersed-boundary geometry and operators (Secs. 2.3-2.4).

Closed forms derived from Eqs. (16), (17), (19), (25), (27); a brute-force
re-derivation of the index lists over every node of tiny grids; exact identities
of the interpolation/spreading pair.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ib
from paper_2607_07432_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), 'golden')


def test_cos_kernel_tabulated_values():
    r = np.array([0.0, 0.5, 1.0, 1.5, 2.0, -0.5, -1.5])
    v = ib.cos_kernel(r, 2.0)
    exp = [0.5, (2 + math.sqrt(2)) / 8, 0.25, (2 - math.sqrt(2)) / 8, 0.0, (2 + math.sqrt(2)) / 8,
           (2 - math.sqrt(2)) / 8]
    assert np.allclose(v, exp, rtol=0, atol=1e-16)
    assert np.allclose(ib.cos_kernel([0.0, 0.5, 1.0], 1.0), [1.0, 0.5, 0.0], rtol=0, atol=1e-16)


@pytest.mark.parametrize('d', [1.0, 2.0])
def test_cos_kernel_partition_of_unity_and_first_moment(d):
    for r in np.linspace(0.0, 0.999, 37):
        nodes = np.arange(-3, 5)
        off = nodes - r
        w = ib.cos_kernel(off, d) * (np.abs(off) < d)
        assert abs(w.sum() - 1.0) < 1e-15
        m1 = (w * off).sum()
        closed = (0.5 - r + (math.sin(math.pi * r / 2) - math.cos(math.pi * r / 2)) / 2 if d == 2.0
                  else 0.5 - r - math.cos(math.pi * r) / 2)
        assert abs(m1 - closed) < 1e-15


def test_cos_kernel_first_moment_extremes():
    rs = np.linspace(0, 1, 200001)
    m2 = 0.5 - rs + (np.sin(np.pi * rs / 2) - np.cos(np.pi * rs / 2)) / 2
    assert abs(np.abs(m2).max() - 0.0210880) < 2e-6
    m1 = 0.5 - rs - np.cos(np.pi * rs) / 2
    assert abs(np.abs(m1).max() - 0.1052568) < 2e-6


def test_roma3_partition_and_first_moment():
    for r in np.linspace(0.0, 0.999, 41):
        off = np.arange(-3, 5) - r
        w = ib.roma3_kernel(off)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((w * off).sum()) < 1e-14


def _fraction(s):
    if s == 'nan':
        return None
    if 'sqrt' in s:
        return eval(s.replace('sqrt', 'math.sqrt'))
    return float(Fraction(s))


def load_flat_wall():
    rows = []
    with open(os.path.join(GOLD, 'ib_flat_wall.txt')) as fh:
        for line in fh:
            if line.startswith('#') or not line.strip():
                continue
            name, method, off, phi, dbv, W, ratio = line.split()
            rows.append((name, method, float(off), _fraction(phi), _fraction(dbv), _fraction(W), _fraction(ratio)))
    return rows


@pytest.mark.parametrize('case', load_flat_wall(), ids=lambda c: c[0])
def test_flat_wall_worked_values(case):
    name, method, off, phi, dbv, W, ratio = case
    nx, ny, y0 = 40, 16, 8.0
    X = np.array([[float(x), y0 + off] for x in range(4, nx - 4)])
    n = np.tile([0.0, 1.0], (len(X), 1))
    m = ib.FODIBM_R if method == 'FODIBM' else ib.DIBM
    g = ib.build_geometry((nx, ny), X, n, m)
    mid = [l for l in range(len(X)) if 12 <= X[l, 0] <= nx - 13]   # away from the wall's ends
    assert np.allclose(g.phi[mid], phi, rtol=0, atol=1e-14)
    assert np.allclose(g.dBV[mid], dbv, rtol=0, atol=1e-14)
    assert np.allclose(g.W[mid], W, rtol=0, atol=1e-13)
    if ratio is not None:
        # no-slip reconstruction factor of Eq. (27): u^Vt / u^P* = -d_BV / d_PB
        assert np.allclose(-g.dBV[mid] / ib.D_N, ratio, rtol=0, atol=1e-14)


def test_linear_profile_reconstruction_exact():
    # u = a * s (s = signed distance from a straight wall on a node row): the projection point
    # sits half-way between rows, where the d = 1 kernel has zero first moment, so u^P* = 1.5 a
    # exactly and Eq. (27) returns -a d_BV, the linear profile's value at V.
    nx, ny, y0, a = 40, 16, 8.0, 0.37
    X = np.array([[float(x), y0] for x in range(4, nx - 4)])
    n = np.tile([0.0, 1.0], (len(X), 1))
    g = ib.build_geometry((nx, ny), X, n, ib.FODIBM_R)
    ys = np.repeat(np.arange(ny), nx).astype(float)
    u = np.stack([a * (ys - y0), np.zeros(nx * ny)])
    mk = ib.Markers(u_wall=np.zeros_like(X), t_kind=np.zeros(len(X), int), t_value=np.zeros(len(X)))
    rho = np.ones(nx * ny)
    T = np.ones(nx * ny)
    mf = ib.marker_forces(g, mk, _Prm(), rho, rho * u, u, T)
    mid = [l for l in range(len(X)) if 12 <= X[l, 0] <= nx - 13]
    assert np.allclose(mf['uP'][mid, 0], 1.5 * a, rtol=0, atol=1e-14)
    assert np.allclose(mf['ut'][mid, 0], -a * g.dBV[mid], rtol=0, atol=1e-14)


@pytest.mark.parametrize('method', [ib.FODIBM_R, ib.FODIBM, ib.DIBM])
def test_moving_wall_targets(method):
    # Wall sliding at U_w along x over a linear profile u = U_w + a s (Couette flow): Eq. (27)
    # extrapolates from the wall velocity, u^Vt = U_w - a d_BV (exact for the profile), while
    # FODIBM and DIBM impose u^Bt = U_w itself (Eqs. (20)-(22)); the Lagrangian force of a fluid
    # carried by the wall is then 2 rho (u^t - u*) and W^IB = rho (|u^t|^2 - |u*|^2) / 2.
    nx, ny, y0, a, Uw, rho0 = 40, 16, 8.0, 0.21, 0.05, 1.3
    X = np.array([[float(x), y0] for x in range(4, nx - 4)])
    n = np.tile([0.0, 1.0], (len(X), 1))
    g = ib.build_geometry((nx, ny), X, n, method)
    ys = np.repeat(np.arange(ny), nx).astype(float)
    u = np.stack([Uw + a * (ys - y0), np.zeros(nx * ny)])
    mk = ib.Markers(u_wall=np.tile([Uw, 0.0], (len(X), 1)), t_kind=np.zeros(len(X), int),
                    t_value=np.zeros(len(X)))
    rho = np.full(nx * ny, rho0)
    mf = ib.marker_forces(g, mk, _Prm(), rho, rho * u, u, np.ones(nx * ny))
    mid = [l for l in range(len(X)) if 12 <= X[l, 0] <= nx - 13]
    if method == ib.FODIBM_R:
        assert np.allclose(mf['uP'][mid, 0], Uw + 1.5 * a, rtol=0, atol=1e-14)
        expect = Uw - a * g.dBV[mid]
    else:
        expect = np.full(len(mid), Uw)
    assert np.allclose(mf['ut'][mid, 0], expect, rtol=0, atol=1e-14)
    assert np.allclose(mf['ut'][mid, 1], 0.0, rtol=0, atol=1e-15)
    ustar = mf['u'][mid, 0]
    assert np.allclose(mf['rho'][mid], rho0, rtol=0, atol=1e-14)
    assert np.allclose(mf['F'][mid, 0], 2 * rho0 * (expect - ustar), rtol=0, atol=1e-14)
    assert np.allclose(mf['Wib'][mid], rho0 * (expect ** 2 - ustar ** 2) / 2, rtol=0, atol=1e-14)


def test_rotating_wall_velocity():
    # omega e_z x (X - c): tangential to the circle, of magnitude omega R, counter-clockwise
    c, R, om = (30.2, 20.7), 7.0, 0.013
    X, n = wl.cylinder_markers(c, R, 40)
    u = wl.rotation_wall_velocity(X, c, om)
    assert np.allclose((u * n).sum(axis=1), 0.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(u, axis=1), om * R, rtol=1e-12)
    assert np.all(n[:, 0] * u[:, 1] - n[:, 1] * u[:, 0] > 0)
    case = wl.cylinder_case(omega_star=0.5)
    assert np.allclose(np.linalg.norm(case.u_wall, axis=1), 0.5 * case.u_ref, rtol=1e-12)


class _Prm:
    Cv = 5.0 / 6.0


def brute_geometry(dims, X, n, one_sided=True):
    """Independent re-derivation over every node of the grid (pure Python loops)."""
    D = len(dims)
    M = len(X)
    nodes = [tuple(p) for p in np.ndindex(*dims[::-1])]
    nodes = [p[::-1] for p in nodes]
    supp = {l: [] for l in range(M)}
    for p in nodes:
        inside = None
        for l in range(M):
            if all(abs(float(p[a]) - X[l][a]) < 2.0 for a in range(D)):
                if inside is None and one_sided:
                    best, bestd = 0, None
                    for k in range(M):
                        dd = 0.0
                        for a in range(D):
                            dd = dd + (float(p[a]) - X[k][a]) * (float(p[a]) - X[k][a])
                        if bestd is None or dd < bestd:
                            best, bestd = k, dd
                    dot = 0.0
                    for a in range(D):
                        dot = dot + (float(p[a]) - X[best][a]) * n[best][a]
                    inside = dot <= 0.0
                if (not one_sided) or inside:
                    lin = 0
                    for a in range(D - 1, -1, -1):
                        lin = lin * dims[a] + p[a]
                    supp[l].append(lin)
    return {l: sorted(v) for l, v in supp.items()}


@pytest.mark.parametrize('D', [2, 3])
def test_lists_match_brute_force(D):
    rng = np.random.default_rng(7 + D)
    if D == 2:
        dims = (24, 20)
        t = np.linspace(0, 2 * np.pi, 17, endpoint=False) + 0.1
        c, R = np.array([11.3, 9.7]), 4.6
        nrm = np.stack([np.cos(t), np.sin(t)], 1)
    else:
        dims = (14, 13, 12)
        m = 40
        z = 1 - (2 * np.arange(m) + 1) / m
        ph = np.arange(m) * np.pi * (3 - np.sqrt(5))
        nrm = np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
        c, R = np.array([6.6, 6.2, 5.9]), 2.9
    X = c + R * nrm + 0.01 * rng.standard_normal(nrm.shape)
    for method, one_sided in ((ib.FODIBM_R, True), (ib.DIBM, False)):
        g = ib.build_geometry(dims, X, nrm, method)
        bf = brute_geometry(dims, X.tolist(), nrm.tolist(), one_sided)
        for l in range(len(X)):
            assert sorted(g.supp_lin[l].tolist()) == bf[l]


def test_star_lists_match_brute_force():
    # the non-convex 5-point star of Eq. (39), turned by 0.4 rad
    c = wl.star_case(40, 0.1, 0.4, 0.1, 20.0, nx=28, ny=26)
    g = ib.build_geometry(c.dims, c.X, c.n, ib.FODIBM_R)
    bf = brute_geometry(c.dims, c.X.tolist(), c.n.tolist(), True)
    assert sum(len(v) for v in bf.values()) > 0
    for l in range(len(c.X)):
        assert sorted(g.supp_lin[l].tolist()) == bf[l]


def test_star_interior_equals_polar_test():
    # Candidate nodes (within a marker's support box) that lie 0.3 .. 1.4 from the surface along
    # the ray from the centre are interior exactly when r < r0 + dr cos 5t in the star's polar
    # coordinates (dense markers, so the nearest-marker test resolves the surface).
    c = wl.star_case(160, 0.1, 0.0, 0.1, 20.0, nx=80, ny=60)
    g = ib.build_geometry(c.dims, c.X, c.n, ib.FODIBM_R)
    r0, dr = c.extra['r0'], c.extra['dr']
    cx, cy = c.extra['center']
    inside = set(g.interior_lin.tolist())
    checked = 0
    for y in range(c.dims[1]):
        for x in range(c.dims[0]):
            px, py = x - cx, y - cy
            r, t = math.hypot(px, py), math.atan2(py, px)
            rs = r0 + dr * math.cos(5 * t)
            if not 0.3 < abs(r - rs) < 1.4:
                continue
            if not np.any(np.all(np.abs(c.X - np.array([x, y])) < 2.0, axis=1)):
                continue
            checked += 1
            assert ((x + c.dims[0] * y) in inside) == (r < rs)
    assert checked > 100


def test_cylinder_interior_equals_closed_disk():
    # The 63-marker cylinder D = 20 at (60, 50): nearest-marker interior test equals |x - c| <= R.
    t = 2 * np.pi * np.arange(63) / 63
    nrm = np.stack([np.cos(t), np.sin(t)], 1)
    X = np.array([60.0, 50.0]) + 10.0 * nrm
    g = ib.build_geometry((200, 100), X, nrm, ib.FODIBM_R)
    cand = np.unique(np.concatenate([ib.linear_index(ib.box_nodes(x, 2.0), (200, 100)) for x in X]))
    xs, ys = cand % 200, cand // 200
    disk = (xs - 60) ** 2 + (ys - 50) ** 2 <= 100
    assert set(g.interior_lin.tolist()) == set(cand[disk].tolist())
    assert int(((xs - 60) ** 2 + (ys - 50) ** 2 == 100).sum()) == 12


def _ring_geometry(method=ib.FODIBM_R):
    t = 2 * np.pi * np.arange(40) / 40
    nrm = np.stack([np.cos(t), np.sin(t)], 1)
    X = np.array([20.3, 19.6]) + 6.4 * nrm
    return ib.build_geometry((40, 40), X, nrm, method), X


@pytest.mark.parametrize('method', [ib.FODIBM_R, ib.DIBM])
def test_spread_conserves_total_force(method):
    # sum_i g_i = sum_l G_l W_l because phi_l sum_{i in S'_l} delta_il = 1 (Eqs. (15), (16)).
    g, X = _ring_geometry(method)
    rng = np.random.default_rng(0)
    F = rng.standard_normal((len(X), 2))
    G = rng.standard_normal(len(X))
    fib, fE = ib.spread(g, F, G)
    assert np.allclose(fib.sum(0), (F * g.W[:, None]).sum(0), rtol=1e-13, atol=1e-13)
    assert abs(fE.sum() - (G * g.W).sum()) < 1e-12


def test_single_marker_reciprocity():
    # One isolated marker: I[S[G]] = G exactly with the weight of Eq. (17).
    X = np.array([[10.37, 9.81]])
    nrm = np.array([[0.6, 0.8]])
    g = ib.build_geometry((24, 24), X, nrm, ib.FODIBM_R)
    fib, fE = ib.spread(g, np.array([[1.7, -0.4]]), np.array([2.5]))
    field = np.zeros((2, 24 * 24))
    field[:, g.rows] = fib.T
    interp = g.phi[0] * (field[:, g.supp_lin[0]] * g.supp_w[0]).sum(1)
    assert np.allclose(interp, [1.7, -0.4], rtol=0, atol=1e-14)


def test_interpolating_a_constant_and_X_star():
    g, X = _ring_geometry()
    for l in range(len(X)):
        # phi_l sum delta = 1, so a constant is reproduced exactly (Eqs. (14), (16))
        assert abs(g.phi[l] * g.supp_w[l].sum() - 1.0) < 1e-14
        # X* is a convex combination of interior nodes: it lies inside, Eq. (25)
        assert ((g.Xstar[l] - X[l]) * (X[l] - [20.3, 19.6])).sum() < 0.0
    gd, _ = _ring_geometry(ib.DIBM)
    # DIBM: the effective boundary is the marker up to the kernel's first moment
    assert np.abs(gd.Xstar - X).max() < 0.0211 * 1.000001


@pytest.mark.parametrize('where', ['low_x', 'high_y', 'projection'])
def test_stencil_leaving_the_grid_is_refused(where):
    # the node numbering does not wrap, so a support or projection stencil outside the grid must
    # not alias onto other nodes
    X = {'low_x': [[0.7, 10.3]], 'high_y': [[10.2, 18.6]], 'projection': [[10.3, 17.7]]}[where]
    n = [[0.0, 1.0]] if where == 'projection' else [[1.0, 0.0]]
    with pytest.raises(ValueError):
        ib.build_geometry((20, 20), np.array(X), np.array(n), ib.FODIBM_R)
    ib.build_geometry((20, 20), np.array([[10.2, 10.3]]), np.array([[1.0, 0.0]]), ib.FODIBM_R)


def _flat_wall_thermal(method, kind, tv, b, T0=1.1, rho0=1.3, u_wall=0.0):
    """Markers on the node row y0 (normal +y) over T = T0 + b s, s = y - y0, at density rho0."""
    nx, ny, y0 = 40, 16, 8.0
    X = np.array([[float(x), y0] for x in range(4, nx - 4)])
    n = np.tile([0.0, 1.0], (len(X), 1))
    g = ib.build_geometry((nx, ny), X, n, method)
    ys = np.repeat(np.arange(ny), nx).astype(float)
    T = T0 + b * (ys - y0)
    mk = ib.Markers(u_wall=np.tile([u_wall, 0.0], (len(X), 1)), t_kind=np.full(len(X), kind, int),
                    t_value=np.full(len(X), tv))
    rho = np.full(nx * ny, rho0)
    u = np.zeros((2, nx * ny))
    mf = ib.marker_forces(g, mk, _Prm(), rho, rho * u, u, T)
    mid = [l for l in range(len(X)) if 12 <= X[l, 0] <= nx - 13]
    return g, mf, mid


# Flat wall on a node row with the closed interior (rows y0 and y0 - 1): d_BV = 1/3 (worked values
# of the flat-wall table); the projection point P = X + 1.5 n sits half-way between rows, where the
# d = 1 kernel has a zero first moment, and X* lies d_BV below the wall, so for a linear profile
# T^P* = T0 + 1.5 b and the one-sided T* = T0 - b d_BV exactly.
DBV_ROW = 1.0 / 3.0
CV = 5.0 / 6.0


@pytest.mark.parametrize('T_w', [1.1, 1.25])
def test_isothermal_reconstruction_and_heat_source(T_w):
    # Eq. (27) for T: T^Vt = T_w - (d_BV / d_PB)(T^P* - T_w); Eq. (32): Q = Cv rho* (T^Vt - T*).
    # With T_w equal to the profile's wall value the target is the profile's value at V, T0 - b d_BV,
    # and the heat source vanishes; otherwise Q follows the closed form.
    b, T0, rho0 = 0.023, 1.1, 1.3
    g, mf, mid = _flat_wall_thermal(ib.FODIBM_R, ib.T_DIRICHLET, T_w, b, T0, rho0)
    assert np.allclose(g.dBV[mid], DBV_ROW, rtol=0, atol=1e-14)
    assert np.allclose(mf['TP'][mid], T0 + 1.5 * b, rtol=0, atol=1e-14)
    assert np.allclose(mf['T'][mid], T0 - b * DBV_ROW, rtol=0, atol=1e-14)
    Tt = T_w - (DBV_ROW / 1.5) * (T0 + 1.5 * b - T_w)
    assert np.allclose(mf['Tt'][mid], Tt, rtol=0, atol=1e-14)
    assert np.allclose(mf['Qib'][mid], CV * rho0 * (Tt - (T0 - b * DBV_ROW)), rtol=0, atol=1e-14)
    if T_w == T0:
        assert np.allclose(mf['Tt'][mid], T0 - b * DBV_ROW, rtol=0, atol=1e-14)
        assert np.abs(mf['Qib'][mid]).max() < 1e-14
    else:
        assert np.abs(mf['Qib'][mid]).min() > 1e-3


@pytest.mark.parametrize('g_wall', [0.023, -0.011, 0.0])
def test_neumann_reconstruction_with_gradient(g_wall):
    # Eq. (29): T^Vt = T^P* - g (d_PB + d_BV). For the linear profile with slope b the target is
    # T0 + 1.5 b - g (1.5 + d_BV); it equals the profile's value at V when g = b, so
    # Q = Cv rho (b - g)(1.5 + d_BV).
    b, T0, rho0 = 0.023, 1.1, 1.3
    g, mf, mid = _flat_wall_thermal(ib.FODIBM_R, ib.T_NEUMANN, g_wall, b, T0, rho0)
    Tt = T0 + 1.5 * b - g_wall * (1.5 + DBV_ROW)
    assert np.allclose(mf['Tt'][mid], Tt, rtol=0, atol=1e-14)
    assert np.allclose(mf['Qib'][mid], CV * rho0 * (b - g_wall) * (1.5 + DBV_ROW), rtol=0, atol=1e-14)


@pytest.mark.parametrize('kind,tv', [(ib.T_DIRICHLET, 1.25), (ib.T_NEUMANN, 0.011)])
def test_fodibm_thermal_targets(kind, tv):
    # FODIBM imposes the boundary values themselves (Eq. (22)): T^t = T_w, or for a Neumann wall
    # the projection-point value carried back over d_PB with the gradient (reading of Eq. (22) with
    # Eq. (29)'s gradient: T^t = T^P* - g d_PB).
    b, T0, rho0 = 0.023, 1.1, 1.3
    g, mf, mid = _flat_wall_thermal(ib.FODIBM, kind, tv, b, T0, rho0)
    Tt = tv if kind == ib.T_DIRICHLET else T0 + 1.5 * b - tv * 1.5
    assert np.allclose(mf['Tt'][mid], Tt, rtol=0, atol=1e-14)
    assert np.allclose(mf['Qib'][mid], CV * rho0 * (Tt - (T0 - b * DBV_ROW)), rtol=0, atol=1e-14)


def test_no_thermal_condition_gives_no_heat():
    _, mf, mid = _flat_wall_thermal(ib.FODIBM_R, ib.T_NONE, 0.0, 0.023)
    assert np.abs(mf['Qib']).max() == 0.0
