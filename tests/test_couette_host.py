"""Host side of the circular Couette check: the analytic profile and the effective-wall fit."""
import copy

import numpy as np

from paper_2607_07432_amd import methods, workloads as wl


def field(case, prof_case):
    nx, ny = case.dims
    cx, cy = case.extra['center']
    ys, xs = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = xs - cx, ys - cy
    r = np.maximum(np.hypot(dx, dy), 1e-12)
    ut = wl.couette_profile(prof_case, r)
    return np.ones((ny, nx)), np.stack([-ut * dy / r, ut * dx / r])


def test_profile_solves_the_steady_problem():
    c = wl.taylor_couette_case(2)
    r1, r2, U = c.extra['r1'], c.extra['r2'], c.extra['speed']
    assert abs(wl.couette_profile(c, r1) - U) < 1e-15 and abs(wl.couette_profile(c, r2)) < 1e-15
    # u'' + u'/r - u/r^2 = 0 (azimuthal momentum, no pressure gradient), by differences
    r = np.linspace(r1, r2, 50)
    h = 1e-3
    u = lambda x: wl.couette_profile(c, x)
    lhs = (u(r + h) - 2 * u(r) + u(r - h)) / h ** 2 + (u(r + h) - u(r - h)) / (2 * h * r) - u(r) / r ** 2
    assert np.abs(lhs).max() < 1e-8 * U


def test_exact_field_has_no_error_and_walls_in_place():
    c = wl.taylor_couette_case(1)
    e = methods.couette_errors(c, *field(c, c))
    assert e['l2_gap'] < 1e-14 and e['max_core'] < 1e-14
    assert abs(e['dr_in']) < 1e-10 and abs(e['dr_out']) < 1e-10


def test_fit_recovers_shifted_walls():
    c = wl.taylor_couette_case(1)
    s = copy.deepcopy(c)
    s.extra['r1'] += 0.3
    s.extra['r2'] -= 0.2
    s.extra['speed'] *= s.extra['r1'] / c.extra['r1']      # the same rigid rotation, met further out
    e = methods.couette_errors(c, *field(c, s))
    assert abs(e['dr_in'] - 0.3) < 1e-10 and abs(e['dr_out'] + 0.2) < 1e-10
    assert e['l2_gap'] > 0.01


def test_case_geometry():
    for sc in (1, 3):
        c = wl.taylor_couette_case(sc)
        k = c.extra['n_inner']
        ctr = np.array(c.extra['center'])
        rad = np.hypot(*(c.X - ctr).T)
        assert np.allclose(rad[:k], c.extra['r1']) and np.allclose(rad[k:], c.extra['r2'])
        # normals point into the fluid: outward on the inner wall, inward on the outer
        radial = (c.X - ctr) / rad[:, None]
        assert np.allclose((c.n[:k] * radial[:k]).sum(1), 1.0) and np.allclose((c.n[k:] * radial[k:]).sum(1), -1.0)
        # the inner wall turns rigidly at speed / r1, the outer is fixed
        om = c.extra['speed'] / c.extra['r1']
        assert np.allclose(c.u_wall[:k], om * np.stack([-(c.X[:k, 1] - ctr[1]), c.X[:k, 0] - ctr[0]], 1))
        assert np.all(c.u_wall[k:] == 0.0)
        assert min(c.X.min(), (np.array(c.dims) - 1 - c.X).min()) > 3.0
