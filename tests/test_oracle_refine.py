"""Pins of the oracle's two-level grid refinement (oracle/refine.py).

The paper refines every mesh locally and states no scheme; these tests fix what the coupling
must do: keep a uniform stream exactly, transfer a state there and back unchanged, carry a shear
wave across the block like the uniform grid does (and closer to the exact decay), and let an
acoustic pulse cross the block with little reflection and little change.
"""
import itertools
import warnings

import numpy as np
import pytest

from oracle import lbm as L
from oracle import refine as RF
from oracle.lattice import for_dim

LAT = for_dim(2)


def _params(mu, u_inf=(0.0, 0.0)):
    cp = 1.4 / 0.4 / 3.0
    return L.Params(mu=mu, lam=mu * cp / 0.71, u_inf=u_inf, T_inf=1.0, bc='periodic')


@pytest.mark.parametrize('D', [2, 3])
def test_uniform_stream_is_a_fixed_point(D):
    lat = for_dim(D)
    if D == 2:
        prm = _params(0.02, (0.08, -0.03))
        st_c = L.freestream_state(lat, prm, (32, 40))
        blk = RF.Block(origin=(10, 8), size=(16, 12))
    else:
        prm = _params(0.02, (0.08, -0.03, 0.05))
        st_c = L.freestream_state(lat, prm, (12, 14, 16))
        blk = RF.Block(origin=(3, 2, 2), size=(8, 9, 8))
    st_f = RF.initial_fine(lat, prm, st_c, blk)
    ref_c, ref_f = st_c.copy(), st_f.copy()
    for _ in range(2):
        st_c, st_f = RF.refined_step(lat, prm, st_c, st_f, blk)
    assert np.abs(st_c.f - ref_c.f).max() < 1e-14 and np.abs(st_c.rhoE - ref_c.rhoE).max() < 1e-14
    assert np.abs(st_f.f - ref_f.f).max() < 1e-14 and np.abs(st_f.rhoE - ref_f.rhoE).max() < 1e-14


def _rich_state(lat, prm, grid, seed):
    """Fields with off-equilibrium populations and a trace-free diagonal force history."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = lat.D
    rho = 1.0 + 0.01 * rng.standard_normal(grid)
    u = 0.02 * rng.standard_normal((D,) + grid)
    T = 1.0 + 0.01 * rng.standard_normal(grid)
    st = L.state_from_fields(lat, prm, rho, u, T)
    st.f = st.f * (1.0 + 1e-3 * rng.standard_normal(st.f.shape))
    for a in range(D):
        st.H2[a, a] = 1e-4 * rng.standard_normal(grid)
    st.H2 -= np.eye(D).reshape((D, D) + (1,) * D) * sum(st.H2[a, a] for a in range(D)) / D
    return st


@pytest.mark.parametrize('D', [2, 3])
def test_transfer_there_and_back_is_the_identity(D):
    # a state with off-equilibrium content and history: prolonged to the fine level and restricted
    # back, the coinciding coarse nodes are unchanged (the two rescalings are inverse)
    lat = for_dim(D)
    prm = _params(0.02)
    if D == 2:
        grid, blk = (30, 36), RF.Block(origin=(6, 5), size=(20, 16))
    else:
        grid, blk = (14, 16, 18), RF.Block(origin=(3, 2, 1), size=(12, 11, 10))
    st_c = _rich_state(lat, prm, grid, 4)
    st_f = RF.initial_fine(lat, prm, st_c, blk)
    back = RF.restrict(lat, prm, RF.fine_params(prm), st_c.copy(), st_f, blk)
    fi, ci = RF.restriction_nodes(blk)
    sc = np.ix_(*reversed(ci))
    sf = np.ix_(*reversed(fi))
    assert all(len(i) > 0 for i in ci)
    assert np.abs(back.f[(slice(None),) + sc] - st_c.f[(slice(None),) + sc]).max() < 1e-15
    assert np.abs(back.rhoE[sc] - st_c.rhoE[sc]).max() == 0.0
    for a in range(D):
        assert np.abs(back.H2[a, a][sc] - st_c.H2[a, a][sc]).max() < 1e-19
    # the fine values there are not the coarse ones (the non-equilibrium part is rescaled)
    assert np.abs(st_f.f[(slice(None),) + sf] - st_c.f[(slice(None),) + sc]).max() > 1e-6
    # and nothing outside the restricted nodes moved
    keep = np.ones(grid, dtype=bool)
    keep[sc] = False
    assert np.array_equal(back.f[:, keep], st_c.f[:, keep])


@pytest.mark.parametrize('D', [2, 3])
def test_interpolation_reproduces_multilinear_fields(D):
    # multilinear interpolation is exact for fields linear in each coordinate (products included),
    # and at coinciding nodes it returns the coarse value
    rng = np.random.Generator(np.random.PCG64(11))
    if D == 2:
        grid, blk = (20, 24), RF.Block(origin=(3, 4), size=(12, 10))
    else:
        grid, blk = (12, 13, 14), RF.Block(origin=(2, 3, 1), size=(8, 6, 7))
    coords_c = np.meshgrid(*[np.arange(n, dtype=float) for n in grid], indexing='ij')   # (z,) y, x
    coef = rng.standard_normal(2 ** D)

    def field(coords):
        xs = list(reversed(coords))           # x, y[, z]
        out = 0.0
        for k, corner in enumerate(itertools.product((0, 1), repeat=D)):
            term = coef[k]
            for a in range(D):
                if corner[a]:
                    term = term * xs[a]
            out = out + term
        return out

    fc = field(coords_c)
    got = RF.interpolate(blk, fc)
    fine_axes = [blk.origin[a] + np.arange(blk.fine_dims[a]) / 2.0 for a in range(D)]
    coords_f = np.meshgrid(*reversed(fine_axes), indexing='ij')
    assert np.abs(got - field(coords_f)).max() < 1e-12
    even = tuple(slice(0, None, 2) for _ in range(D))
    sl = tuple(slice(blk.origin[a], blk.origin[a] + blk.size[a]) for a in reversed(range(D)))
    assert np.array_equal(got[even], fc[sl])


def test_band_and_restriction_sets():
    blk = RF.Block(origin=(5, 7), size=(10, 9), G=4, R=8)
    m = RF.band_mask(blk)
    assert m.shape == (18, 20)
    assert m.sum() == 18 * 20 - (18 - 8) * (20 - 8)
    assert not m[4:14, 4:16].any() and m[:4].all() and m[:, -4:].all()
    fi, ci = RF.restriction_nodes(blk)
    assert list(fi[0]) == [8, 10] and list(fi[1]) == [8]
    assert list(ci[0]) == [9, 10] and list(ci[1]) == [11]


def _shear_wave(N=200, mu=0.02, U=0.02):
    prm = _params(mu)
    ny, nx = 48, 64
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    u = np.stack([np.zeros((ny, nx)), U * np.sin(2 * np.pi * x / nx)])
    st_c = L.state_from_fields(LAT, prm, np.ones((ny, nx)), u, np.ones((ny, nx)))
    st_u = st_c.copy()
    blk = RF.Block(origin=(16, 12), size=(32, 24))
    st_f = RF.initial_fine(LAT, prm, st_c, blk)
    for _ in range(N):
        st_c, st_f = RF.refined_step(LAT, prm, st_c, st_f, blk)
        st_u = L.lbm_step(LAT, prm, st_u)
    uc = L.fields(LAT, prm, st_c)[1]
    uu = L.fields(LAT, prm, st_u)[1]
    k = 2 * np.pi / nx
    exact = U * np.exp(-mu * k * k * N)
    return np.abs(uc[1]).max(), np.abs(uu[1]).max(), exact, np.abs(uc - uu).max() / U


@pytest.mark.slow
def test_shear_wave_crosses_the_block():
    # measured: amplitude 1.92332e-2 refined, 1.92279e-2 uniform, 1.92436e-2 exact; largest
    # velocity difference to the uniform grid 1.5e-3 U (several times more without the factor 2 of
    # the non-equilibrium rescaling or with the coarse viscosity on the fine level)
    amp_r, amp_u, exact, diff = _shear_wave()
    print(f'shear wave: refined {amp_r:.6e} uniform {amp_u:.6e} exact {exact:.6e}, difference {diff:.3e} U')
    assert diff < 4e-3
    assert abs(amp_r - exact) < abs(amp_u - exact)


def _pulse(N=220, mu=0.005):
    prm = _params(mu)
    ny, nx = 24, 160
    c = np.sqrt(1.4 / 3.0)
    x = np.arange(nx, dtype=float)
    dp = 1e-3 * np.exp(-0.5 * ((x - 25.0) / 4.0) ** 2)
    rho1 = 1.0 + dp / c ** 2
    T1 = (1.0 / 3.0 + dp) / (rho1 / 3.0)
    rho, T = np.tile(rho1, (ny, 1)), np.tile(T1, (ny, 1))
    u = np.stack([np.tile(dp / c, (ny, 1)), np.zeros((ny, nx))])
    st_c = L.state_from_fields(LAT, prm, rho, u, T)
    st_u = st_c.copy()
    blk = RF.Block(origin=(50, 4), size=(60, 16))
    st_f = RF.initial_fine(LAT, prm, st_c, blk)
    up_r, up_u, dn_r, dn_u = [], [], [], []
    for _ in range(N):
        st_c, st_f = RF.refined_step(LAT, prm, st_c, st_f, blk)
        st_u = L.lbm_step(LAT, prm, st_u)
        pr = L.fields(LAT, prm, st_c)[3]
        pu = L.fields(LAT, prm, st_u)[3]
        up_r.append(pr[12, 40]); up_u.append(pu[12, 40])
        dn_r.append(pr[12, 135]); dn_u.append(pu[12, 135])
    up_r, up_u, dn_r, dn_u = map(np.array, (up_r, up_u, dn_r, dn_u))
    refl = np.abs(up_r - up_u).max() / np.abs(up_u - prm.R).max()
    trans = np.abs(dn_r - dn_u).max() / np.abs(dn_u - prm.R).max()
    return refl, trans


@pytest.mark.slow
def test_acoustic_pulse_crosses_the_block():
    # a plane pulse through a block 60 x 16 coarse cells: at a probe upstream, the refined grid
    # differs from the uniform one by the waves its interfaces reflect (measured 6.2e-4 of the
    # pulse), downstream by what the crossing changes (7.8e-3). Mistimed band values or no
    # interpolation in x raise both several times (with a band of four nodes: 3.5e-3 and 3.0e-2
    # for the coarse state of the end of the step at both fine steps)
    with warnings.catch_warnings():
        warnings.simplefilter('ignore')
        refl, trans = _pulse()
    print(f'pulse: reflected {refl:.3e}, transmitted difference {trans:.3e}')
    assert refl < 1.5e-3 and trans < 1.5e-2


def test_nest_of_three_levels_keeps_a_uniform_stream():
    prm = _params(0.01, (0.06, 0.02))
    st0 = L.freestream_state(LAT, prm, (40, 48))
    blocks = [RF.Block(origin=(8, 8), size=(28, 20)), RF.Block(origin=(14, 10), size=(24, 16))]
    states = RF.initial_nest(LAT, prm, st0, blocks)
    ref = [s.copy() for s in states]
    assert [s.f.shape[1:] for s in states] == [(40, 48), (40, 56), (32, 48)]
    states = RF.nested_step(LAT, prm, states, blocks)
    for s, r in zip(states, ref):
        assert np.abs(s.f - r.f).max() < 1e-14 and np.abs(s.rhoE - r.rhoE).max() < 1e-14


def _nest_pulse(N=220, mu=0.0025):
    """The pulse of the two-level pin through a block (60 x 16 coarse cells at (50, 4)) with and
    without a second one inside it (60 x 16 cells of level 1 at (30, 8)). Returns the reflection
    and transmission of the nest seen on level 0, and those of the inner block seen on level 1
    (upstream and downstream of it), each relative to the pulse."""
    prm = _params(mu)
    prm1 = RF.fine_params(prm)
    ny, nx = 24, 160
    c = np.sqrt(1.4 / 3.0)
    x = np.arange(nx, dtype=float)
    dp = 1e-3 * np.exp(-0.5 * ((x - 25.0) / 4.0) ** 2)
    rho1 = 1.0 + dp / c ** 2
    T1 = (1.0 / 3.0 + dp) / (rho1 / 3.0)
    rho, T = np.tile(rho1, (ny, 1)), np.tile(T1, (ny, 1))
    u = np.stack([np.tile(dp / c, (ny, 1)), np.zeros((ny, nx))])
    st0 = L.state_from_fields(LAT, prm, rho, u, T)
    su = st0.copy()
    blocks = [RF.Block(origin=(50, 4), size=(60, 16)), RF.Block(origin=(30, 8), size=(60, 16))]
    nest = RF.initial_nest(LAT, prm, st0, blocks)
    two = RF.initial_nest(LAT, prm, st0, blocks[:1])
    h = {k: [] for k in ('up', 'up_u', 'dn', 'dn_u', 'up1', 'up1_2', 'dn1', 'dn1_2')}
    for _ in range(N):
        nest = RF.nested_step(LAT, prm, nest, blocks)
        two = RF.nested_step(LAT, prm, two, blocks[:1])
        su = L.lbm_step(LAT, prm, su)
        p0, pu = L.fields(LAT, prm, nest[0])[3], L.fields(LAT, prm, su)[3]
        p1, p12 = L.fields(LAT, prm1, nest[1])[3], L.fields(LAT, prm1, two[1])[3]
        h['up'].append(p0[12, 40]); h['up_u'].append(pu[12, 40])
        h['dn'].append(p0[12, 135]); h['dn_u'].append(pu[12, 135])
        h['up1'].append(p1[16, 15]); h['up1_2'].append(p12[16, 15])
        h['dn1'].append(p1[16, 105]); h['dn1_2'].append(p12[16, 105])
    h = {k: np.array(v) for k, v in h.items()}
    amp = lambda a: np.abs(a - prm.R).max()
    return (np.abs(h['up'] - h['up_u']).max() / amp(h['up_u']), np.abs(h['dn'] - h['dn_u']).max() / amp(h['dn_u']),
            np.abs(h['up1'] - h['up1_2']).max() / amp(h['up1_2']), np.abs(h['dn1'] - h['dn1_2']).max() / amp(h['dn1_2']))


@pytest.mark.slow
def test_acoustic_pulse_crosses_a_nest_of_three_levels():
    # seen on level 0 the nest reflects 7.2e-4 of the pulse and changes it by 9.1e-3; seen on
    # level 1 the inner block reflects 2.1e-4 and changes the pulse by 1.1e-3
    with warnings.catch_warnings():
        warnings.simplefilter('ignore')
        refl, trans, refl1, trans1 = _nest_pulse()
    print(f'nest pulse: level 0 {refl:.3e} / {trans:.3e}, inner block on level 1 {refl1:.3e} / {trans1:.3e}')
    assert refl < 1.5e-3 and trans < 1.5e-2
    assert refl1 < 5e-4 and trans1 < 2e-3


def _nest_shear(blocks, N=200, mu=0.02, U=0.02):
    prm = _params(mu)
    ny, nx = 48, 64
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    u = np.stack([np.zeros((ny, nx)), U * np.sin(2 * np.pi * x / nx)])
    st = L.state_from_fields(LAT, prm, np.ones((ny, nx)), u, np.ones((ny, nx)))
    states = RF.initial_nest(LAT, prm, st, blocks)
    for _ in range(N):
        states = RF.nested_step(LAT, prm, states, blocks)
    uc = L.fields(LAT, prm, states[0])[1]
    k = 2 * np.pi / nx
    return np.abs(uc[1]).max() - U * np.exp(-mu * k * k * N), uc


@pytest.mark.slow
def test_shear_wave_error_falls_with_each_level():
    # the shear wave of the two-level pin with a third level inside the block (24 x 18 cells of
    # level 1): the amplitude error after 200 coarse steps falls from -1.57e-5 (uniform) to
    # -1.044e-5 (two levels) and -9.93e-6 (three), and the third level changes the coarse velocity
    # by 6.3e-4 U
    outer = RF.Block(origin=(16, 12), size=(32, 24))
    inner = RF.Block(origin=(8, 6), size=(24, 18))
    e2, u2 = _nest_shear([outer])
    e3, u3 = _nest_shear([outer, inner])
    d = np.abs(u3 - u2).max() / 0.02
    print(f'shear wave errors: two levels {e2:.3e}, three {e3:.3e}; change {d:.2e} U')
    assert e2 < e3 < 0.0
    assert 1e-4 < d < 2e-3
