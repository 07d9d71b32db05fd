"""Edge cases of the GPU path against the oracle (FP64, both sweeps):

  * no body: the pure lattice Boltzmann step on periodic boxes, including the smallest grids the
    ABI accepts (nx = 5, two rows in 2D, two planes in 3D, where the two-node stencils wrap onto
    themselves) and marching axes shorter than the macros ring; smaller grids are refused;
  * a body whose markers all have an empty interior support (inactive: no forcing, counted);
  * grids larger than one tile in every in-plane direction with ragged last tiles (the one-
    conditional-wrap path of the fused sweep), in 2D and 3D, FP64 and FP32;
  * zero steps leave the state untouched;
  * a body 3 cells from a periodic edge of a multi-tile grid (tile footprints wrap onto it).
"""
import numpy as np
import pytest

from oracle.lattice import for_dim
from paper_2607_07432_amd import workloads as wl

from parity_util import oracle_geometry, oracle_markers, oracle_step, random_state, rel

pytestmark = pytest.mark.gpu

SWEEPS = {'fused': 0, 'threepass': 1}


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def periodic_box(dims):
    if len(dims) == 2:
        c = wl.cylinder_case(nx=dims[0], ny=dims[1], center=(dims[0] / 2, dims[1] / 2), diameter=2.0, markers=8,
                             steps=1, T_wall_ratio=None)
    else:
        c = wl.sphere_case(nx=dims[0], ny=dims[1], nz=dims[2], diameter=2.0, markers=8, steps=1,
                           center=tuple(d / 2 for d in dims))
    c.bc = 'periodic'
    return c


def march(lbmib, case, st, steps, sweep, with_body, precision=64):
    s = lbmib.Solver.from_case(case, precision=precision, sweep=sweep, markers=with_body)
    s.set_state(st.f, st.rhoE, st.H2)
    g = oracle_geometry(case) if with_body else None
    mk = oracle_markers(case) if with_body else None
    ref = st
    for _ in range(steps):
        ref, _ = oracle_step(case, ref, g, mk)
    s.step(steps)
    f, e, H = s.get_state()
    return s, ref, f, e, H


@pytest.mark.parametrize('sweep', list(SWEEPS))
@pytest.mark.parametrize('dims', [(40, 30), (5, 2), (7, 3), (9, 4), (12, 10, 8), (5, 4, 3), (6, 5, 2), (5, 2, 2)],
                         ids=lambda d: 'x'.join(map(str, d)))
def test_no_body_periodic(lbmib, dims, sweep):
    case = periodic_box(dims)
    st = random_state(case, None, seed=3)
    s, ref, f, e, H = march(lbmib, case, st, 3, SWEEPS[sweep], with_body=False)
    print(dims, sweep, 'rel f', rel(f, ref.f), 'rel rhoE', rel(e, ref.rhoE), flush=True)
    assert rel(f, ref.f) < 1e-12 and rel(e, ref.rhoE) < 1e-12
    assert np.abs(H - ref.H2).max() < 1e-15
    s.close()


@pytest.mark.parametrize('dims', [(6, 1), (4, 8), (6, 5, 1), (6, 1, 5)], ids=lambda d: 'x'.join(map(str, d)))
def test_too_small_grids_are_refused(lbmib, dims):
    case = periodic_box(dims)
    with pytest.raises(lbmib.LbmError) as ei:
        lbmib.Solver.from_case(case, markers=False)
    assert ei.value.code == lbmib.LBM_E_INVAL


def test_all_markers_inactive(lbmib):
    # a cylinder of radius 0.3 centred between nodes holds no node: every support is empty
    case = wl.cylinder_case(nx=40, ny=30, center=(20.5, 15.5), diameter=0.6, markers=8, steps=1)
    g = oracle_geometry(case)
    assert not g.active.any()
    st = random_state(case, g, seed=5)
    for sweep in SWEEPS.values():
        s, ref, f, e, H = march(lbmib, case, st, 2, sweep, with_body=True)
        L = s.loads()
        assert L['n_inactive'] == len(case.X) and L['n_markers'] == len(case.X)
        assert np.all(L['F'] == 0.0) and L['Cd'] == 0.0
        assert rel(f, ref.f) < 1e-12 and rel(e, ref.rhoE) < 1e-12
        # and the step equals the step without a body
        s2, _, f2, e2, _ = march(lbmib, case, st, 2, sweep, with_body=False)
        assert np.array_equal(f, f2) and np.array_equal(e, e2)
        s.close()
        s2.close()


@pytest.mark.parametrize('precision', [64, 32])
@pytest.mark.parametrize('dim', [2, 3])
def test_ragged_multi_tile_grids(lbmib, dim, precision):
    # 2D: 300 = 254 + 46 columns; 3D: 40 = 30 + 10, 20 = 14 + 6 (FP32 tile) or 3 x 6 + 2 (FP64)
    if dim == 2:
        case = wl.cylinder_case(nx=300, ny=40, center=(90.3, 20.2), diameter=10.0, markers=32, steps=1)
    else:
        case = wl.sphere_case(nx=40, ny=20, nz=16, diameter=6.0, markers=113, steps=1, center=(15.2, 10.1, 7.9),
                              T_wall_ratio=1.2)
    g = oracle_geometry(case)
    st = random_state(case, g, seed=9)
    s, ref, f, e, H = march(lbmib, case, st, 2, 0, with_body=True, precision=precision)
    tol = 1e-12 if precision == 64 else 1e-5
    print(dim, precision, 'rel f', rel(f, ref.f), 'rel rhoE', rel(e, ref.rhoE), flush=True)
    if precision == 64:
        assert rel(f, ref.f) < tol and rel(e, ref.rhoE) < tol
    else:
        lat = for_dim(dim)
        w = lat.w.reshape((-1,) + (1,) * dim)
        assert np.abs(f - ref.f).max() <= tol * np.abs(ref.f - w).max()
        assert rel(e, ref.rhoE) < tol
    s.close()


def test_zero_steps_leave_state(lbmib):
    case = wl.cylinder_case(nx=40, ny=30, center=(15.3, 14.8), diameter=8.0, markers=24, steps=1)
    g = oracle_geometry(case)
    st = random_state(case, g, seed=2)
    s = lbmib.Solver.from_case(case, precision=64)
    s.set_state(st.f, st.rhoE, st.H2)
    a = s.get_state()
    s.step(0)
    b = s.get_state()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    s.close()


@pytest.mark.parametrize('dim', [2, 3])
def test_body_near_a_periodic_edge(lbmib, dim):
    # markers 3 cells from the low x edge of a periodic multi-tile grid: the last tile's footprint
    # wraps onto the first columns, and the tiles select the forcing instantiation by the forced
    # nodes' bounding box, so this checks that no tile misses forcing it needs
    if dim == 2:
        case = wl.cylinder_case(nx=300, ny=40, center=(8.3, 20.2), diameter=10.0, markers=32, steps=1)
    else:
        case = wl.sphere_case(nx=40, ny=20, nz=16, diameter=6.0, markers=113, steps=1, center=(6.3, 10.1, 7.9),
                              T_wall_ratio=1.2)
    case.bc = 'periodic'
    assert case.X[:, 0].min() > 3.0 and case.X[:, 0].min() < 3.6
    g = oracle_geometry(case)
    st = random_state(case, g, seed=13)
    for sweep in SWEEPS.values():
        s, ref, f, e, H = march(lbmib, case, st, 2, sweep, with_body=True)
        print(dim, sweep, 'rel f', rel(f, ref.f), 'rel rhoE', rel(e, ref.rhoE), flush=True)
        assert rel(f, ref.f) < 1e-12 and rel(e, ref.rhoE) < 1e-12
        s.close()
