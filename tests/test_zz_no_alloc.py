"""ib_wall_loads_noalloc (scratch in the library's static device array) against ib_wall_loads
(scratch in the handle's workspace), through the C ABI.

Two calls in a row on different bodies, the second with fewer markers, so that the static array
holds the larger first call's contents when the second call runs. The two entry points run the
same kernels in the same order, so the loads agree exactly.
"""
import numpy as np
import pytest

from paper_2607_07432_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ('Q_heat', 'Cd', 'Cl', 'Nu', 'eps_dir', 'eps_neu', 'eps_iso', 'n_inactive', 'n_markers')


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def _compare(solver):
    ref = solver.loads()
    got = solver.loads(noalloc=True)
    np.testing.assert_array_equal(got['F'], ref['F'])
    for k in KEYS:
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.isfinite(ref['F']).all() and ref['n_markers'] > 0
    return ref


def _bodies():
    big = wl.cylinder_case(nx=160, ny=96, center=(50.3, 47.6), diameter=40.0, markers=126, steps=1,
                           reynolds=80.0)
    small = wl.cylinder_case(nx=160, ny=96, center=(50.3, 47.6), diameter=14.0, markers=44, steps=1,
                             T_wall_ratio=None)
    return big, small


@pytest.mark.parametrize('precision', [64, 32])
def test_noalloc_loads_match_workspace_loads_two_calls(lbmib, precision):
    big, small = _bodies()
    print(f'[no_alloc] 2D cylinder 160x96, f{precision}: {len(big.X)} then {len(small.X)} markers', flush=True)
    s = lbmib.Solver.from_case(big, precision=precision)
    s.step(5)
    first = _compare(s)
    assert first['n_markers'] == len(big.X)
    # second call: a smaller body (44 markers, adiabatic) on the same handle
    s.set_markers(small.X, small.n, small.u_wall, small.t_kind, small.t_value, method=small.method)
    s.step(3)
    second = _compare(s)
    assert second['n_markers'] == len(small.X) < first['n_markers']
    assert second['eps_iso'] == 0.0 and first['eps_iso'] > 0.0
    s.close()


def test_noalloc_loads_sphere_then_cylinder(lbmib):
    """A 3D handle (3217 markers) then a 2D handle (44 markers) share the device's static array."""
    sph = wl.sphere_case(nx=96, ny=64, nz=64, diameter=32.0, center=(40.0, 32.0, 32.0), steps=1,
                         reynolds=300.0)
    print(f'[no_alloc] sphere 96x64x64 f32: {len(sph.X)} markers', flush=True)
    s3 = lbmib.Solver.from_case(sph, precision=32)
    s3.step(4)
    a = _compare(s3)
    assert a['n_markers'] == len(sph.X)
    s3.close()
    _, small = _bodies()
    s2 = lbmib.Solver.from_case(small, precision=64)
    s2.step(2)
    b = _compare(s2)
    assert b['n_markers'] == len(small.X)
    s2.close()


def test_noalloc_requires_a_step(lbmib):
    _, small = _bodies()
    s = lbmib.Solver.from_case(small, precision=64)
    with pytest.raises(lbmib.LbmError):
        s.loads(noalloc=True)
    s.close()
