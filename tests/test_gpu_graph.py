"""lbm_step replays pairs of steps as a captured HIP graph for calls of five steps or more.

The graph path must give the states of stepping one call at a time, bit for bit, on every
replay: each case below alternates graph calls with host reads of the state (eager work and
synchronisation between the replays), over both state parities, and again after a new body
forces a new capture.
"""
import numpy as np
import pytest

from paper_2607_07432_amd import workloads as wl

from parity_util import random_state, small_sphere_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def _case(name):
    if name == 'cylinder':
        return wl.cylinder_case(nx=96, ny=48, center=(30.3, 24.2), diameter=10.0, markers=32, steps=1)
    if name == 'cylinder_char':
        c = wl.cylinder_case(nx=96, ny=48, center=(30.3, 24.2), diameter=10.0, markers=32, steps=1)
        c.bc = 'characteristic'
        return c
    return small_sphere_case()


def _same(a, b):
    fa, ea, ha = a.get_state()
    fb, eb, hb = b.get_state()
    return np.array_equal(fa, fb) and np.array_equal(ea, eb) and np.array_equal(ha, hb)


@pytest.mark.parametrize('name,precision,sweep', [('cylinder', 64, 0), ('cylinder', 32, 0), ('cylinder_char', 32, 0),
                                                  ('cylinder', 32, 1), ('sphere', 32, 0)])
def test_graph_replay_equals_single_steps(lbmib, name, precision, sweep):
    case = _case(name)
    print(f'[graph] {name} {case.dims} f{precision} sweep {sweep}', flush=True)
    a = lbmib.Solver.from_case(case, precision=precision, sweep=sweep)
    b = lbmib.Solver.from_case(case, precision=precision, sweep=sweep)
    st = random_state(case, None, seed=3)
    for s in (a, b):
        s.set_state(st.f, st.rhoE, st.H2)
    for n in (9, 6, 5, 8):          # both parities of the pairs, odd and even calls
        a.step(n)
        for _ in range(n):
            b.step(1)
        assert _same(a, b), n
        assert a.residual() == b.residual()
    # a new body is captured anew
    X = case.X + np.array([0.37, -0.21] + ([0.13] if case.dim == 3 else []))
    for s in (a, b):
        s.set_markers(X, case.n, case.u_wall, case.t_kind, case.t_value, case.method)
    a.step(7)
    for _ in range(7):
        b.step(1)
    assert _same(a, b)
    assert a.residual() == b.residual()
    la, lb = a.loads(), b.loads()
    assert la['Cd'] == lb['Cd'] and la['Nu'] == lb['Nu']


def _wide_case(name):
    # grids larger than one sweep tile (254 nodes wide in 2D, 30 x 14 in 3D), so that a grid holds
    # several work items
    if name == 'cylinder_wide':
        return wl.cylinder_case(nx=400, ny=96, center=(100.3, 48.2), diameter=16.0, markers=50, steps=1)
    return wl.sphere_case(nx=96, ny=48, nz=40, diameter=12.0, center=(30.3, 24.2, 19.9), mach=0.3,
                          reynolds=100.0, steps=1)


@pytest.mark.parametrize('name,precision', [('sphere_mid', 32), ('sphere_mid', 64), ('cylinder_wide', 32)])
def test_states_agree_across_chunks(lbmib, name, precision, monkeypatch):
    """The fused sweep's work items march over chunks of planes whose first planes recompute what
    the previous chunk's last ones computed. The chunk only decides which tile code covers a plane
    (with the forcing path near the body, without it elsewhere), and the two round a few products
    differently: after 9 steps from a perturbed state the chunk lbm_init_grid picks and explicit
    ones (LBMIB_FUSED_CHUNK) agree to 1e-14 of max|f| in FP64 and within the 1e-5 field bar in
    FP32 (measured 1.4e-15 and 8e-7 on the sphere)."""
    case = _wide_case(name)
    st = random_state(case, None, seed=11)
    states = {}
    for chunk in (None, 8, 13, 64):
        if chunk is None:
            monkeypatch.delenv('LBMIB_FUSED_CHUNK', raising=False)
        else:
            monkeypatch.setenv('LBMIB_FUSED_CHUNK', str(chunk))
        print(f'[chunk] {name} f{precision} chunk {chunk or "auto"}', flush=True)
        s = lbmib.Solver.from_case(case, precision=precision)
        s.set_state(st.f, st.rhoE, st.H2)
        s.step(3)
        s.step(6)
        states[chunk] = s.get_state()
        s.close()
    ref = states[None]
    bar = 1e-14 if precision == 64 else 1e-5
    for chunk, got in states.items():
        for a, b in zip(got, ref):
            d = np.abs(a - b).max() / np.abs(b).max()
            print(f'[chunk] {chunk}: {d:.2e}', flush=True)
            assert d <= bar, chunk
