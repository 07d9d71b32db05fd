"""Batched persistent step of uneven 2D cases (lbm_batch_*), through the C ABI.

The batch runs the same per-node update as the single-grid step, so it is checked
(a) against the FP64 oracle directly, case by case, on small uneven ellipse cases;
(b) against the single-grid path over many steps (odd and even step counts, both precisions,
    every tile width), state, loads and residual;
(c) for the bookkeeping: autotuning leaves the state unchanged, a case stepped or given a new
    body between batch calls is picked up, invalid batches are refused.
"""
import numpy as np
import pytest

from paper_2607_07432_amd import workloads as wl

from parity_util import oracle_geometry, oracle_markers, oracle_step, random_state, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def small_cases(count=5, seed0=1000, isothermal=False):
    # nx = 4M from 64 to 192: every tile width leaves a ragged last tile somewhere
    return wl.batched_cases(count, seed0=seed0, m_lo=16, m_hi=48, isothermal=isothermal)


def solvers_for(lbmib, cases, precision):
    return [lbmib.Solver.from_case(c, precision=precision) for c in cases]


def state_rel(a, b):
    return max(rel(x, y) for x, y in zip(a, b))


def test_batch_matches_oracle_fp64(lbmib):
    """Three uneven FP64 cases (isothermal walls) from injected random states: every step within
    1e-12 of the oracle."""
    cases = small_cases(3, seed0=2000, isothermal=True)
    sols = solvers_for(lbmib, cases, lbmib.F64)
    sts, geoms, mks = [], [], []
    for k, (c, s) in enumerate(zip(cases, sols)):
        g = oracle_geometry(c)
        st = random_state(c, g, seed=40 + k)
        s.set_state(st.f, st.rhoE, st.H2)
        sts.append(st)
        geoms.append(g)
        mks.append(oracle_markers(c))
    batch = lbmib.Batch(sols, autotune=False)
    for step in range(3):
        batch.step(1)
        for k, c in enumerate(cases):
            sts[k], _ = oracle_step(c, sts[k], geoms[k], mks[k])
            f, e, H2 = sols[k].get_state()
            err = state_rel((f, e), (sts[k].f, sts[k].rhoE))
            print(f'step {step + 1} case {k} {c.dims}: rel {err:.2e}', flush=True)
            assert err <= 1e-12
    batch.close()


@pytest.mark.parametrize('precision', ['F32', 'F64'])
def test_batch_matches_single_grid(lbmib, precision):
    prec = getattr(lbmib, precision)
    cases = small_cases(5)
    ref = solvers_for(lbmib, cases, prec)
    bat = solvers_for(lbmib, cases, prec)
    batch = lbmib.Batch(bat, autotune=True)
    cfg = batch.config()
    print('tuned', cfg, flush=True)
    assert cfg['markers'] == sum(len(c.X) for c in cases)
    for s in ref:
        s.step(9)
    batch.step(9)                 # odd count: ends on the other parity
    for s in ref:
        s.step(4)
    batch.step(4)
    # not bit-exact: tile widths are separate instantiations, whose FMA contraction may differ;
    # the bars are those of the single-grid path against the oracle
    tol = 1e-12 if prec == lbmib.F64 else 1e-5
    gathered = batch.residuals()
    for k, (a, b) in enumerate(zip(ref, bat)):
        sa, sb = a.get_state(), b.get_state()
        err = state_rel(sb, sa)
        la, lb = a.loads(), b.loads()
        ra, rb = a.residual(), b.residual()
        print(f'case {k} {cases[k].dims}: state rel {err:.2e}, Cd {la["Cd"]:.6f}/{lb["Cd"]:.6f}, '
              f'residual {ra:.6e}/{rb:.6e}', flush=True)
        assert err <= tol
        assert abs(la['Cd'] - lb['Cd']) <= (1e-10 if prec == lbmib.F64 else 1e-4) * max(1.0, abs(la['Cd']))
        assert abs(ra - rb) <= (1e-10 if prec == lbmib.F64 else 1e-4) * ra
        assert gathered[k] == rb
    batch.close()


def test_batch_mixes_methods_walls_and_bodies(lbmib):
    """One batch holding the three methods, fixed and turning walls, isothermal and adiabatic
    walls, an ellipse, a cylinder and a star: each case equals its single-grid run (FP64)."""
    cases = [
        wl.cylinder_case(nx=96, ny=48, center=(30.2, 24.3), diameter=12.0, markers=38, method=wl.METHOD_DIBM,
                         mach=0.1, steps=1),
        wl.cylinder_case(nx=80, ny=40, center=(24.6, 19.8), diameter=10.0, markers=32, method=wl.METHOD_FODIBM,
                         mach=0.1, T_wall_ratio=None, omega_star=0.5, steps=1),
        wl.star_case(48, 0.1, 0.3, 0.1, 30.0, nx=128, ny=64, steps=1),
        wl.ellipse_case(40, 2.0, 0.4, 0.12, 40.0, None, nx=160, ny=80),
    ]
    cases[3].u_wall = wl.rotation_wall_velocity(cases[3].X, cases[3].extra['center'], -0.004)
    ref = solvers_for(lbmib, cases, lbmib.F64)
    bat = solvers_for(lbmib, cases, lbmib.F64)
    batch = lbmib.Batch(bat, autotune=False)
    for s in ref:
        s.step(7)
    batch.step(7)
    for k, (a, b) in enumerate(zip(ref, bat)):
        err = state_rel(b.get_state(), a.get_state())
        la, lb = a.loads(), b.loads()
        print(f'case {k} ({cases[k].name}, method {cases[k].method}): state rel {err:.2e}, '
              f'eps_dir {la["eps_dir"]:.4e}/{lb["eps_dir"]:.4e}', flush=True)
        assert err <= 1e-12
        for key in ('Cd', 'Cl', 'eps_dir', 'eps_neu', 'eps_iso'):
            assert abs(la[key] - lb[key]) <= 1e-10 * max(1.0, abs(la[key]))
    batch.close()


@pytest.mark.parametrize('tile', [62, 126, 254])
def test_batch_tile_widths_agree(lbmib, tile):
    """Every tile width gives the single-grid result (FP64, 6 steps)."""
    cases = small_cases(4, seed0=3000)
    ref = solvers_for(lbmib, cases, lbmib.F64)
    bat = solvers_for(lbmib, cases, lbmib.F64)
    for s in ref:
        s.step(6)
    batch = lbmib.Batch(bat, autotune=False)
    batch.set_tile(tile, 16)
    assert batch.config()['tile_x'] == tile and batch.config()['chunk'] == 16
    batch.step(6)
    for a, b in zip(ref, bat):
        assert state_rel(b.get_state(), a.get_state()) <= 1e-12
    batch.close()


def test_batch_autotune_keeps_state(lbmib):
    cases = small_cases(3, seed0=4000)
    sols = solvers_for(lbmib, cases, lbmib.F32)
    for s in sols:
        s.step(3)
    before = [s.get_state() for s in sols]
    batch = lbmib.Batch(sols, autotune=True)
    after = [s.get_state() for s in sols]
    for x, y in zip(before, after):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    batch.close()


def test_batch_resyncs_after_single_steps_and_new_body(lbmib):
    cases = small_cases(3, seed0=5000)
    ref = solvers_for(lbmib, cases, lbmib.F64)
    bat = solvers_for(lbmib, cases, lbmib.F64)
    batch = lbmib.Batch(bat, autotune=False)
    batch.step(2)
    bat[1].step(1)                # one case advanced on its own
    batch.step(3)
    for k, s in enumerate(ref):
        s.step(6 if k == 1 else 5)
    for a, b in zip(ref, bat):
        assert state_rel(b.get_state(), a.get_state()) <= 1e-12
    # a new body on one case: the batch rebuilds its marker and row numbering
    c = cases[2]
    X = c.X + np.array([0.37, -0.21])
    for s in (ref[2], bat[2]):
        s.set_markers(X, c.n, c.u_wall, c.t_kind, c.t_value, c.method)
    batch.step(2)
    for s in ref:
        s.step(2)
    for a, b in zip(ref, bat):
        assert state_rel(b.get_state(), a.get_state()) <= 1e-12
    batch.close()


def test_batch_refuses_invalid(lbmib):
    from parity_util import small_sphere_case
    c2 = small_cases(1)[0]
    s2 = lbmib.Solver.from_case(c2, precision=lbmib.F32)
    s2b = lbmib.Solver.from_case(c2, precision=lbmib.F64)
    s3 = lbmib.Solver.from_case(small_sphere_case(), precision=lbmib.F32)
    for group in ([s2, s3], [s2, s2b], [s2, s2]):
        with pytest.raises(lbmib.LbmError):
            lbmib.Batch(group)
    b = lbmib.Batch([s2], autotune=False)
    with pytest.raises(lbmib.LbmError):
        b.set_tile(100, 16)
    with pytest.raises(lbmib.LbmError):
        b.set_tile(62, 0)
    b.close()


def test_untuned_small_batch_takes_short_chunks(lbmib):
    """Without autotuning a batch too small to give eight 32-row items per workgroup of the
    persistent launch takes 16-row chunks; its steps equal the single-grid steps (FP64)."""
    cases = small_cases(3, seed0=3100)
    ref = solvers_for(lbmib, cases, lbmib.F64)
    bat = solvers_for(lbmib, cases, lbmib.F64)
    for s in ref:
        s.step(5)
    batch = lbmib.Batch(bat, autotune=False)
    cfg = batch.config()
    print('untuned', cfg, flush=True)
    assert cfg['tile_x'] == 62 and cfg['chunk'] == 16
    batch.step(5)
    for a, b in zip(ref, bat):
        assert state_rel(b.get_state(), a.get_state()) <= 1e-12
    batch.close()
