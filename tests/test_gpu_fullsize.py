"""Parity at the benchmark sizes, in the launch configurations the benchmark times, on sampled
nodes the oracle can compute one by one.

One step of the GPU path is compared, at sample nodes, with the oracle run on a small periodic
window of the GPU's own previous state centred on the node. The new state of a node depends on
the old state within three nodes (macros of the collision neighbours' neighbours), so a window of
radius 5 gives the centre exactly; sample windows contain no forced node and no node of the
inflow/outflow columns. The GPU state goes through its canonical FP64 export, so FP32 storage is
compared at its own rounding (relative 1e-5 of the largest population deviation), FP64 at 1e-12.
"""
import numpy as np
import pytest

from oracle import lbm as olbm
from oracle.lattice import for_dim
from paper_2607_07432_amd import workloads as wl

from parity_util import oracle_params

pytestmark = pytest.mark.gpu

R = 5          # window radius


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def window_params(case):
    prm = oracle_params(case)
    prm.bc = 'periodic'
    return prm


def pick_samples(grid, forced, count, seed, xmargin):
    """Centres whose window holds no forced node and no inflow/outflow column."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = len(grid)
    near = np.zeros(grid, dtype=bool)
    if len(forced):
        idx = np.array(np.unravel_index(forced, grid))
        for off in np.ndindex(*([2 * R + 1] * D)):
            sh = tuple((idx[d] + off[d] - R) % grid[d] for d in range(D))
            near[sh] = True
    out = []
    while len(out) < count:
        c = tuple(int(rng.integers(0, g)) for g in grid)
        x = c[-1]
        if x < xmargin + R or x > grid[-1] - 1 - xmargin - R or near[c]:
            continue
        out.append(c)
    return out


def window(arr, c, lead):
    """Periodic window of radius R around c over the trailing grid axes of arr."""
    sl = arr
    for d, cd in enumerate(c):
        ax = lead + d
        n = arr.shape[ax]
        ids = np.arange(cd - R, cd + R + 1) % n
        sl = np.take(sl, ids, axis=ax)
    return sl


def check(lbmib, solver, case, dim, samples, tol):
    lat = for_dim(dim)
    prm = window_params(case)
    f0, e0, H0 = solver.get_state()
    solver.step(1)
    f1, e1, _ = solver.get_state()
    scale_f = np.abs(f1 - lat.w.reshape((-1,) + (1,) * dim)).max()
    scale_e = np.abs(e1).max()
    worst = 0.0
    ctr = (R,) * dim
    for c in samples:
        st = olbm.State(f=window(f0, c, 1), rhoE=window(e0, c, 0), H1=np.zeros((2 * R + 1,) * dim),
                        H2=window(H0, c, 2))
        new = olbm.lbm_step(lat, prm, st)
        df = np.abs(new.f[(slice(None),) + ctr] - f1[(slice(None),) + c]).max() / scale_f
        de = abs(new.rhoE[ctr] - e1[c]) / scale_e
        worst = max(worst, df, de)
    print(f'{len(samples)} sampled nodes: worst relative difference {worst:.2e}', flush=True)
    assert worst <= tol


@pytest.mark.parametrize('precision', [32, 64])
def test_sphere_full_size_sampled(lbmib, precision):
    """The 384 x 192 x 192 sphere (FP32: the benchmark workload and launch configuration)."""
    case = wl.config2(reynolds=300.0)
    s = lbmib.Solver.from_case(case, precision=precision)
    s.step(20)
    g = s.geometry()
    grid = (case.dims[2], case.dims[1], case.dims[0])
    samples = pick_samples(grid, g['rows'], 40, seed=5, xmargin=3)
    check(lbmib, s, case, 3, samples, 1e-5 if precision == 32 else 1e-12)


def test_batch_full_size_sampled(lbmib):
    """The 64-case batch (FP32, autotuned tiles, graph-replayed steps as benchmarked)."""
    cases = wl.batched_cases(64)
    sols = [lbmib.Solver.from_case(c, precision=32) for c in cases]
    batch = lbmib.Batch(sols, autotune=True)
    batch.step(20)
    lat = for_dim(2)
    picks = [0, 17, 40, 63]
    before = {k: sols[k].get_state() for k in picks}
    batch.step(1)
    worst = 0.0
    for k in picks:
        c = cases[k]
        prm = window_params(c)
        f0, e0, H0 = before[k]
        f1, e1, _ = sols[k].get_state()
        grid = (c.dims[1], c.dims[0])
        samples = pick_samples(grid, sols[k].geometry()['rows'], 10, seed=k, xmargin=3)
        scale_f = np.abs(f1 - lat.w.reshape((-1, 1, 1))).max()
        scale_e = np.abs(e1).max()
        for cc in samples:
            st = olbm.State(f=window(f0, cc, 1), rhoE=window(e0, cc, 0), H1=np.zeros((2 * R + 1,) * 2),
                            H2=window(H0, cc, 2))
            new = olbm.lbm_step(lat, prm, st)
            df = np.abs(new.f[:, R, R] - f1[(slice(None),) + cc]).max() / scale_f
            de = abs(new.rhoE[R, R] - e1[cc]) / scale_e
            worst = max(worst, df, de)
    print('batch config', batch.config(), f'worst relative difference {worst:.2e}', flush=True)
    assert worst <= 1e-5
    batch.close()
