"""Throughput of the fused LBM + FODIBM-R time step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision 32|64] [--gpus 1]

Workload: the 384 x 192 x 192 D3Q19 box with a D = 32 sphere (3217 Fibonacci markers,
no-slip adiabatic wall, Ma 0.3, Re 300, FODIBM-R), inputs resident in HBM before the timed
region. One step = marker interpolation + reconstruction + forces, spreading, and the grid
sweep (collision, streaming, LB fluxes, MUSCL energy update), i.e. every row of the hot path.
Prints one JSON line. The FP64 CPU oracle is timed beside it on a bounded crop of the same
problem (the sphere in a 96 x 48 x 48 box).

    python bench.py --copy-kernel BYTES

runs only a plain device-to-device copy of BYTES bytes (the reference kernel that the
rocprofv3 FETCH_SIZE / WRITE_SIZE counters are calibrated against).
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak


def state_values_per_node(dim, q):
    """Values of the minimal state one node update must read and write: populations,
    rho E and the dense (diagonal, traceless) force history."""
    return q + 1 + (dim - 1)


def sweep_sources_hash():
    h = hashlib.sha1()
    for f in ('node_math.hpp', 'lattice.hpp', 'sweep_split.hip', 'sweep_fused.hip'):
        p = os.path.join(ROOT, 'paper_2607_07432_amd', 'csrc', f)
        if os.path.exists(p):
            h.update(open(p, 'rb').read())
    return h.hexdigest()[:12]


def read_traffic(kernel_tag, hash_now):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources; None otherwise."""
    path = os.path.join(ROOT, 'profiles', f'{kernel_tag}_traffic.md')
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith('|') and ':' not in line.split('|')[1]:
            parts = [p.strip() for p in line.strip().strip('|').split('|')]
            if len(parts) >= 2:
                fields[parts[0]] = parts[1]
    if fields.get('sources_hash') != hash_now:
        return None
    try:
        return float(fields['hbm_bytes_per_launch'])
    except (KeyError, ValueError):
        return None


def copy_kernel(nbytes):
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device='cuda:0')
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({'copy_bytes': n * 4, 'launches': 3}))


def measured_copy_gbs(nbytes=2 << 30, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second, GB/s), median of reps
    copies of nbytes timed with events on the current stream."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device='cuda:0')
    b = torch.empty_like(a)
    b.copy_(a)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)[reps // 2]
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def cpu_baseline(seconds_hint=20.0):
    """FP64 oracle on a bounded crop: the same sphere (D = 32, 3217 markers) in 96 x 48 x 48."""
    from oracle import ib as oib
    from oracle import lbm as olbm
    from oracle.lattice import for_dim
    from paper_2607_07432_amd import workloads as wl
    case = wl.config2(nx=96, ny=48, nz=48, reynolds=300.0)
    lat = for_dim(3)
    prm = olbm.Params(mu=case.mu, lam=case.lam, gamma=case.gamma, sigma=case.sigma, rho_inf=case.rho_inf,
                      u_inf=tuple(case.u_inf), T_inf=case.T_inf, bc=case.bc)
    geom = oib.build_geometry(case.dims, case.X, case.n, case.method, case.kernel)
    mk = oib.Markers(case.u_wall, case.t_kind, case.t_value)
    st = olbm.freestream_state(lat, prm, tuple(case.dims[::-1]))
    t0 = time.perf_counter()
    steps = 0
    while True:
        fib, fE, _ = oib.ib_step_forcing(lat, prm, geom, mk, st)
        st = olbm.lbm_step(lat, prm, st, fib, fE)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_hint or steps >= 40:
            break
    glups = case.n_nodes * steps / el / 1e9
    return {'value': glups, 'unit': 'GLUPS', 'cores': 1, 'kind': 'oracle',
            'sample': f'FP64 NumPy oracle, sphere D=32 with 3217 markers in a 96x48x48 crop '
                      f'({case.n_nodes} nodes), {steps} FODIBM-R steps in {el:.1f} s, single thread '
                      f'({platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()})'}


def bench_batch(args):
    """64 uneven 2D ellipse cases (256x128 .. 1024x512, FP32) in one batch: graph-replayed steps."""
    import torch
    from paper_2607_07432_amd import lbmib
    from paper_2607_07432_amd import workloads as wl
    cases = wl.batched_cases(64)
    prec = lbmib.F64 if args.precision == 64 else lbmib.F32
    sols = [lbmib.Solver.from_case(c, precision=prec) for c in cases]
    N = sum(c.n_nodes for c in cases)
    M = sum(len(c.X) for c in cases)
    t0 = time.perf_counter()
    batch = lbmib.Batch(sols, autotune=True)
    cfg = batch.config()
    print(f'[bench] batch of {len(cases)} cases, N={N}, markers={M}, tuned {cfg} in '
          f'{time.perf_counter() - t0:.1f} s', file=sys.stderr, flush=True)
    batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    glups = N * args.steps / (t1 - t0) / 1e9
    kernel_ms = batch.step_timed(min(args.steps, 50))
    res = batch.residuals()
    bad = [k for k, r in enumerate(res) if not np.isfinite(r)]
    n_bad = len(bad)
    for k in bad:
        c = cases[k]
        print(f'[bench] case {k} non-finite: {c.dims} Ma {c.extra["mach"]:.3f} Re {c.extra["reynolds"]:.1f} '
              f'tau {3 * c.mu + 0.5:.4f} kappa {wl.conduction_number(c):.3f}', file=sys.stderr, flush=True)
    print(f'[bench] {ms_per_step:.3f} ms/step, {glups:.2f} GLUPS (graph replay), kernels (markers, spread, '
          f'sweep) ms {kernel_ms.round(4).tolist()}, residual max {np.nanmax(res):.3e}', file=sys.stderr, flush=True)
    vals = state_values_per_node(2, 9)
    bytes_per_node = 2 * vals * (args.precision // 8)
    sweep_ms = float(kernel_ms[2])
    achieved = bytes_per_node * N / (sweep_ms * 1e-3) / 1e9
    out = {
        'metric': 'GLUPS of fused LBM+FODIBM step (batched 2D cases)',
        'value': round(glups, 4), 'unit': 'GLUPS', 'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': round(ms_per_step, 5), 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': f'f{args.precision}', 'data': 'synthetic',
        'config': {'workload': 'batch64: 64 uneven D2Q9 ellipse cases 256x128..1024x512, 64..256 markers, '
                               'FODIBM-R adiabatic no-slip, Ma 0.1-0.5, Re 20-200, one persistent graph-replayed step',
                   'nodes': N, 'markers': M, 'tuned': cfg, 'parallelism': 'single GPU'},
        'roofline': {'bound': 'hbm', 'kernel': 'persistent batched fused sweep', 'achieved': round(achieved, 1),
                     'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4),
                     'bytes_per_node': bytes_per_node, 'sweep_ms': round(sweep_ms, 5),
                     'traffic': read_traffic('batch64_d2q9_f32', sweep_sources_hash())
                     if args.precision == 32 and cfg.get('tile_x') == 254 else None},
        'kernel_ms': {'markers': round(float(kernel_ms[0]), 5), 'spread': round(float(kernel_ms[1]), 5),
                      'sweep': round(sweep_ms, 5)},
        'nonfinite_cases': n_bad,
    }
    batch.close()
    copy_gbs = measured_copy_gbs()
    out['roofline']['measured_copy_gbs'] = round(copy_gbs, 1)
    out['roofline']['frac_of_copy'] = round(achieved / copy_gbs, 4)
    print(json.dumps(out))


def bench_learned(args):
    """Learned warm start on 256 x 128 ellipses: solver-generated steady data, training, and the
    time to steady state (FP64, r < 1e-8) warm vs cold on held-out seeds."""
    from paper_2607_07432_amd import learned
    argv = ['--train', str(args.train_cases), '--heldout', str(args.heldout_cases), '--epochs', str(args.epochs),
            '--shape', args.shape, '--clip', str(args.clip), '--warmup-epochs', str(args.warmup_epochs),
            '--eval-tol', str(args.eval_tol)]
    if args.eval_shapes:
        argv += ['--eval-shapes', args.eval_shapes]
    ev = learned.main(argv)
    out = {
        'metric': f'time-to-steady warm vs cold at L2 residual {args.eval_tol:g} (FP64), 256x128 {ev["eval_shape"]}s',
        'value': round(ev['speedup_wall'], 4), 'unit': 'x (cold wall time / warm wall time incl. inference)',
        'n_gpus': 1, 'steps': None, 'warmup': 0, 'ms_per_step': None, 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f64 solver, bf16 network', 'data': 'synthetic',
        'config': {'workload': f'learned: {args.train_cases} steady training cases ({args.shape}), {args.heldout_cases} '
                               f'held-out seeds ({ev["eval_shape"]}), {args.epochs} epochs, 5-level U-Net 32..256 '
                               'channels'},
        'roofline': {'bound': 'mfma', 'kernel': 'U-Net training step (forward + backward + Adam), batch 16',
                     'achieved': round(ev['train_tflops'], 2), 'peak': 2500.0, 'unit': 'TFLOP/s',
                     'frac': round(ev['train_tflops'] / 2500.0, 4), 'traffic': None},
        'learned': ev,
    }
    print(json.dumps(out))


def bench_methods(args):
    """DIBM vs FODIBM vs FODIBM-R on the same bodies (fixed and turning walls): boundary-condition
    errors, loads and the per-step cost of each method."""
    from paper_2607_07432_amd import methods
    log = lambda msg: print(f'[methods] {msg}', file=sys.stderr, flush=True)
    res = methods.compare(quick=args.quick, log=log)
    red_dir = methods.reduction(res, 0, 'eps_dir')
    sph = res[3]['methods']
    cost = None
    if sph['FODIBM-R'].get('finite') and sph['FODIBM'].get('finite'):
        cost = 100.0 * (sph['FODIBM-R']['step_ms'] - sph['FODIBM']['step_ms']) / sph['FODIBM']['step_ms']
    out = {
        'metric': 'change of the mean no-slip error, FODIBM-R vs FODIBM (cylinder, Re 40, isothermal)',
        'value': None if red_dir is None else round(red_dir, 3), 'unit': '%', 'n_gpus': 1, 'steps': None,
        'warmup': 0, 'ms_per_step': None, 'higher_is_better': False, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f64 (2D), f32 (3D)', 'data': 'synthetic',
        'config': {'workload': 'methods: DIBM / FODIBM / FODIBM-R on a 200x100 cylinder at Ma 0.1 (isothermal, adiabatic, '
                               'turning) and a 384x192x192 sphere (fixed, turning at omega* 0.3 and 0.6)'},
        'reconstruction_cost_pct': None if cost is None else round(cost, 3),
        'changes_pct': {
            'eps_dir_isothermal_cylinder': red_dir,
            'eps_iso_isothermal_cylinder': methods.reduction(res, 0, 'eps_iso'),
            'eps_dir_adiabatic_cylinder': methods.reduction(res, 1, 'eps_dir'),
            'eps_neu_adiabatic_cylinder': methods.reduction(res, 1, 'eps_neu'),
            'eps_dir_turning_cylinder': methods.reduction(res, 2, 'eps_dir'),
            'eps_dir_sphere': methods.reduction(res, 3, 'eps_dir'),
            'eps_neu_sphere': methods.reduction(res, 3, 'eps_neu'),
        },
        'cases': res,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=100)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--precision', type=int, default=32, choices=(32, 64))
    ap.add_argument('--reynolds', type=float, default=300.0)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--copy-kernel', type=int, default=0)
    ap.add_argument('--sweep', choices=('fused', 'threepass'), default='fused')
    ap.add_argument('--workload', choices=('sphere3d', 'batch64', 'learned', 'methods'), default='sphere3d')
    ap.add_argument('--quick', action='store_true', help='methods workload: shorter runs')
    ap.add_argument('--train-cases', type=int, default=2000)
    ap.add_argument('--heldout-cases', type=int, default=512)
    ap.add_argument('--epochs', type=int, default=240)
    ap.add_argument('--shape', choices=('ellipse', 'star', 'mixed'), default='ellipse',
                    help='learned workload: bodies of the training cases')
    ap.add_argument('--eval-shapes', default=None, help='learned workload: bodies of the held-out cases')
    ap.add_argument('--clip', type=float, default=1.0, help='learned workload: gradient-norm clipping (0: off)')
    ap.add_argument('--warmup-epochs', type=float, default=1.0, help='learned workload: linear learning-rate warm-up')
    ap.add_argument('--eval-tol', type=float, default=1e-8, help='learned workload: residual of the held-out comparison')
    args = ap.parse_args()

    if args.gpus != 1:
        print(f'bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slab '
              'decomposition is designed (z slabs with one halo exchange per step) but not implemented.', file=sys.stderr)
        sys.exit(2)
    if args.copy_kernel:
        copy_kernel(args.copy_kernel)
        return
    if args.workload == 'batch64':
        bench_batch(args)
        return
    if args.workload == 'learned':
        bench_learned(args)
        return
    if args.workload == 'methods':
        bench_methods(args)
        return

    import torch
    from paper_2607_07432_amd import lbmib
    from paper_2607_07432_amd import workloads as wl

    case = wl.config2(reynolds=args.reynolds)
    solver = lbmib.Solver.from_case(case, precision=args.precision,
                                    sweep=lbmib.SWEEP_FUSED if args.sweep == 'fused' else lbmib.SWEEP_THREE_PASS)
    N = case.n_nodes
    print(f'[bench] {case.name} {case.dims} N={N} markers={len(case.X)} precision=f{args.precision}',
          file=sys.stderr, flush=True)

    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms = solver.step_timed(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    glups = N * args.steps / (t1 - t0) / 1e9
    resid = solver.residual()
    loads = solver.loads()
    print(f'[bench] {ms_per_step:.3f} ms/step, {glups:.2f} GLUPS, kernels (markers, spread, sweep) ms '
          f'{kernel_ms.round(4).tolist()}, Cd {loads["Cd"]:.4f}, residual {resid:.3e}', file=sys.stderr, flush=True)

    vals = state_values_per_node(3, 19)
    bytes_per_node = 2 * vals * (args.precision // 8)
    sweep_ms = float(kernel_ms[2])
    achieved = bytes_per_node * N / (sweep_ms * 1e-3) / 1e9
    tag = f'sweep_d3q19_f{args.precision}_384x192x192'
    traffic = read_traffic(tag, sweep_sources_hash())
    out = {
        'metric': 'GLUPS of fused LBM+FODIBM step; time-to-steady warm vs cold at L2 tol',
        'value': round(glups, 4), 'unit': 'GLUPS', 'n_gpus': 1, 'steps': args.steps, 'warmup': args.warmup,
        'ms_per_step': round(ms_per_step, 5), 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': f'f{args.precision}', 'data': 'synthetic',
        'config': {'workload': 'sphere3d: D3Q19 384x192x192, sphere D=32, 3217 markers, FODIBM-R, '
                               f'adiabatic no-slip, Ma 0.3, Re {args.reynolds:g}, inflow/outflow in x',
                   'nodes': N, 'markers': len(case.X), 'method': 'FODIBM-R', 'parallelism': 'single GPU'},
        'roofline': {'bound': 'hbm', 'kernel': f'grid sweep, {args.sweep} (collision + streaming + fluxes + energy)',
                     'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                     'frac': round(achieved / HBM_PEAK_GBS, 4),
                     'bytes_per_node': bytes_per_node, 'sweep_ms': round(sweep_ms, 5),
                     'traffic': traffic},
        'kernel_ms': {'markers': round(float(kernel_ms[0]), 5), 'spread': round(float(kernel_ms[1]), 5),
                      'sweep': round(sweep_ms, 5)},
        'Cd': loads['Cd'], 'residual': resid,
    }
    solver.close()
    del solver
    torch.cuda.empty_cache()
    copy_gbs = measured_copy_gbs()
    out['roofline']['measured_copy_gbs'] = round(copy_gbs, 1)
    out['roofline']['frac_of_copy'] = round(achieved / copy_gbs, 4)
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline()
    print(json.dumps(out))


if __name__ == '__main__':
    main()
