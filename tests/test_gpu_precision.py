"""Precision of the FP32 sweep (deviation-stored populations) on the isothermal sphere of the
512 x 256 x 256 box (D = 32, T_w = 1.2 T_inf, Ma 0.2, Re 300), against the FP64 oracle on the
96^3 crop around the sphere, and FP32 against the GPU FP64 path on the full box.

Bars: GPU FP64 within 1e-11 of the oracle after 10 steps; FP32 within 1e-5 relative L2 error in
the fields and 1e-4 in Cd and Nu (the maximum-norm error is printed beside it).
"""
import numpy as np
import pytest

from oracle import lbm as olbm
from oracle import loads as oloads
from oracle.lattice import for_dim
from paper_2607_07432_amd import workloads as wl

from parity_util import oracle_geometry, oracle_markers, oracle_params, oracle_step, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def lbmib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip('no GPU')
    from paper_2607_07432_amd import lbmib as mod
    mod.load_library()
    return mod


def crop_case():
    # the sphere of the 512 x 256 x 256 configuration in a 96^3 box
    return wl.precision_case(nx=96, ny=96, nz=96, center=(38.3, 48.2, 47.9))


@pytest.fixture(scope='module')
def oracle_run():
    case = crop_case()
    lat = for_dim(3)
    prm = oracle_params(case)
    g = oracle_geometry(case)
    mk = oracle_markers(case)
    st = olbm.freestream_state(lat, prm, (96, 96, 96))
    mf = None
    for k in range(10):
        st, mf = oracle_step(case, st, g, mk)
        print('oracle step', k + 1, flush=True)
    Fb, Qh = oloads.body_loads(g, mf)
    Cd, Cl, Nu = oloads.coefficients(Fb, Qh, case.rho_inf, case.u_ref, case.ref_len, case.ref_area, case.surface,
                                     case.lam, case.T_wall, case.T_inf)
    return case, olbm.fields(lat, prm, st), st, (Cd, Nu)


def l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.mark.parametrize('precision', [64, 32])
def test_crop_against_oracle(lbmib, oracle_run, precision):
    case, (orho, ou, oT, _), st, (Cd, Nu) = oracle_run
    s = lbmib.Solver.from_case(case, precision=precision)
    s.step(10)
    rho, u, T, _ = s.fields()
    L = s.loads()
    er, eu, eT = l2(rho, orho), l2(u, ou), l2(T, oT)
    print(f'FP{precision}: relative L2 rho {er:.2e} u {eu:.2e} T {eT:.2e}; max-norm rho {rel(rho, orho):.2e} '
          f'u {rel(u, ou):.2e} T {rel(T, oT):.2e}; Cd {L["Cd"]:.6f}/{Cd:.6f} Nu {L["Nu"]:.5f}/{Nu:.5f}', flush=True)
    if precision == 64:
        f, e, _ = s.get_state()
        assert rel(f, st.f) <= 1e-11 and rel(e, st.rhoE) <= 1e-11
        assert abs(L['Cd'] - Cd) <= 1e-9 * abs(Cd) and abs(L['Nu'] - Nu) <= 1e-9 * abs(Nu)
    else:
        assert er <= 1e-5 and eT <= 1e-5 and eu <= 1e-5
        assert abs(L['Cd'] - Cd) <= 1e-4 * abs(Cd) and abs(L['Nu'] - Nu) <= 1e-4 * abs(Nu)


def test_full_box_fp32_against_fp64(lbmib):
    import torch
    case = wl.precision_case()
    out = {}
    for prec in (64, 32):
        s = lbmib.Solver.from_case(case, precision=prec)
        s.step(100)
        out[prec] = s.fields(), s.loads()
        s.close()
        del s
        torch.cuda.empty_cache()
    (r64, u64, T64, _), L64 = out[64]
    (r32, u32, T32, _), L32 = out[32]
    e = dict(rho=l2(r32, r64), u=l2(u32, u64), T=l2(T32, T64), rho_dev=l2(r32 - 1.0, r64 - 1.0),
             rho_max=rel(r32, r64), u_max=rel(u32, u64), T_max=rel(T32, T64),
             Cd=abs(L32['Cd'] - L64['Cd']) / abs(L64['Cd']), Nu=abs(L32['Nu'] - L64['Nu']) / abs(L64['Nu']))
    print('512x256x256, 100 steps, FP32 vs FP64:', e, flush=True)
    assert e['rho'] <= 1e-5 and e['u'] <= 1e-5 and e['T'] <= 1e-5
    assert e['Cd'] <= 1e-4 and e['Nu'] <= 1e-4
