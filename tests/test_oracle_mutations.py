"""Seeded mistakes in the oracle are caught by its pins.

Each case copies the oracle package into a temporary directory, plants one plausible mistake
(a dropped term, a flipped sign, a wrong factor or index) by replacing one exact line fragment,
and runs the pins named for it against the mutated copy in a fresh interpreter that writes and
reads no bytecode cache. The pins must fail. The mistakes are planted on the CPU only; the HIP
path is not involved.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
T = 'tests/'

# (oracle file, exact fragment, replacement, pins that must fail, what the mistake is)
MUTATIONS = [
    ('lattice.py', 'by_speed = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}', 'by_speed = {0: 1 / 3, 1: 1 / 18, 2: 1 / 18}',
     T + 'test_oracle_lattice.py::test_equilibrium_moments', 'D3Q19 weight of a diagonal (Eq. (A.2))'),
    ('lattice.py', '[(1, _XXY), (-1, _YZZ)]', '[(1, _XXY), (-1, _YYZ)]',
     T + 'test_oracle_lattice.py::test_3r_basis_orthogonal_with_known_norms', 'H_4 as printed in Eq. (A.6)'),
    ('lbm.py', 'rest * rho * (theta - 1.0)', 'rest * rho * (1.0 - theta)',
     T + 'test_oracle_lattice.py::test_equilibrium_moments', 'sign of the rest-population temperature term, Eq. (A.3)'),
    ('lbm.py', 'h2uu * rho / (2 * cs2 ** 2)', 'h2uu * rho / (cs2 ** 2)',
     T + 'test_oracle_lattice.py::test_equilibrium_moments', 'second-order equilibrium factor'),
    ('lbm.py', 'return w * (h2pi / (2 * cs2 ** 2)) + w * h3', 'return w * (h2pi / (2 * cs2 ** 2))',
     T + 'test_oracle_lattice.py::test_regularized_neq_moments', 'recursive Pi^(3) of Eq. (A.8) dropped'),
    ('lbm.py', "np.einsum('ia,a...->i...', lat.h1, fu) / cs2", "np.einsum('ia,a...->i...', lat.h1, fu) * cs2",
     T + 'test_oracle_lattice.py::test_force_population_moments', 'first-order force factor, Eq. (7)'),
    ('lbm.py', 'eye * cs2 * dgdt + aC + fu_uf', 'eye * cs2 * dgdt + aC',
     T + 'test_oracle_lbm.py::test_uniform_forcing_and_force_history', 'f u + u f of Eq. (A.9) dropped'),
    ('lbm.py', '+ 0.5 * st.H2)', ')',
     T + 'test_oracle_lbm.py::test_uniform_forcing_and_force_history', 'F(t - dt)/2 of Eq. (A.7) dropped'),
    ('lbm.py', '(1.0 - 1.0 / taubar) * fneq + 0.5 * F', '(1.0 - 1.0 / taubar) * fneq + 1.0 * F',
     T + 'test_oracle_lbm.py::test_uniform_forcing_and_force_history', 'F/2 of Eq. (6) doubled'),
    ('lbm.py', 'taubar = prm.mu / (rho * cs2) + 0.5', 'taubar = prm.mu / (rho * cs2) + 0.4',
     T + 'test_oracle_lbm.py::test_shear_wave_decay_literal_tau', 'tau-bar = tau + 1/2 of Eq. (6)'),
    ('lbm.py', 'prm.gamma * p_cs2 * div', 'p_cs2 * div',
     T + 'test_oracle_lbm.py::test_acoustic_attenuation_at_rest',
     'gamma of the pressure balance in d/dt[rho(1 - theta)]'),
    ('lbm.py', 'aF = (2.0 / D) * eye * rho * cs2 * div', 'aF = (1.0 / D) * eye * rho * cs2 * div',
     T + 'test_oracle_lbm.py::test_acoustic_attenuation_at_rest', '(2/D) rho cs^2 div u term of Eq. (A.9)'),
    ('lbm.py', 'part = 0.5 * (fcol[i] + at(fcol[i], unit(D, a, 1) - ci, D))',
     'part = 0.5 * (fcol[i] + at(fcol[i], unit(D, a, 1) + ci, D))',
     T + 'test_oracle_lbm.py::test_general_flux_rule_matches_explicit_d3q19_terms', 'face-flux stencil, Eqs. (A.11)-(A.13)'),
    ('lbm.py', 'eta = (2.0 * u - sign0(u, u_zero)) / 3.0', 'eta = (2.0 * u + sign0(u, u_zero)) / 3.0',
     T + 'test_oracle_lbm.py::test_muscl_update_is_third_order', 'sign term of eta, Eq. (A.16)'),
    ('lbm.py', 'eta = (2.0 * u - sign0(u, u_zero)) / 3.0', 'eta = 0.0 * u',
     T + 'test_oracle_lbm.py::test_muscl_update_is_third_order', 'eta = 0 (second-order slope)'),
    ('lbm.py', 'left = phi + 0.5 * slope(phi, ua) * (1.0 - ua)', 'left = phi + 0.5 * slope(phi, ua)',
     T + 'test_oracle_lbm.py::test_advected_entropy_wave', 'Hancock predictor (1 - u) of Eq. (A.15) dropped'),
    ('lbm.py', 'return np.where(utilde >= -u_zero, left, right)', 'return np.where(utilde >= -u_zero, right, left)',
     T + 'test_oracle_lbm.py::test_advected_entropy_wave', 'downwind instead of upwind state, Eq. (A.14)'),
    ('lbm.py', 'flux = flux + hk_f * (Frho[a] - muscl_face(rho * ua, ua, a, D, uz))', 'flux = flux',
     T + 'test_oracle_lbm.py::test_advected_entropy_wave', '(h - k)[F^rho - F*(rho u)] of Eq. (11) dropped'),
    ('lbm.py', 'flux = flux + ub_f * (Fmom[a, b] - muscl_face(phi, ua, a, D, uz))', 'flux = flux',
     T + 'test_oracle_lbm.py::test_advected_entropy_wave', 'u_b[F^(rho u_b) - F*(...)] of Eq. (11) dropped'),
    ('lbm.py', 'H = k + prm.Cv * T + p / rho', 'H = prm.Cv * T + p / rho',
     T + 'test_oracle_lbm.py::test_advected_entropy_wave', 'kinetic energy missing from H'),
    ('lbm.py', 'hk_f = 0.5 * ((h - k) + at(h - k, e, D))', 'hk_f = 0.5 * ((h + k) + at(h + k, e, D))',
     T + 'test_oracle_lbm.py::test_energy_flux_correction_weights', '(h + k) for (h - k) in Eq. (11)'),
    ('lbm.py', 'flux = flux - prm.lam * (at(T, e, D) - T)', 'flux = flux + prm.lam * (at(T, e, D) - T)',
     T + 'test_oracle_lbm.py::test_thermal_mode_decay', 'sign of the conduction flux'),
    ('lbm.py', 'return np.stack([at(fcol[i], -lat.c[i], D) for i in range(lat.Q)])',
     'return np.stack([at(fcol[i], lat.c[i], D) for i in range(lat.Q)])',
     T + 'test_oracle_lbm.py::test_discrete_mass_and_momentum_flux_identities', 'push instead of pull streaming'),
    ('lbm.py', 'rhoE_new = st.rhoE - div + fE', 'rhoE_new = st.rhoE + div + fE',
     T + 'test_oracle_lbm.py::test_thermal_mode_decay', 'sign of the flux divergence in Eq. (10)'),
    ('lbm.py', 'scale = (prm.rho_inf * prm.T_inf) / (rho3 * T3)', 'scale = (rho3 * T3) / (prm.rho_inf * prm.T_inf)',
     T + 'test_oracle_lbm.py::test_inflow_outflow_closure', 'outlet pressure rescaling inverted'),
    ('lbm.py', 'T = (rhoE / rho - 0.5 * (u * u).sum(axis=0)) / prm.Cv', 'T = (rhoE / rho - 0.5 * (u * u).sum(axis=0)) / prm.Cp',
     T + 'test_oracle_lbm.py::test_freestream_is_a_fixed_point', 'Cp for Cv in T from rho E'),
    ('lbm.py', 'eta = (2.0 * u - sign0(u, u_zero)) / 3.0', 'eta = (2.0 * u - np.sign(u)) / 3.0',
     T + 'test_oracle_lbm.py::test_muscl_dead_zone_keeps_symmetry_and_bounds_its_effect', 'no MUSCL dead zone'),
    ('ib.py', '(1.0 + np.cos(np.pi * r / d)) / (2.0 * d)', '(1.0 + np.cos(np.pi * r / d)) / (4.0 * d)',
     T + 'test_oracle_ib.py::test_cos_kernel_tabulated_values', 'kernel normalisation, Eq. (19)'),
    ('ib.py', 'inner = (1.0 + np.sqrt(np.maximum(1.0 - 3.0 * a * a, 0.0))) / 3.0',
     'inner = (1.0 + np.sqrt(np.maximum(1.0 - 3.0 * a * a, 0.0))) / 2.0',
     T + 'test_oracle_ib.py::test_roma3_partition_and_first_moment', 'ROMA3 inner branch'),
    ('ib.py', 'out[k] = dot[l] <= 0.0', 'out[k] = dot[l] < 0.0',
     T + 'test_oracle_ib.py::test_cylinder_interior_equals_closed_disk', 'open instead of closed interior'),
    ('ib.py', 'phi[l] = 1.0 / s if one_sided else 1.0', 'phi[l] = 1.0',
     T + 'test_oracle_ib.py::test_flat_wall_worked_values', 'phi of Eq. (16) dropped'),
    ('ib.py', 'W[l] = 1.0 / tot', 'W[l] = 1.0',
     T + 'test_oracle_ib.py::test_flat_wall_worked_values', 'W of Eq. (17) dropped'),
    ('ib.py', 'ut = ub - ratio * (uP - ub)', 'ut = ub + ratio * (uP - ub)',
     T + 'test_oracle_ib.py::test_linear_profile_reconstruction_exact', 'sign of the extrapolation, Eq. (27)'),
    ('ib.py', 'Tt = tv - ratio * (TP - tv)', 'Tt = tv + ratio * (TP - tv)',
     T + 'test_oracle_ib.py::test_isothermal_reconstruction_and_heat_source', 'sign of the T extrapolation, Eq. (27)'),
    ('ib.py', 'Tt = TP - tv * (D_N + geom.dBV[l])', 'Tt = TP - tv * (D_N - geom.dBV[l])',
     T + 'test_oracle_ib.py::test_neumann_reconstruction_with_gradient', 'd_PB - d_BV in Eq. (29)'),
    ('ib.py', 'Tt = TP - tv * D_N', 'Tt = TP + tv * D_N',
     T + 'test_oracle_ib.py::test_fodibm_thermal_targets', 'sign of the FODIBM Neumann target'),
    ('ib.py', "out['F'][l] = 2.0 * (r_l * ut - j_l)", "out['F'][l] = 1.0 * (r_l * ut - j_l)",
     T + 'test_oracle_ib.py::test_moving_wall_targets', 'factor 2 of Eqs. (20)/(30)'),
    ('ib.py', "out['Wib'][l] = r_l * ((ut * ut).sum() - (u_l * u_l).sum()) / 2.0",
     "out['Wib'][l] = r_l * ((ut * ut).sum() - (u_l * u_l).sum()) / 1.0",
     T + 'test_oracle_ib.py::test_moving_wall_targets', 'factor 1/2 of Eqs. (21)/(31)'),
    ('ib.py', 'prm.Cv * r_l * (Tt - T_l)', 'r_l * (Tt - T_l)',
     T + 'test_oracle_ib.py::test_isothermal_reconstruction_and_heat_source', 'Cv of Eqs. (22)/(32)'),
    ('ib.py', 'fib[r] = (s[:, None] * F[k]).sum(axis=0)', 'fib[r] = 2.0 * (s[:, None] * F[k]).sum(axis=0)',
     T + 'test_oracle_ib.py::test_spread_conserves_total_force', 'spreading weight of Eq. (15)'),
    ('loads.py', "Fb = -(mf['F'][act] * geom.W[act, None]).sum(axis=0)", "Fb = (mf['F'][act] * geom.W[act, None]).sum(axis=0)",
     T + 'test_oracle_loads.py::test_body_force_and_heat_balance_one_step', 'sign of the body force'),
    ('loads.py', "Qh = (mf['Qib'][act] * geom.W[act]).sum()", "Qh = (mf['Qib'][act]).sum()",
     T + 'test_oracle_loads.py::test_nusselt_of_radial_conduction', 'marker weight missing from Q_heat'),
    ('loads.py', 'q = 0.5 * rho_inf * u_ref * u_ref * ref_area', 'q = rho_inf * u_ref * u_ref * ref_area',
     T + 'test_oracle_loads.py::test_drag_of_a_cosine_pressure_on_a_circle', 'dynamic pressure without 1/2'),
    ('loads.py', '(lam * (T_wall - T_inf) * surface)', '(lam * (T_wall - T_inf) * ref_area)',
     T + 'test_oracle_loads.py::test_nusselt_of_radial_conduction', 'Nu over the frontal length'),
    ('loads.py', 'e_iso.append(abs(Ts - mk.t_value[l]) / mk.t_value[l])', 'e_iso.append(abs(Ts - mk.t_value[l]) / T_inf)',
     T + 'test_oracle_loads.py::test_bc_errors_on_linear_fields', 'normaliser of Eq. (38)'),
    ('loads.py', '(TPs - Ts) / D_N - mk.t_value[l]', '(TPs - Ts) / 1.0 - mk.t_value[l]',
     T + 'test_oracle_loads.py::test_bc_errors_on_linear_fields', 'd_n of Eq. (36)'),
    ('loads.py', '(u_ref * np.sqrt(N))', '(u_ref * N)',
     T + 'test_oracle_loads.py::test_residual_of_known_differences', 'sqrt(N) of the residual'),
    ('unet.py', 'u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000', 'u = (u + 0x8000) & 0xFFFF0000',
     T + 'test_oracle_unet.py::test_bf16_rounding_values', 'bf16 ties away from even'),
    ('unet.py', "return X.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))",
     "return X.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))",
     T + 'test_oracle_unet.py::test_pool_and_up_adjoints', 'sum instead of mean pooling'),
    ('unet.py', 'g = 2.0 * m[..., None] * (out - tgt) / cnt', 'g = 1.0 * m[..., None] * (out - tgt) / cnt',
     T + 'test_oracle_unet.py::test_backward_matches_finite_differences', 'loss gradient factor'),
    ('unet.py', 'mh = m / (1 - b1 ** t)', 'mh = m',
     T + 'test_oracle_unet.py::test_adam_first_step_closed_form', 'Adam bias correction dropped'),
    ('unet.py', 'g * (max_norm / norm)', 'g * (norm / max_norm)',
     T + 'test_oracle_unet.py::test_clip_grad_norm_closed_form', 'clipping factor inverted'),
    ('warmstart.py', 'inside = s < 0.0', 'inside = s > 0.0',
     T + 'test_oracle_unet.py::test_signed_distance_of_a_circle', 'sign of the signed distance'),
    ('warmstart.py', "out[..., 0] = (rho - rho_inf) / (rho_inf * m2)", "out[..., 0] = (rho - rho_inf) / rho_inf",
     T + 'test_oracle_unet.py::test_normalisation_of_free_stream_and_round_trip', 'density normalisation'),
    ('warmstart.py', 'taubar = prm.mu / (rho * cs2) + 0.5', 'taubar = prm.mu / (rho * cs2) + 0.0',
     T + 'test_oracle_unet.py::test_warm_state_moments_of_a_shear_flow', 'tau-bar of the warm-start stress'),
    ('lbm.py', 'p_n = pp - 0.5 * (L5 + L1)', 'p_n = pp - 0.5 * (L5 - L1)',
     T + 'test_oracle_outlet.py::test_incoming_wave_pulls_the_outlet_pressure_to_p_inf',
     'sign of the incoming wave in the outlet pressure (LODI)'),
    ('lbm.py', '(ux + c) * (dp + r * c * du[0])', '(ux + c) * dp',
     T + 'test_oracle_outlet.py::test_characteristic_outlet_absorbs_an_acoustic_pulse',
     'velocity part of the outgoing acoustic amplitude L5'),
    ('lbm.py', 'c = np.sqrt(prm.gamma * pp / r)', 'c = np.sqrt(pp / r)',
     T + 'test_oracle_outlet.py::test_characteristic_outlet_absorbs_an_acoustic_pulse',
     'isothermal instead of adiabatic sound speed at the outlet'),
    ('refine.py', 'lambda rho: _taubar(prm_f, rho) / (2.0 * _taubar(prm_c, rho))', 'lambda rho: 1.0 + 0.0 * rho',
     T + 'test_oracle_refine.py::test_shear_wave_crosses_the_block',
     'non-equilibrium populations not rescaled from coarse to fine'),
    ('refine.py', 'mu=2.0 * prm_c.mu, lam=2.0 * prm_c.lam', 'mu=prm_c.mu, lam=prm_c.lam',
     T + 'test_oracle_refine.py::test_shear_wave_crosses_the_block', 'fine viscosity not doubled in lattice units'),
    ('refine.py', 'fill_band(lat, prm, prm_f, states[k + 1], old, new, 0.5 * s, blocks[k])',
     'fill_band(lat, prm, prm_f, states[k + 1], old, new, 1.0, blocks[k])',
     T + 'test_oracle_refine.py::test_acoustic_pulse_crosses_the_block', 'no time interpolation of the band'),
    ('refine.py', 'frac.append((xf % 2) * 0.5)', 'frac.append((xf % 2) * 0.0)',
     T + 'test_oracle_refine.py::test_acoustic_pulse_crosses_the_block', 'no spatial interpolation of the band'),
    ('refine.py', 'hi.append((i0 + 1) % nc)', 'hi.append((i0 - 1) % nc)',
     T + 'test_oracle_refine.py::test_interpolation_reproduces_multilinear_fields', 'interpolation neighbour'),
    ('refine.py', 'lambda rho: 2.0 * _taubar(prm_c, rho) / _taubar(prm_f, rho)',
     'lambda rho: _taubar(prm_f, rho) / (2.0 * _taubar(prm_c, rho))',
     T + 'test_oracle_refine.py::test_transfer_there_and_back_is_the_identity',
     'restriction scales the non-equilibrium part like the prolongation'),
    ('refine.py', 'H2d = 0.5 * np.stack', 'H2d = 1.0 * np.stack',
     T + 'test_oracle_refine.py::test_transfer_there_and_back_is_the_identity', 'force history not halved on the fine level'),
    ('refine.py', '((x < G) | (x >= n - G))', '((x < G) | (x > n - G))',
     T + 'test_oracle_refine.py::test_band_and_restriction_sets', 'band one node short at the upper edges'),
    ('refine.py', 'i = i[(i >= block.R) & (i <= n - 1 - block.R)]', 'i = i[(i > block.R) & (i <= n - 1 - block.R)]',
     T + 'test_oracle_refine.py::test_band_and_restriction_sets', 'restriction margin off by one'),
    ('refine.py', 'advance(k + 1, prm_f)', 'advance(k + 1, prm_f if k == 0 else prm)',
     T + 'test_oracle_refine.py::test_shear_wave_error_falls_with_each_level', 'third level viscosity doubled once only'),
    ('refine.py', 'states[k] = restrict(lat, prm, prm_f, states[k], states[k + 1], blocks[k])',
     'states[k] = restrict(lat, prm, prm_f, states[k], states[k + 1], blocks[k]) if k == 0 else states[k]',
     T + 'test_oracle_refine.py::test_shear_wave_error_falls_with_each_level', 'inner level not restricted'),
    ('refine.py', 'states[k + 1] = fill_band(lat, prm, prm_f, states[k + 1], old, new, 0.5 * s, blocks[k])',
     'states[k + 1] = fill_band(lat, prm, prm_f, states[k + 1], old, new, 0.5 * s if k == 0 else 1.0, blocks[k])',
     T + 'test_oracle_refine.py::test_acoustic_pulse_crosses_a_nest_of_three_levels',
     'inner band taken from the end of the middle step'),
]


def _run(mut, tmp_root):
    fname, old, new, pins, what = mut
    src = os.path.join(ROOT, 'oracle', fname)
    text = open(src).read()
    if text.count(old) != 1:
        return mut, 'fragment not found exactly once'
    dst_root = os.path.join(tmp_root, f'm{MUTATIONS.index(mut)}')
    shutil.copytree(os.path.join(ROOT, 'oracle'), os.path.join(dst_root, 'oracle'),
                    ignore=shutil.ignore_patterns('__pycache__'))
    with open(os.path.join(dst_root, 'oracle', fname), 'w') as fh:
        fh.write(text.replace(old, new))
    env = dict(os.environ, PYTHONPATH=dst_root + os.pathsep + ROOT, PYTHONDONTWRITEBYTECODE='1',
               OMP_NUM_THREADS='1')
    # run from the copy's directory: `python -m` puts the working directory first on sys.path
    cmd = [sys.executable, '-B', '-m', 'pytest', '-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu',
           '--rootdir', ROOT] + [os.path.join(ROOT, p) for p in pins.split()]
    res = subprocess.run(cmd, cwd=dst_root, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    out = res.stdout.decode(errors='replace')
    if res.returncode == 1 and ' failed' in out:
        return mut, None
    return mut, f'pins did not fail (rc {res.returncode}): {out[-400:]}'


@pytest.mark.slow
def test_planted_mistakes_fail_their_pins(tmp_path):
    workers = min(4, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda m: _run(m, str(tmp_path)), MUTATIONS))
    survivors = [(m[0], m[4], why) for m, why in results if why]
    assert not survivors, survivors


def test_mutated_oracle_is_imported_from_the_copy(tmp_path):
    # the harness itself: a copy with a planted syntax error must be the one imported
    dst = tmp_path / 'oracle'
    shutil.copytree(os.path.join(ROOT, 'oracle'), dst, ignore=shutil.ignore_patterns('__pycache__'))
    (dst / 'lattice.py').write_text('raise ImportError("planted")\n')
    env = dict(os.environ, PYTHONPATH=str(tmp_path) + os.pathsep + ROOT, PYTHONDONTWRITEBYTECODE='1')
    res = subprocess.run([sys.executable, '-B', '-m', 'pytest', '-q', '-p', 'no:cacheprovider', '--rootdir', ROOT,
                          os.path.join(ROOT, T + 'test_oracle_lattice.py')], cwd=str(tmp_path), env=env,
                         stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    assert res.returncode != 0 and b'planted' in res.stdout
