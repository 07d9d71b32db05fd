"""Pins of the oracle's lattice, equilibrium, off-equilibrium and force populations.

Each check is a moment identity the Hermite construction of the paper's Appendix A
must satisfy (Eqs. (A.3)-(A.9)), evaluated on random fields; a dropped term, a
wrong coefficient or a transposed index in the oracle breaks one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice, lbm

LATS = [lattice.d2q9(), lattice.d3q19()]


def rnd_fields(lat, seed=0, shape=(3, 4)):
    rng = np.random.default_rng(seed)
    D = lat.D
    grid = shape if D == 2 else shape + (2,)
    rho = 1.0 + 0.1 * rng.standard_normal(grid)
    u = 0.1 * rng.standard_normal((D,) + grid)
    th = 1.0 + 0.1 * rng.standard_normal(grid)
    return rho, u, th


def test_printed_d3q19_weights_are_misprinted():
    # Eq. (A.2) as printed sums to 37/36 and disagrees with |c|^2 of Eq. (A.1) at entries 9, 10, 11.
    printed = lattice.printed_d3q19_weights()
    assert sum(printed) == Fraction(37, 36)
    lat = lattice.d3q19()
    bad = [i for i, (p, ci) in enumerate(zip(printed, lat.c))
           if p != {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[int((ci * ci).sum())]]
    assert bad == [9, 10, 11]


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_isotropy_exact(lat):
    D = lat.D
    assert lattice.exact_moment(lat, [0] * D) == 1
    for a in range(D):
        e = [0] * D
        e[a] = 1
        assert lattice.exact_moment(lat, e) == 0
        e[a] = 2
        assert lattice.exact_moment(lat, e) == Fraction(1, 3)
        e[a] = 4
        assert lattice.exact_moment(lat, e) == Fraction(1, 3)        # 3 cs^4
        for b in range(a + 1, D):
            e2 = [0] * D
            e2[a] = e2[b] = 2
            assert lattice.exact_moment(lat, e2) == Fraction(1, 9)   # cs^4
            e2[a] = e2[b] = 1
            assert lattice.exact_moment(lat, e2) == 0


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_opposites_and_paper_order(lat):
    assert (lat.c[lat.opp] == -lat.c).all()
    if lat.name == 'D3Q19':
        # opp(i) = i +- 9 in the paper's ordering, Eq. (A.1)
        assert all(lat.opp[i] == (i + 9 if i <= 9 else i - 9) for i in range(1, 19))


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_3r_basis_orthogonal_with_known_norms(lat):
    G = np.einsum('i,ik,il->kl', lat.w, lat.h3r, lat.h3r)
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-16
    cs6 = (1.0 / 3.0) ** 3
    expect = [2 * cs6] * 2 if lat.D == 2 else [2 * cs6] * 3 + [6 * cs6] * 3
    assert np.allclose(np.diag(G), expect, rtol=0, atol=1e-15)
    # orthogonal to H0, H1, H2
    assert np.abs(np.einsum('i,ik->k', lat.w, lat.h3r)).max() < 1e-16
    assert np.abs(np.einsum('i,ik,ia->ka', lat.w, lat.h3r, lat.h1)).max() < 1e-16
    assert np.abs(np.einsum('i,ik,iab->kab', lat.w, lat.h3r, lat.h2)).max() < 1e-16


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_equilibrium_moments(lat):
    D = lat.D
    rho, u, th = rnd_fields(lat)
    feq = lbm.equilibrium(lat, rho, u, th)
    cf = lat.c.astype(float)
    eye = np.eye(D).reshape((D, D) + (1,) * rho.ndim)
    assert np.abs(feq.sum(0) - rho).max() < 1e-15
    assert np.abs(np.einsum('ia,i...->a...', cf, feq) - rho * u).max() < 1e-15
    P = np.einsum('ia,ib,i...->ab...', cf, cf, feq)
    assert np.abs(P - (rho * u[:, None] * u[None] + eye * rho * th / 3.0)).max() < 1e-15
    a3r = lat.tensor3_to_3r(rho * u[:, None, None] * u[None, :, None] * u[None, None, :])
    assert np.abs(np.einsum('ik,i...->k...', lat.h3r, feq) - a3r).max() < 1e-15
    # the lattice's diagonal defect that the a^C correction addresses: sum f c_a^3 = rho u_a
    for a in range(D):
        assert np.abs(np.einsum('i,i...->...', cf[:, a] ** 3, feq) - rho * u[a]).max() < 1e-15
    # rest population: w_0 rho + (w_0 - 1) rho (theta - 1) at u = 0
    f0 = lbm.equilibrium(lat, rho, 0 * u, th)[0]
    assert np.abs(f0 - rho * (lat.w[0] + (lat.w[0] - 1.0) * (th - 1.0))).max() < 1e-15


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_regularized_neq_moments(lat):
    D = lat.D
    rng = np.random.default_rng(1)
    rho, u, th = rnd_fields(lat, 2)
    A = rng.standard_normal((D, D) + rho.shape)
    Pi = 0.5 * (A + A.transpose((1, 0) + tuple(range(2, A.ndim))))
    Pi = Pi - np.eye(D).reshape((D, D) + (1,) * rho.ndim) * sum(Pi[a, a] for a in range(D)) / D
    fneq = lbm.regularized_neq(lat, Pi, u)
    cf = lat.c.astype(float)
    assert np.abs(fneq.sum(0)).max() < 1e-15
    assert np.abs(np.einsum('ia,i...->a...', cf, fneq)).max() < 1e-15
    assert np.abs(np.einsum('ia,ib,i...->ab...', cf, cf, fneq) - Pi).max() < 1e-14
    Pi3 = (u[:, None, None] * Pi[None] + u[None, :, None] * Pi[:, None, :] + u[None, None, :] * Pi[:, :, None])
    assert np.abs(np.einsum('ik,i...->k...', lat.h3r, fneq) - lat.tensor3_to_3r(Pi3)).max() < 1e-15


@pytest.mark.parametrize('lat', LATS, ids=lambda l: l.name)
def test_force_population_moments(lat):
    D = lat.D
    rng = np.random.default_rng(3)
    rho, u, th = rnd_fields(lat, 4)
    fu = rng.standard_normal((D,) + rho.shape)
    A = rng.standard_normal((D, D) + rho.shape)
    aF = 0.5 * (A + A.transpose((1, 0) + tuple(range(2, A.ndim))))
    F = lbm.force_populations(lat, fu, aF)
    cf = lat.c.astype(float)
    assert np.abs(F.sum(0)).max() < 1e-14
    assert np.abs(np.einsum('ia,i...->a...', cf, F) - fu).max() < 1e-14
    assert np.abs(np.einsum('ia,ib,i...->ab...', cf, cf, F) - aF).max() < 1e-14
    dev = lbm.deviatoric_second_moment(lat, F)
    tr = sum(aF[a, a] for a in range(D))
    assert np.abs(dev - (aF - np.eye(D).reshape((D, D) + (1,) * rho.ndim) * tr / D)).max() < 1e-14


def test_printed_h4_is_not_orthogonal():
    # Eq. (A.6) prints H_4 = H_xxy - H_yyz. With that entry the "3r" set is no longer orthogonal
    # under the lattice weights (the Gram matrix couples H_4 with H_1, H_3 and H_6), so the
    # projection with the norms N_k would not reproduce the moments sum f^eq H^(3r)_k = a^(3r)_k;
    # the pairing of the other five (each sum/difference of the same two components) gives
    # H_4 = H_xxy - H_yzz, which is orthogonal to every other entry with norm 6 c_s^6.
    lat = lattice.d3q19()
    xxy = lat.h3[:, 0, 0, 1]
    yyz = lat.h3[:, 1, 1, 2]
    yzz = lat.h3[:, 1, 2, 2]
    printed = xxy - yyz
    gram = lambda a, b: float((lat.w * a * b).sum())
    others = [lat.h3r[:, k] for k in (0, 1, 2, 4, 5)]
    assert max(abs(gram(printed, h)) for h in others) > 1e-2
    assert abs(gram(printed, lat.h3r[:, 0])) > 1e-2            # couples with H_1 = H_xxy + H_yzz
    corrected = xxy - yzz
    assert np.allclose(corrected, lat.h3r[:, 3], rtol=0, atol=0)
    assert max(abs(gram(corrected, h)) for h in others) < 1e-16
    # the printed entry breaks the moment identity of the projected equilibrium
    rho, u, th = 1.1, np.array([0.12, -0.07, 0.05]), 0.9
    uuu = rho * u[:, None, None] * u[None, :, None] * u[None, None, :]
    a_printed = uuu[0, 0, 1] - uuu[1, 1, 2]
    basis = [lat.h3r[:, 0], lat.h3r[:, 1], lat.h3r[:, 2], printed, lat.h3r[:, 4], lat.h3r[:, 5]]
    coeffs = lat.tensor3_to_3r(uuu)
    coeffs[3] = a_printed
    h3 = sum(b * (a / gram(b, b)) for b, a in zip(basis, coeffs))
    assert abs(float((lat.w * h3 * printed).sum()) - a_printed) > 1e-5
