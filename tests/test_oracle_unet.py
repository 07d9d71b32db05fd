"""Pins of the FP64 reference of the neural operator and of the warm-start helpers.

The paper has no network, so the reference is pinned against definitions that do not go
through its own code: loop convolution, adjointness of pooling and upsampling, central finite
differences of the loss, the closed form of one Adam step, exact bfloat16 values, the exact
distance to a circle, and the free stream.
"""
import numpy as np
import pytest

from oracle import unet as U
from oracle import warmstart as WS
from paper_2607_07432_amd import workloads as wl


def test_param_count_from_shapes():
    shapes = U.layer_shapes()
    assert len(shapes) == 2 * U.LEVELS + 2 * (U.LEVELS - 1) + 1
    assert shapes[0] == (8, 32, 9) and shapes[-1] == (32, 4, 1)
    assert shapes[2 * U.LEVELS] == (256 + 256, 256, 9)         # first decoder conv, level 3
    assert U.param_count() == sum(co * t * ci + co for ci, co, t in shapes)
    assert 4.5e6 < U.param_count() < 5.5e6


def test_conv_matches_loop_definition():
    rng = np.random.Generator(np.random.PCG64(1))
    X = rng.standard_normal((2, 4, 5, 3))
    for taps in (9, 1):
        W = rng.standard_normal((2, taps, 3))
        b = rng.standard_normal(2)
        z, _ = U.conv(X, W, b, taps, relu=False)
        assert np.allclose(z, U.conv_brute(X, W, b, taps), rtol=0, atol=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose((U.pool(x) * y).sum(), (x * U.pool_adjoint(y)).sum(), rtol=1e-13)
    assert np.isclose((U.up(y) * x).sum(), (y * U.up_adjoint(x)).sum(), rtol=1e-13)
    assert np.allclose(U.pool(U.up(y)), y)


def test_im2col_col2im_adjoint():
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((1, 5, 7, 2))
    c = rng.standard_normal((1, 5, 7, 18))
    assert np.isclose((U.im2col(x, 9) * c).sum(), (x * U.col2im(c, 9, 2)).sum(), rtol=1e-13)


@pytest.fixture(scope='module')
def tiny():
    rng = np.random.Generator(np.random.PCG64(4))
    theta = wl.init_params(U.layer_shapes(), seed=5)
    theta += 0.01 * rng.standard_normal(theta.shape)     # nonzero biases too
    x = rng.standard_normal((1, 16, 16, 4))
    tgt = rng.standard_normal((1, 16, 16, 4))
    mask = (rng.uniform(size=(1, 16, 16)) > 0.2).astype(np.float64)
    return theta, x, tgt, mask


def test_backward_matches_finite_differences(tiny):
    theta, x, tgt, mask = tiny
    out, cache = U.forward(theta, x)
    g, L = U.backward(theta, cache, out, tgt, mask)
    assert np.isclose(L, U.loss(out, tgt, mask))
    rng = np.random.Generator(np.random.PCG64(6))
    eps = 1e-6

    def Lof(th):
        o, _ = U.forward(th, x)
        return U.loss(o, tgt, mask)

    # a random direction, and single parameters in the first, a middle and the head layer
    # (unit direction: a small step crosses no ReLU kink)
    d = rng.standard_normal(theta.shape)
    d /= np.linalg.norm(d)
    fd = (Lof(theta + eps * d) - Lof(theta - eps * d)) / (2 * eps)
    assert abs(fd - g @ d) <= 1e-5 * abs(fd) + 1e-12
    picks = [0, 100, U.param_count() // 2, U.param_count() - 3, U.param_count() - 140]
    for i in picks:
        e = np.zeros_like(theta)
        e[i] = 1.0
        fdi = (Lof(theta + eps * e) - Lof(theta - eps * e)) / (2 * eps)
        assert abs(fdi - g[i]) <= 1e-5 * max(abs(fdi), 1e-8) + 1e-10, i


def test_bf16_emulated_backward_stays_within_rounding_of_exact(tiny):
    # storing activation gradients in bfloat16 perturbs each layer's gradient by a few units of
    # 2^-8 at most, and does perturb it (the rounding is applied on the way down)
    theta, x, tgt, mask = tiny
    out, cache = U.forward(theta, x, emulate_bf16=True)
    g_ex, L_ex = U.backward(theta, cache, out, tgt, mask)
    g_bf, L_bf = U.backward(theta, cache, out, tgt, mask, emulate_bf16=True)
    assert L_ex == L_bf
    off = 0
    for k, (ci, co, t) in enumerate(U.layer_shapes()):
        n = co * t * ci + co
        a, b = g_bf[off:off + n], g_ex[off:off + n]
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        if k < len(U.layer_shapes()) - 1:
            assert 0.0 < e <= 2e-2, (k, e)
        else:
            assert e == 0.0                    # the head's gradient uses no stored gradient
        off += n


def test_float32_accumulation_is_a_small_perturbation(tiny):
    # the float32-sum variant of the forward pass stays within the FP32 rounding of the exact one
    # (no bf16 storage: nothing cascades), and differs from it
    theta, x, tgt, mask = tiny
    o64, _ = U.forward(theta, x)
    o32, _ = U.forward(theta, x, accum32=True)
    e = np.linalg.norm(o32 - o64) / np.linalg.norm(o64)
    assert 0.0 < e < 1e-5


def test_adam_first_step_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    th, m, v = U.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=1e-8, wd=0.1)
    expect = theta - 0.01 * (g / (np.abs(g) + 1e-8) + 0.1 * theta)
    assert np.allclose(th, expect, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_clip_grad_norm_closed_form():
    # a 3-4-12 vector has norm 13: clipped to 6.5 it halves; below the bound it is unchanged
    g = np.array([3.0, -4.0, 12.0])
    c, n = U.clip_grad_norm(g, 6.5)
    assert n == 13.0 and np.array_equal(c, g / 2)
    c, n = U.clip_grad_norm(g, 20.0)
    assert n == 13.0 and np.array_equal(c, g)


def test_bf16_rounding_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -3.14159265, 0.0])
    r = U.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1.0 + 2 ** -7            # above the tie
    assert r[3] == 1.0 + 2 ** -6            # tie -> even (odd mantissa rounds up)
    assert r[4] == -3.140625
    assert r[5] == 0.0


def test_signed_distance_of_a_circle():
    c = wl.cylinder_case(nx=64, ny=48, center=(30.3, 24.6), diameter=16.0, markers=128)
    sdf, inside = WS.signed_distance(64, 48, c.X, c.n)
    ys, xs = np.mgrid[0:48, 0:64].astype(np.float64)
    exact = np.hypot(xs - 30.3, ys - 24.6) - 8.0
    # the markers lie on the circle: the nearest-marker distance is at least the distance to the
    # circle and exceeds it by at most half the marker spacing (triangle inequality)
    spacing = np.pi * 16.0 / 128
    assert np.all(np.abs(sdf) >= np.abs(exact) - 1e-12)
    assert np.all(np.abs(sdf) - np.abs(exact) <= spacing / 2 + 1e-12)
    far = np.abs(exact) > 1.0
    assert np.array_equal(inside[far], (exact < 0)[far])


def test_normalisation_of_free_stream_and_round_trip():
    rho_inf, u_inf, T_inf, gamma = 1.0, np.array([0.07, 0.0]), 1.0, 1.4
    rho = np.full((3, 4), rho_inf)
    u = np.zeros((2, 3, 4))
    u[0] = u_inf[0]
    T = np.full((3, 4), T_inf)
    p = WS.normalise(rho, u, T, rho_inf, u_inf, T_inf, gamma)
    assert np.allclose(p[..., 0], 0) and np.allclose(p[..., 1], 1) and np.allclose(p[..., 2], 0)
    assert np.allclose(p[..., 3], 0)
    rng = np.random.Generator(np.random.PCG64(7))
    q = rng.standard_normal((3, 4, 4))
    r2, u2, T2 = WS.denormalise(q, rho_inf, u_inf, T_inf, gamma)
    assert np.allclose(WS.normalise(r2, u2, T2, rho_inf, u_inf, T_inf, gamma), q, atol=1e-12)
    m2 = WS.mach2(u_inf, T_inf, gamma)
    assert np.isclose(m2, 0.07 ** 2 / (1.4 / 3.0))


def test_warm_state_moments_of_a_shear_flow():
    """Zero-th and first moments are the fields' (the added part has none); the deviatoric second
    moment of f - f^eq is -rho c_s^2 tau_bar S, here for u_x = g y: Pi_xy = -rho c_s^2 tau_bar g."""
    from oracle.lattice import for_dim
    from oracle import lbm as olbm
    lat = for_dim(2)
    ny, nx, g, mu = 12, 10, 1e-3, 0.05
    prm = olbm.Params(mu=mu, lam=0.1, gamma=1.4, sigma=0.98, rho_inf=1.0, u_inf=(0.05, 0.0), T_inf=1.0,
                      bc='periodic')
    rho = np.full((ny, nx), 1.02)
    T = np.full((ny, nx), 0.97)
    u = np.zeros((2, ny, nx))
    u[0] = g * np.arange(ny)[:, None]
    f = WS.warm_state(lat, prm, rho, u, T)
    feq = olbm.equilibrium(lat, rho, u, T)
    cf = lat.c.astype(np.float64)
    assert np.allclose(f.sum(0), rho, atol=1e-14)
    assert np.allclose(np.einsum('ia,i...->a...', cf, f), rho * u, atol=1e-14)
    Pi = olbm.deviatoric_second_moment(lat, f - feq)
    inner = slice(1, ny - 1)                  # away from the periodic wrap of the linear profile
    taubar = mu / (1.02 / 3.0) + 0.5
    assert np.allclose(Pi[0, 1][inner], -1.02 / 3.0 * taubar * g, rtol=1e-12, atol=0)
    assert np.allclose(Pi[0, 0][inner], 0.0, atol=1e-15) and np.allclose(Pi[1, 1][inner], 0.0, atol=1e-15)
