"""Pins of the learned-warm-start oracle (network, gradients, optimiser, features).

Each pin compares the oracle with something independent of it: a library
correlation routine, finite differences, the adjoint identity, torch's own
BF16 conversion, closed-form Adam steps, or analytic derivatives.
"""
import math

import numpy as np
import pytest

from oracle import Grid, Solver
from oracle import warmstart as ws


def _rand_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(ws.PARAM_COUNT) * scale


def test_param_count():
    assert ws.PARAM_COUNT == 32 * 9 * 8 + 32 + 32 * 9 * 32 + 32 + 32 * 32 + 32 + 2 * 32 + 2


def test_conv3x3_matches_scipy_wrap_correlation():
    from scipy.ndimage import correlate
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 8, 12, 3))
    W = rng.standard_normal((4, 9, 3))
    b = rng.standard_normal(4)
    z = ws.conv3x3(a, W, b)
    for bb in range(2):
        for o in range(4):
            ref = np.full((8, 12), b[o])
            for c in range(3):
                ref += correlate(a[bb, :, :, c], W[o, :, c].reshape(3, 3), mode="wrap")
            assert np.abs(z[bb, :, :, o] - ref).max() < 1e-12


def test_conv3x3_input_gradient_is_adjoint():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((1, 6, 10, 5))
    g = rng.standard_normal((1, 6, 10, 7))
    W = rng.standard_normal((7, 9, 5))
    lhs = np.sum(g * ws.conv3x3(a, W, np.zeros(7)))
    rhs = np.sum(ws.conv3x3_grad_input(g, W) * a)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    # weight gradient: d/dW of <g, conv(a, W)> is linear in W with that coefficient
    dW = ws.conv3x3_grad_weight(g, a)
    assert abs(np.sum(dW * W) - lhs) < 1e-11 * abs(lhs)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 8, 8)) * 0.7
    t = rng.standard_normal((2, 8, 8, 2)) * 0.2
    theta = _rand_theta(4)
    _, g = ws.loss_and_grad(theta, x, t, bf16_weights=False)
    # a sample of parameters from every tensor
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in ws.SHAPES])
    idx = []
    for i in range(len(ws.SHAPES)):
        idx += list(rng.integers(offs[i], offs[i + 1], size=min(6, offs[i + 1] - offs[i])))
    h = 1e-4

    def L(i, d):
        tp = theta.copy()
        tp[i] += d
        return ws.loss_and_grad(tp, x, t, bf16_weights=False)[0]

    for i in idx:
        # fourth-order central difference
        fd = (-L(i, 2 * h) + 8 * L(i, h) - 8 * L(i, -h) + L(i, -2 * h)) / (12 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, 65504.0]])
    ref = torch.tensor(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ws.bf16(v), ref)
    assert ws.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie to even (down)
    assert ws.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6   # tie to even (up)


def test_adam_first_step_and_convergence():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = ws.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # minimise 0.5 * a (x - 3)^2
    a = np.array([1.0, 10.0])
    x = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    for s in range(1, 3001):
        x, m, v = ws.adam_step(x, m, v, a * (x - 3.0), s, lr=0.05)
    assert np.abs(x - 3.0).max() < 1e-3


def test_untrained_network_gives_linear_seed():
    g = Grid(32, 16, 8 * np.pi, 4 * np.pi)
    X, Y = np.meshgrid(np.arange(32), np.arange(16))
    depth = 1.0 - 0.2 * np.exp(-((X - 10) ** 2 + (Y - 8) ** 2) / 20.0)
    s = Solver(g, depth, h_ref=1.0)
    rng = np.random.default_rng(6)
    eta = 0.05 * np.cos(2 * np.pi * (3 * X / 32 + Y / 16) + 0.3)
    phi = 0.2 * np.sin(2 * np.pi * (2 * X / 32 - Y / 16) + 0.1)
    theta = ws.init_params(0)
    V0, dB = ws.seed(theta, np.ones(8), (1.0, 1.0), s, eta, phi)
    _, wlin = ws.features(s, eta, phi)
    assert np.abs(V0 - wlin).max() == 0.0 and np.abs(dB).max() == 0.0
    assert rng is not None


def test_labels_seed_the_fixed_point():
    # seeding both unknowns with the labels of a state reaches the fixed point
    # in one sweep; either label alone does not
    g = Grid(32, 16, 8 * np.pi, 4 * np.pi)
    X, Y = np.meshgrid(np.arange(32), np.arange(16))
    depth = 1.0 - 0.3 * np.exp(-((X - 10) ** 2 + (Y - 8) ** 2) / 20.0)
    s = Solver(g, depth, h_ref=1.0, mode="iter", max_sweeps=200)
    eta = 0.06 * np.cos(2 * np.pi * (3 * X / 32 + Y / 16) + 0.3)
    phi = 0.3 * np.sin(2 * np.pi * (2 * X / 32 - Y / 16) + 0.1)
    dV, dB, info = ws.labels(s, eta, phi, tol=1e-13)
    assert info.status == 0 and info.sweeps > 8
    _, wlin = ws.features(s, eta, phi)
    _, both = s.vertical_velocity(eta, phi, tol=1e-10, seed=wlin + dV, seed_b=dB)
    _, vonly = s.vertical_velocity(eta, phi, tol=1e-10, seed=wlin + dV)
    _, lin = s.vertical_velocity(eta, phi, tol=1e-10)
    assert both.sweeps == 1
    assert vonly.sweeps > 3 and lin.sweeps > 3


def test_features_single_mode_closed_form():
    g = Grid(32, 16, 8 * np.pi, 4 * np.pi)
    x = np.arange(32) * g.lx / 32
    y = np.arange(16) * g.ly / 16
    X, Y = np.meshgrid(x, y)
    kx, ky = 2 * np.pi * 3 / g.lx, 2 * np.pi * 2 / g.ly
    k = math.hypot(kx, ky)
    h = 1.3
    s = Solver(g, np.full((16, 32), h))
    eta = 0.1 * np.cos(kx * X + ky * Y + 0.2)
    phi = 0.4 * np.sin(kx * X - ky * Y + 0.7)
    f, wlin = ws.features(s, eta, phi)
    assert np.abs(f[..., 0] - eta).max() < 1e-15
    assert np.abs(wlin - k * math.tanh(k * h) * phi).max() < 1e-13
    assert np.abs(f[..., 2] + 0.1 * kx * np.sin(kx * X + ky * Y + 0.2)).max() < 1e-13
    assert np.abs(f[..., 3] + 0.1 * ky * np.sin(kx * X + ky * Y + 0.2)).max() < 1e-13
    assert np.abs(f[..., 4] - 0.4 * kx * np.cos(kx * X - ky * Y + 0.7)).max() < 1e-13
    assert np.abs(f[..., 5] + 0.4 * ky * np.cos(kx * X - ky * Y + 0.7)).max() < 1e-13
    assert np.abs(f[..., 6]).max() == 0.0
    assert np.abs(f[..., 7] - eta * wlin).max() < 1e-15


def test_training_reduces_loss_on_a_smooth_target():
    # the network can fit a local nonlinear map of its inputs (a sanity pin of
    # forward + backward + Adam working together)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 8, 8, 8))
    t = np.stack([0.3 * np.tanh(x[..., 0] * x[..., 1]) + 0.2 * x[..., 2], 0.2 * x[..., 6] * x[..., 3]], axis=-1)
    theta = ws.init_params(1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0, _ = ws.loss_and_grad(theta, x, t)
    for s in range(1, 301):
        l, g = ws.loss_and_grad(theta, x, t)
        theta, m, v = ws.adam_step(theta, m, v, g, s, lr=3e-3)
    assert l < 0.1 * l0


def test_net_seed_is_used_only_without_history():
    """seed 'net': the network starts the first solve; later solves start from
    the previous-solve seed (same sweeps as seed 'prev' from then on)."""
    g = Grid(32, 16, 8 * np.pi, 4 * np.pi)
    X, Y = np.meshgrid(np.arange(32), np.arange(16))
    depth = 1.0 - 0.3 * np.exp(-((X - 10) ** 2 + (Y - 8) ** 2) / 20.0)
    eta = 0.06 * np.cos(2 * np.pi * (3 * X / 32 + Y / 16) + 0.3)
    phi = 0.3 * np.sin(2 * np.pi * (2 * X / 32 - Y / 16) + 0.1)
    theta = ws.init_params(2)
    p = ws.unpack(theta.copy())
    p["W4"] = np.random.default_rng(3).standard_normal((2, 32)) * 0.05
    theta = ws.pack(p)
    net = (theta, np.ones(8), (0.01, 0.01))
    en, pn, sn_info = Solver(g, depth, h_ref=1.0, mode="iter", seed="net", net=net, max_sweeps=200).step(
        eta, phi, 0.1, 2, tol=1e-10)
    ep, pp, sp_info = Solver(g, depth, h_ref=1.0, mode="iter", seed="prev", max_sweeps=200).step(
        eta, phi, 0.1, 2, tol=1e-10)
    assert all(i.status == 0 and not i.fallback for i in sn_info)
    assert sn_info[0].history[0] != sp_info[0].history[0]   # the first solve: net vs linear seed
    assert np.abs(en - ep).max() < 1e-8 * np.abs(ep).max()
