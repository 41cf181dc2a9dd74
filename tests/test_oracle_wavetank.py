"""Pins of the oracle's numerical wave tank (Sec. 3.2): the pneumatic
wavemaker p_g and the damping pressure p_d of Eq. (pd), entering the dynamic
surface condition as a surface pressure."""
import math

import numpy as np
import pytest

from oracle import Grid, Solver
import sbi_inputs as si


def _tank_solver(nx, ny, lx, ly, h=1.0, **wm):
    g = Grid(nx, ny, lx, ly)
    return g, Solver(g, np.full((ny, nx), h), mode="sa", wavemaker=dict(comps=[], x0=0.0, **wm))


def test_damping_pressure_closed_form_1d():
    # in 1D p_d is the zero-mean antiderivative of mu phi_x; with phi = sin(kx) and
    # mu = 1 + eps cos(qx) that is sin(kx) + (eps k/2)(sin((k+q)x)/(k+q) + sin((k-q)x)/(k-q))
    L = 8 * math.pi
    g, s = _tank_solver(64, 1, L, 1.0)
    x = np.arange(64) * L / 64
    k, q, eps = 2 * math.pi * 3 / L, 2 * math.pi * 2 / L, 0.4
    mu = (1 + eps * np.cos(q * x))[None]
    pd = g.ifft(s.damping_pressure_hat(g.MF(np.sin(k * x)[None]), mu))[0]
    exact = np.sin(k * x) + 0.5 * eps * k * (np.sin((k + q) * x) / (k + q) + np.sin((k - q) * x) / (k - q))
    assert np.abs(pd - exact).max() < 1e-13


def test_damping_pressure_closed_form_2d():
    # p_d = Laplacian^-1 div(mu grad phi); phi = sin(ky y), mu = 1 + eps cos(qx):
    # p_d = sin(ky y) + eps ky^2/(q^2 + ky^2) cos(qx) sin(ky y)
    L, Ly = 8 * math.pi, 4 * math.pi
    g, s = _tank_solver(64, 32, L, Ly)
    X, Y = np.meshgrid(np.arange(64) * L / 64, np.arange(32) * Ly / 32)
    ky, q, eps = 2 * math.pi * 2 / Ly, 2 * math.pi * 3 / L, 0.3
    mu = 1 + eps * np.cos(q * X)
    pd = g.ifft(s.damping_pressure_hat(g.MF(np.sin(ky * Y)), mu))
    exact = np.sin(ky * Y) + eps * ky ** 2 / (q ** 2 + ky ** 2) * np.cos(q * X) * np.sin(ky * Y)
    assert np.abs(pd - exact).max() < 1e-13


def test_uniform_weight_returns_the_potential():
    g, s = _tank_solver(64, 16, 10.0, 5.0)
    gs = si.GridSpec(64, 16, 10.0, 5.0)
    phi = si.band_limited_random(gs, 3, amp=0.5, slope=2.0)
    ph = g.MF(phi)
    pd = g.ifft(s.damping_pressure_hat(ph, np.ones((16, 64))))
    ref = g.ifft(ph)
    assert np.abs(pd - (ref - ref.mean())).max() < 1e-13


def test_damping_weight_is_periodic_and_centred():
    L = 64 * math.pi
    g, s = _tank_solver(256, 1, L, 1.0, width=2.0)
    s.wm["x0"] = 7 * L / 8
    mu = s.damping_weight()[0]
    x = np.arange(256) * L / 256
    d = (x - 7 * L / 8 + L / 2) % L - L / 2
    assert np.allclose(mu, np.exp(-(d / 2.0) ** 2), rtol=0, atol=1e-15)
    assert mu.argmax() == 224


def _wavetank_envelope(h, a=1e-4, nx=512, nlam=64, per=16):
    # linear run (order 1, tiny amplitude) from rest: generator at x = 0 (both
    # ends), damping centred at 7L/8; envelope max|eta| over the last two periods
    # after the front has crossed the region between generator and damping
    L = nlam * 2 * math.pi
    g = Grid(nx, 1, L)
    om = math.sqrt(math.tanh(h))
    s = Solver(g, np.full((1, nx), h), order=1, mode="sa", wavemaker=dict(comps=[(a, 1.0, om, 0.3)], x0=7 * L / 8))
    T = 2 * math.pi / om
    cg = 0.5 * om * (1 + 2 * h / math.sinh(2 * h))
    dt = T / per
    n = int(math.ceil(1.6 * (5 * L / 8) / cg / dt))
    eh = np.zeros((1, nx // 2 + 1), complex)
    ph = eh.copy()
    env = np.zeros(nx)
    t = 0.0
    for i in range(n + 2 * per):
        eh, ph = s.step_hat(eh, ph, dt, 0.0, None, t)
        t += dt
        if i >= n:
            env = np.maximum(env, np.abs(g.ifft(eh)[0]))
    x = np.arange(nx) * L / nx
    return env[(x > L / 8) & (x < 5 * L / 8)] / a


@pytest.mark.parametrize("h", [20.0, 1.0])
def test_wavemaker_radiates_its_target_amplitude(h):
    # linear theory of a surface pressure P exp(-(kx)^2/2) sin(omega t): the
    # far-field amplitude is omega P F(k)/(2 c_g), F the Fourier transform of the
    # bell, = P sqrt(2 pi/e)/(1 + 2kh/sinh 2kh); the generator's prefactor
    # inverts this, so waves of amplitude a_j leave it (kh = 1: the depth factor
    # is 1.55, so a missing or wrong factor fails).  The flat envelope between
    # generator and damping (<2% ripple) shows that the damping reflects little.
    env = _wavetank_envelope(h)
    assert abs(env.mean() - 1.0) < 0.005, env.mean()
    assert env.max() - env.min() < 0.02, (env.min(), env.max())
