"""Pins of the oracle's time step (integrating-factor RK4 on Eq. prognostic)."""
import math

import numpy as np
import pytest

from oracle import Grid, Solver
import sbi_inputs as si


def test_linear_problem_is_exact_for_any_dt():
    # tiny amplitude: nonlinear terms ~1e-16 relative, so E(t) propagation must be exact
    g = Grid(64, 1, 4 * np.pi)
    h = 0.8
    x = np.arange(64) * g.lx / 64
    a = 1e-9
    m = 3
    k = 2 * np.pi * m / g.lx
    om = math.sqrt(k * math.tanh(k * h))
    eta = a * np.cos(k * x)[None, :]
    phi = (a / om) * np.sin(k * x)[None, :]
    s = Solver(g, np.full((1, 64), h), mode="sa")
    dt = 0.7  # large step
    e, p, _ = s.step(eta, phi, dt, 5)
    t = 5 * dt
    assert np.abs(e - a * np.cos(k * x - om * t)).max() < 1e-15
    assert np.abs(p - (a / om) * np.sin(k * x - om * t)).max() < 1e-15


def test_self_convergence_order_four():
    cfg = si.config_c1()
    gs = cfg["grid"]
    g = Grid(gs.nx, 1, gs.lx)
    s = Solver(g, cfg["depth"], h_ref=cfg["h_ref"], mode="sa")
    Tp = cfg["period"]
    res = {}
    for n in (8, 16, 32):
        res[n], _, _ = s.step(cfg["eta"], cfg["phi"], Tp / n, n)
    d1 = np.abs(res[8] - res[16]).max()
    d2 = np.abs(res[16] - res[32]).max()
    order = math.log(d1 / d2) / math.log(2)
    assert order > 3.8, order


def test_mass_conserved_and_energy_drift_small():
    # mass is exact; the energy drift is set by truncation/dealiasing, not dt,
    # and shrinks with steepness (the paper reports ~1e-5, Sec. 3.1)
    gs = si.GridSpec(32, 16, 4 * np.pi, 4 * np.pi)
    g = Grid(32, 16, gs.lx, gs.ly)
    Tp = 2 * np.pi / math.sqrt(math.tanh(3.0))
    drifts = []
    for hs in (0.05, 0.02):
        eta, phi = si.jonswap_crossing_sea(gs, 3.0, seed=1, hs_half=hs)
        eta = eta + 0.01  # non-zero mean
        s = Solver(g, np.full((16, 32), 3.0), mode="sa")
        m0, E0 = s.diagnostics(eta, phi)
        e, p, _ = s.step(eta, phi, Tp / 32, 32)
        m1, E1 = s.diagnostics(e, p)
        assert abs(m1 - m0) < 1e-13 * max(1.0, abs(m0))
        drifts.append(abs(E1 - E0) / E0)
    assert drifts[0] < 2e-4 and drifts[1] < 2e-5 and drifts[1] < drifts[0] / 4, drifts


def test_stokes_wave_translates():
    gs = si.GridSpec(64, 1, 2 * np.pi)
    a = 0.05
    eta, phi, om, c = si.stokes3_deep(gs, a)
    g = Grid(64, 1, 2 * np.pi)
    s = Solver(g, np.full((1, 64), 40.0), mode="sa")
    T = 2 * np.pi / om
    e, p, _ = s.step(eta, phi, T / 32, 32)
    # after one period the steady wave is back where it started, shape error O(eps^4)
    assert np.abs(e - eta).max() < 4 * a ** 4
    # the diagnostic itself: V = eta_t = -c eta_x for a steady wave, to the
    # accuracy of the third-order input (mismatch O(a^3), ratio 8 per doubling)
    errs = []
    for aa in (0.025, 0.05):
        eta, phi, om, c = si.stokes3_deep(gs, aa)
        W, _ = s.vertical_velocity(eta, phi)
        ex = g.ifft(1j * g.kx * g.fft(eta))
        errs.append(np.abs(W + c * ex).max())
    assert errs[1] < 0.05 ** 3 and 6.0 < errs[1] / errs[0] < 10.0, errs


def test_filter_is_identity_inside_band():
    g = Grid(64, 1, 2 * np.pi * 8)
    s = Solver(g, np.full((1, 64), 1.0), mode="sa", filter_beta=(8.0, 30.0))
    s2 = Solver(g, np.full((1, 64), 1.0), mode="sa")
    eta, phi, _ = si.stokes2_finite_depth(si.GridSpec(64, 1, g.lx), 0.05, 1.0)
    e1, _, _ = s.step(eta, phi, 0.1, 3)
    e2, _, _ = s2.step(eta, phi, 0.1, 3)
    assert np.abs(e1 - e2).max() < 1e-14
