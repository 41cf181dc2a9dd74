"""Pins of the oracle's diagnostics (Eq. energy), low-pass filter (Eq. filter),
relaxation zones (the bar-tank generator of the configuration, not the paper's)
and control paths (divergence rule, depth criterion of Sec. 5).

Each pin is fixed by something other than the oracle's own formula: closed-form
energies of states whose W is known exactly, values of the filter that its
definition fixes at special wavenumbers, the linearised equations of motion
that a relaxation target must satisfy, and the wave a linear tank radiates.
"""
import math

import numpy as np
import pytest

from oracle import Grid, Solver
from oracle import sbi_oracle as so


# ---------------------------------------------------------------------------
# Diagnostics, Eq. (energy) of Sec. 3.1: M = dA sum eta, E = dA/2 sum (V phi + eta^2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ny", [1, 16])
def test_energy_of_pure_potential_state(ny):
    # eta = 0 over a flat bed: V = k tanh(kh) phi exactly (the linear flat limit,
    # Sec. 2.4 initiation), so for phi = A cos(k.x): E = Lx Ly k tanh(kh) A^2 / 4, M = 0
    nx = 32
    lx, ly = 4 * math.pi, 2 * math.pi
    g = Grid(nx, ny, lx, ly if ny > 1 else 1.0)
    h = 0.7
    x = np.arange(nx) * lx / nx
    y = np.arange(ny) * ly / ny if ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(x, y)
    mx, my = 3, (2 if ny > 1 else 0)
    kx, ky = 2 * math.pi * mx / lx, 2 * math.pi * my / ly
    k = math.hypot(kx, ky)
    A = 0.37
    phi = A * np.cos(kx * X + ky * Y + 0.3)
    s = Solver(g, np.full((ny, nx), h), mode="iter")
    m, E = s.diagnostics(np.zeros((ny, nx)), phi, tol=1e-14)
    area = lx * (ly if ny > 1 else 1.0)
    assert abs(m) < 1e-15
    assert abs(E - area * k * math.tanh(k * h) * A * A / 4) < 1e-13 * E


@pytest.mark.parametrize("ny", [1, 16])
def test_energy_of_pure_elevation_state_over_a_variable_bed(ny):
    # phi = 0: every term of the W solve carries phi or a product with V, so
    # W = 0 exactly whatever the bed; eta = c + a cos(k.x) gives
    # M = c Lx Ly and E = Lx Ly (c^2 + a^2/2) / 2
    nx = 32
    lx, ly = 4 * math.pi, 2 * math.pi
    g = Grid(nx, ny, lx, ly if ny > 1 else 1.0)
    x = np.arange(nx) * lx / nx
    y = np.arange(ny) * ly / ny if ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(x, y)
    depth = 1.0 - 0.3 * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 3) ** 2))
    c, a = 0.013, 0.08
    eta = c + a * np.cos(2 * math.pi * 2 * X / lx + (2 * math.pi * Y / ly if ny > 1 else 0.0))
    area = lx * (ly if ny > 1 else 1.0)
    for mode in ("sa", "iter"):
        s = Solver(g, depth, mode=mode)
        m, E = s.diagnostics(eta, np.zeros((ny, nx)), tol=1e-14)
        assert abs(m - c * area) < 1e-14 * area
        assert abs(E - area * (c * c + a * a / 2) / 2) < 1e-14 * area


def test_energy_of_a_linear_progressive_wave():
    # eta = a cos(kx), phi = (a/omega) sin(kx): half potential, half kinetic,
    # E = L a^2 / 2; the first nonlinear term of <V phi> projects to zero on the
    # wave's mode, so the relative correction is O((ka)^2)
    nx = 64
    g = Grid(nx, 1, 8 * math.pi)
    h = 1.1
    x = np.arange(nx) * g.lx / nx
    k = 2 * math.pi * 5 / g.lx
    om = math.sqrt(k * math.tanh(k * h))
    for a in (1e-3, 1e-4):
        s = Solver(g, np.full((1, nx), h), mode="iter")
        m, E = s.diagnostics((a * np.cos(k * x))[None], ((a / om) * np.sin(k * x))[None], tol=1e-14)
        assert abs(m) < 1e-15
        assert abs(E / (g.lx * a * a / 2) - 1.0) < 5 * (k * a) ** 2


# ---------------------------------------------------------------------------
# Low-pass filter, Eq. (filter): Lambda = exp(-|k/beta1|^beta2), applied to the
# state after each step
# ---------------------------------------------------------------------------
def _filter_ratio(beta, modes):
    # tiny linear waves over a flat bed: the filtered step equals the unfiltered
    # step times Lambda(|k|), mode by mode, for both eta and phi
    nx = ny = 64
    lx = ly = 2 * math.pi
    g = Grid(nx, ny, lx, ly)
    x = np.arange(nx) * lx / nx
    X, Y = np.meshgrid(x, x)
    eta = np.zeros((ny, nx))
    phi = np.zeros((ny, nx))
    for i, (mx, my) in enumerate(modes):
        eta += 1e-9 * np.cos(mx * X + my * Y + 0.2 * i)
        phi += 1e-9 * np.sin(mx * X + my * Y + 0.5 * i)
    depth = np.full((ny, nx), 1.0)
    s0 = Solver(g, depth, mode="sa", order=1)
    s1 = Solver(g, depth, mode="sa", order=1, filter_beta=beta)
    e0, p0, _ = s0.step(eta, phi, 0.05, 1)
    e1, p1, _ = s1.step(eta, phi, 0.05, 1)
    out = []
    for mx, my in modes:
        iy = my % ny
        r_e = g.fft(e1)[iy, mx] / g.fft(e0)[iy, mx]
        r_p = g.fft(p1)[iy, mx] / g.fft(p0)[iy, mx]
        out.append((r_e, r_p))
    return out


@pytest.mark.parametrize("beta2", [30.0, 2.0])
def test_filter_outside_the_band(beta2):
    # |k| = beta1 is damped by 1/e for any beta2, in 2D along a diagonal
    # (k = (3, 4), |k| = 5: a filter of k_x or k_y alone would not give 1/e);
    # |k| = beta1 2^(1/beta2) by 1/e^2; the mean mode is untouched
    b1 = 5.0
    k2 = b1 * 2 ** (1 / beta2)
    modes = [(3, 4), (5, 0), (0, 5), (0, 0)]
    rs = _filter_ratio((b1, beta2), modes)
    for r_e, r_p in rs[:3]:
        assert abs(r_e - math.exp(-1)) < 1e-9 and abs(r_p - math.exp(-1)) < 1e-9, (r_e, r_p)
    # the mean of eta (phi's mean is a gauge and its projection is 0 here)
    assert abs(rs[3][0] - 1.0) < 1e-12
    # a mode at beta1 * 2^(1/beta2) along x (only exact when it is an integer:
    # build the grid check from the closed form of the ratio instead)
    if beta2 == 2.0:
        # modes (1, 7): |k|^2 = 50 = 2 beta1^2 -> exp(-2)
        (r_e, r_p), = _filter_ratio((b1, beta2), [(1, 7)])
        assert abs(r_e - math.exp(-2)) < 1e-9 and abs(r_p - math.exp(-2)) < 1e-9
    else:
        # beyond the cut-off the mode is removed: |k| = 7 gives exp(-(7/5)^30) ~ 1e-11
        (r_e, r_p), = _filter_ratio((b1, beta2), [(7, 0)])
        assert abs(r_e) < 1e-10 and abs(r_p) < 1e-10
    assert k2 > b1


# ---------------------------------------------------------------------------
# Relaxation zones (configuration C2's generator; not a device of the paper)
# ---------------------------------------------------------------------------
def _rz(a=0.02, om=None, h=1.0):
    om = om if om is not None else math.sqrt(math.tanh(h))
    lam = 2 * math.pi
    return dict(a=a, k=1.0, omega=om, gen_len=2 * lam, abs_len=3 * lam, ramp_periods=3.0)


def test_relaxation_weights_at_special_points():
    nx = 1024
    L = 16 * 2 * math.pi
    g = Grid(nx, 1, L)
    rz = _rz()
    s = Solver(g, np.full((1, nx), 1.0), mode="sa", relaxation_zone=rz)
    wg, wa = s.relaxation_weights()
    x = np.arange(nx) * L / nx
    dx = L / nx
    gen, absl = rz["gen_len"], rz["abs_len"]
    # generation zone: 1 at the end wall, 1/2 half way, 0 beyond it; a smooth
    # step: w(s) + w(1 - s) = 1 and flat at both ends
    assert wg[0, 0] == 1.0
    i_half = int(round(gen / 2 / dx))
    assert abs(x[i_half] - gen / 2) < 1e-12 and abs(wg[0, i_half] - 0.5) < 1e-14
    assert np.all(wg[0, x >= gen] == 0.0)
    inside = (x > 0) & (x < gen)
    mirror = np.interp(gen - x[inside], x, wg[0])
    assert np.abs(wg[0, inside] + mirror - 1.0).max() < 1e-3  # linear interpolation of a smooth step
    assert 1.0 - wg[0, 1] < 4 * (dx / gen) ** 2  # zero slope at the wall
    # absorption zone: 0 outside, rising to 1 towards the far wall, 1/2 half way
    assert np.all(wa[0, x <= L - absl] == 0.0)
    j_half = int(round((L - absl / 2) / dx))
    assert abs(wa[0, j_half] - 0.5) < 1e-14
    assert np.all(np.diff(wa[0, x > L - absl]) > 0)


def test_relaxation_target_is_a_linear_wave_of_the_bed():
    # after the ramp the target solves the linearised equations of motion,
    # eta_t = F^-1{k tanh(kh) phi_hat}, phi_t = -eta (Eq. prognostic without N),
    # i.e. it travels towards +x at the linear phase speed; the ramp is 0 at
    # t = 0, 1/2 half way and 1 from ramp_periods periods on
    nx = 256
    L = 8 * 2 * math.pi
    h = 1.3
    g = Grid(nx, 1, L)
    rz = _rz(h=h)
    s = Solver(g, np.full((1, nx), h), mode="sa", relaxation_zone=rz)
    T = 2 * math.pi / rz["omega"]
    t = 4.2 * T
    eps = 1e-5
    e0, p0 = s.relaxation_target(t)
    ep, pp = s.relaxation_target(t + eps)
    em, pm = s.relaxation_target(t - eps)
    eta_t = (ep - em) / (2 * eps)
    phi_t = (pp - pm) / (2 * eps)
    dn_phi = g.ifft(g.k * np.tanh(g.k * h) * g.fft(p0))
    assert np.abs(eta_t - dn_phi).max() < 1e-9 * rz["a"] * 10
    assert np.abs(phi_t + e0).max() < 1e-9 * rz["a"] * 10
    # travelling towards +x: eta(x, t + dt) = eta(x - c dt, t)
    c = rz["omega"] / rz["k"]
    x = np.arange(nx) * L / nx
    assert np.abs(s.relaxation_target(t + 0.3)[0][0] - rz["a"] * np.cos(x - c * 0.3 - rz["omega"] * t)).max() < 1e-14
    tr = rz["ramp_periods"] * T
    xs = np.arange(nx) * L / nx
    full = rz["a"] * np.cos(rz["k"] * xs)
    assert np.abs(s.relaxation_target(0.0)[0]).max() == 0.0
    assert np.abs(s.relaxation_target(tr / 2)[0][0] - 0.5 * rz["a"] * np.cos(xs - rz["omega"] * tr / 2)).max() < 1e-15
    assert np.abs(s.relaxation_target(tr)[0][0] - rz["a"] * np.cos(xs - rz["omega"] * tr)).max() < 1e-15
    assert full.shape == (nx,)


def test_relaxation_passes_its_own_target_through():
    # a state equal to the (band-limited) target is left unchanged when no grid
    # point lies in the absorption zone
    nx = 256
    L = 8 * 2 * math.pi
    g = Grid(nx, 1, L)
    rz = _rz()
    rz["abs_len"] = 0.5 * L / nx
    s = Solver(g, np.full((1, nx), 1.0), mode="sa", relaxation_zone=rz)
    t = 5.0 * 2 * math.pi / rz["omega"]
    et, pt = s.relaxation_target(t)
    eh, ph = s.apply_relaxation(g.MF(et), g.MF(pt), t)
    assert np.abs(g.ifft(eh) - et).max() < 1e-16 + 1e-14 * rz["a"]
    assert np.abs(g.ifft(ph) - pt).max() < 1e-16 + 1e-14 * rz["a"]


def test_relaxation_tank_radiates_the_target_wave():
    # a linear tank (order 1, tiny amplitude, deep bed) driven by the
    # generation zone: between the zones the wave has the target's amplitude
    # and phase a cos(kx - omega t) (a wrong sign of the potential target would
    # send it the other way or leave a standing wave)
    h, a, nx, nlam = 3.0, 1e-4, 512, 24
    lam = 2 * math.pi
    L = nlam * lam
    g = Grid(nx, 1, L)
    om = math.sqrt(math.tanh(h))
    rz = dict(a=a, k=1.0, omega=om, gen_len=2 * lam, abs_len=3 * lam, ramp_periods=3.0)
    s = Solver(g, np.full((1, nx), h), order=1, mode="sa", relaxation_zone=rz)
    T = 2 * math.pi / om
    cg = 0.5 * om * (1 + 2 * h / math.sinh(2 * h))
    per = 32
    dt = T / per
    x = np.arange(nx) * L / nx
    xe = L - 3 * lam
    n = int(math.ceil((3 * T + (xe - 2 * lam) / cg * 1.3) / dt))
    eh = np.zeros((1, nx // 2 + 1), complex)
    ph = eh.copy()
    t = 0.0
    env = np.zeros(nx)
    for i in range(n + per):
        eh, ph = s.step_hat(eh, ph, dt, 0.0, None, t)
        t += dt
        eh, ph = s.apply_relaxation(eh, ph, t)
        if i >= n:
            env = np.maximum(env, np.abs(g.ifft(eh)[0]))
    m = (x > 3 * lam) & (x < xe - lam)
    assert abs(env[m].mean() / a - 1.0) < 0.01
    assert env[m].min() / a > 0.94 and env[m].max() / a < 1.06
    e = g.ifft(eh)[0][m]
    th = x[m] - om * t
    cpart = np.sum(e * np.cos(th)) / np.sum(np.cos(th) ** 2) / a
    spart = np.sum(e * np.sin(th)) / np.sum(np.sin(th) ** 2) / a
    assert abs(cpart - 1.0) < 0.03 and abs(spart) < 0.03, (cpart, spart)


# ---------------------------------------------------------------------------
# Control paths of the iteration and the depth criterion of Sec. 5
# ---------------------------------------------------------------------------
def _steep_case():
    g = Grid(64, 1, 4 * math.pi)
    x = np.arange(64) * g.lx / 64
    eta = (0.15 * np.cos(2 * math.pi * 3 * x / g.lx) + 0.02 * np.cos(2 * math.pi * 11 * x / g.lx + 1.0))[None]
    phi = (0.5 * np.sin(2 * math.pi * 3 * x / g.lx) + 0.1 * np.sin(2 * math.pi * 7 * x / g.lx))[None]
    return g, eta, phi


def test_divergence_rule_stops_plain_sweeps_on_a_steep_crest():
    # k_band max(eta) > ln 2: plain sweeps converge on the long waves first and
    # then expand on the short ones (the local symbol of the sweep exceeds one
    # at the crest), so the residual falls and rises again; the rule stops the
    # iteration at the first residual above ten times the smallest one, after
    # the third sweep.  (Its other branch, a residual above 1e6, guards against
    # overflow; the relative residual of a real field stays near or below 2.)
    g, eta, phi = _steep_case()
    assert g.kband * eta.max() > math.log(2.0)
    s = Solver(g, np.full((1, 64), 1.0), mode="iter", max_sweeps=500, relax=False)
    _, info = s.vertical_velocity(eta, phi, tol=1e-12)
    assert info.status == so.ERR_DIVERGED
    h = info.history
    assert info.sweeps == len(h) and info.sweeps >= 4
    assert h[-1] > 10 * min(h[:-1])
    assert all(h[i] <= 10 * min(h[:i + 1]) for i in range(3, len(h) - 1))
    assert min(h) < 0.5 * h[0]  # it converged for a while first
    # the relaxed sweeps converge on the same input
    s2 = Solver(g, np.full((1, 64), 1.0), mode="iter", max_sweeps=500, relax=True)
    _, i2 = s2.vertical_velocity(eta, phi, tol=1e-12)
    assert i2.status == so.OK and i2.omega < 1.0


def test_depth_criterion_flag():
    # Sec. 5: the expansion in delta is valid while k |delta| < 2.4 at the
    # largest resolved wavenumber
    g = Grid(64, 1, 8 * math.pi)
    x = np.arange(64) * g.lx / 64
    bump = np.exp(-((x - g.lx / 2) / 2.0) ** 2)[None]
    for kd, warn in ((2.3, False), (2.5, True)):
        d = kd / g.kband
        s = Solver(g, 2.0 - d * bump, h_ref=2.0, mode="sa")
        assert s.depth_warning == warn
