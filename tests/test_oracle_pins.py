"""Pins of the FP64 oracle against things the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares it with a
brute-force DFT, a closed form, an exact potential-flow solution, an invariant,
or an independent second coding.
"""
import math

import numpy as np
import pytest

from oracle import Grid, Solver, w_sa_appc
from oracle import sbi_oracle as so
from oracle.dft import dft2, idft2
import sbi_inputs as si


def _rand_band(g, seed, nmodes=12, amp=0.3):
    rng = np.random.default_rng(seed)
    x = np.arange(g.nx) * g.lx / g.nx
    y = np.arange(g.ny) * g.ly / g.ny if g.ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(x, y)
    f = np.zeros((g.ny, g.nx))
    for _ in range(nmodes):
        mx = int(rng.integers(-g.Mx, g.Mx + 1))
        my = int(rng.integers(-g.My, g.My + 1)) if g.ny > 1 else 0
        a = amp * rng.standard_normal() / (1 + abs(mx) + abs(my))
        f += a * np.cos(2 * np.pi * (mx * X / g.lx + my * Y / g.ly) + rng.uniform(0, 2 * np.pi))
    return f


# ---------------------------------------------------------------------------
# FFT primitive vs brute-force DFT (Sec. 2.2 transform convention)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(1, 16), (1, 64), (8, 16), (16, 32), (32, 8)])
def test_fft_matches_bruteforce_dft(shape):
    ny, nx = shape
    g = Grid(nx, ny, 2 * np.pi, 3.0)
    f = np.random.default_rng(nx * 31 + ny).standard_normal(shape)
    F = dft2(f)
    assert np.abs(g.fft(f) - F[:, : nx // 2 + 1]).max() < 1e-13 * nx * ny
    # inverse of a Hermitian spectrum
    assert np.abs(g.ifft(g.fft(f)) - f).max() < 1e-14 * nx * ny
    assert np.abs(idft2(F).real - f).max() < 1e-13


def test_fft_sign_convention():
    # F{cos(k x)} puts +N/2 at +k with the exp(-i k x) kernel; F{sin(kx)} -> -i N/2
    g = Grid(32, 1, 2 * np.pi)
    x = np.arange(32) * 2 * np.pi / 32
    F = g.fft(np.sin(3 * x)[None, :])
    assert abs(F[0, 3] - (-16j)) < 1e-12


def test_mask_half_nyquist():
    # Sec. 4: 64 points per wavelength keep "the first 16 Fourier modes" (0..15);
    # Sec. 3.2: 1024 points over 64 m keep waves longer than 0.25 m, i.e. |m| < 256
    g = Grid(64, 32, 1.0, 1.0)
    assert g.Mx == 15 and g.My == 7
    assert g.mask[0, 15] == 1 and g.mask[0, 16] == 0
    assert g.mask[7, 0] == 1 and g.mask[8, 0] == 0 and g.mask[-7, 0] == 1 and g.mask[-8, 0] == 0
    assert Grid(1024, 1, 64.0).Mx == 255


# ---------------------------------------------------------------------------
# Linear flat-bottom limit, Sec. 2.4 initiation: F{V1} = k tanh(kh) F{phi}
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["sa", "iter"])
@pytest.mark.parametrize("ny", [1, 16])
def test_linear_flat_limit(mode, ny):
    nx = 64
    g = Grid(nx, ny, 4 * np.pi, 2 * np.pi)
    h = 1.3
    x = np.arange(nx) * g.lx / nx
    y = np.arange(ny) * g.ly / ny if ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(x, y)
    mx, my = 3, (2 if ny > 1 else 0)
    kx, ky = 2 * np.pi * mx / g.lx, 2 * np.pi * my / g.ly
    k = math.hypot(kx, ky)
    phi = np.cos(kx * X + ky * Y + 0.4)
    s = Solver(g, np.full((ny, nx), h), mode=mode)
    W, info = s.vertical_velocity(np.zeros((ny, nx)), phi, tol=1e-14)
    assert np.abs(W - k * math.tanh(k * h) * phi).max() < 1e-13
    if mode == "iter":
        assert info.sweeps == 1 and info.residual == 0.0


# ---------------------------------------------------------------------------
# Deep water: the recursion of Sec. 4 (T = 1, S = 0) coded independently
# ---------------------------------------------------------------------------
def test_deep_water_recursion():
    g = Grid(64, 1, 2 * np.pi)
    eta = _rand_band(g, 1, amp=0.08)
    phi = _rand_band(g, 2, amp=0.5)
    s = Solver(g, np.full((1, 64), 60.0), mode="sa")   # k_min h = 60 -> tanh = 1, sech ~ 1e-26
    W, _ = s.vertical_velocity(eta, phi)
    # independent coding of the deep-water reduction
    k = np.abs(np.fft.rfftfreq(64, 1 / 64))[None, :]
    M = (np.arange(33) < 16)[None, :].astype(float)   # modes 0..15 of 64 points (Sec. 4)
    F = lambda f: M * np.fft.rfft(f, axis=1)
    Fi = lambda X: np.fft.irfft(X, 64, axis=1)
    ph = F(phi)
    phx = Fi(1j * k * ph)
    V = {1: k * ph}
    for l in range(2, 8):
        acc = 0
        for j in range(1, l):
            acc = acc - k ** j / math.factorial(j) * F(eta ** j * Fi(V[l - j]))
        acc = acc - k ** (l - 2) / math.factorial(l - 1) * (1j * k) * F(eta ** (l - 1) * phx)
        V[l] = acc
    Wd = Fi(sum(V.values()))
    assert np.abs(W - Wd).max() < 1e-13 * np.abs(Wd).max()


# ---------------------------------------------------------------------------
# Constant delta, eta = 0: the exact solution is the flat bottom at depth h - delta
# ---------------------------------------------------------------------------
def _tanh_taylor_multiplier(K, h, dl, order=6):
    """k * sum_{m<=order} (-k dl)^m/m! tanh^(m)(kh): Taylor of k tanh(k(h-dl))."""
    T = np.tanh(K * h)
    P = [np.array([0.0, 1.0])]
    for _ in range(order):
        p = P[-1]
        P.append(np.polynomial.polynomial.polymul(np.polynomial.polynomial.polyder(p), [1, 0, -1]))
    mult = sum(((-K * dl) ** m / math.factorial(m)) * np.polynomial.polynomial.polyval(T, P[m])
               for m in range(order + 1))
    return K * mult


@pytest.mark.parametrize("dl", [0.1, 0.3])
def test_constant_delta_sa_is_taylor_of_shifted_depth(dl):
    g = Grid(64, 1, 4 * np.pi)
    h = 1.0
    phi = _rand_band(g, 3)
    s = Solver(g, np.full((1, 64), h - dl), h_ref=h, mode="sa")
    W, _ = s.vertical_velocity(np.zeros((1, 64)), phi)
    ph = g.MF(phi)
    Wt = g.ifft(_tanh_taylor_multiplier(g.k, h, dl) * ph)
    assert np.abs(W - Wt).max() < 1e-13 * np.abs(Wt).max()
    # and it approximates the exact shifted-depth operator to O((k dl)^7)
    We = g.ifft(g.k * np.tanh(g.k * (h - dl)) * ph)
    assert np.abs(W - We).max() < 5 * (g.kband * dl) ** 7 / 5040 * np.abs(phi).max() * g.kband + 1e-12


def test_constant_delta_iter_fixed_point_closed_form():
    g = Grid(64, 1, 4 * np.pi)
    h, dl = 1.0, 0.2
    phi = _rand_band(g, 4)
    s = Solver(g, np.full((1, 64), h - dl), h_ref=h, mode="iter", max_sweeps=200)
    W, info = s.vertical_velocity(np.zeros((1, 64)), phi, tol=1e-13)
    assert info.status == 0
    K = g.k
    T = np.tanh(K * h)
    S = 1 / np.cosh(K * h)
    x = K * dl
    sinh6 = x + x ** 3 / 6 + x ** 5 / 120
    C6 = sum(((-x) ** j) * (T if j % 2 else 1.0) / math.factorial(j) for j in range(7))
    Wc = g.ifft(K * (T - S * S * sinh6 / C6) * g.MF(phi))
    assert np.abs(W - Wc).max() < 1e-11 * np.abs(Wc).max()


# ---------------------------------------------------------------------------
# Exact flat-bottom potential flow (manufactured), nonlinear eta:
# truncation error of the 7-order expansion is O(eta^7) for O(1) phi
# ---------------------------------------------------------------------------
def _manufactured(g, h, eps):
    L = g.lx
    x = np.arange(g.nx) * L / g.nx
    modes = [(1, 1.0, 0.3), (2, 0.4, 1.1), (3, 0.15, 2.0)]
    eta = eps * (np.cos(2 * np.pi * x / L + 0.2) + 0.5 * np.sin(4 * np.pi * x / L))
    etax = eps * (-np.sin(2 * np.pi * x / L + 0.2) * 2 * np.pi / L + 0.5 * np.cos(4 * np.pi * x / L) * 4 * np.pi / L)
    phi = np.zeros(g.nx)
    phz = np.zeros(g.nx)
    phx = np.zeros(g.nx)
    for m, a, th in modes:
        k = 2 * np.pi * m / L
        c = np.cosh(k * (eta + h)) / np.cosh(k * h)
        s_ = np.sinh(k * (eta + h)) / np.cosh(k * h)
        phi += a * c * np.cos(k * x + th)
        phz += a * k * s_ * np.cos(k * x + th)
        phx += -a * k * c * np.sin(k * x + th)
    return eta[None, :], phi[None, :], (phz - etax * phx)[None, :]


@pytest.mark.parametrize("mode", ["sa", "iter"])
def test_manufactured_flat_truncation_order(mode):
    g = Grid(128, 1, 4 * np.pi)
    h = 1.5
    errs = []
    for eps in (0.025, 0.05, 0.1):
        eta, phi, Vex = _manufactured(g, h, eps)
        s = Solver(g, np.full((1, 128), h), mode=mode, max_sweeps=400)
        W, info = s.vertical_velocity(eta, phi, tol=1e-15)
        errs.append(np.abs(W - Vex).max())
    slopes = [math.log(errs[i + 1] / errs[i]) / math.log(2) for i in range(2)]
    assert all(6.7 < sl < 7.8 for sl in slopes), (errs, slopes)


def test_order_truncation_is_monotone():
    # lower orders L converge like eta^L
    g = Grid(128, 1, 4 * np.pi)
    h = 1.5
    for L in (2, 3, 4):
        errs = []
        for eps in (0.025, 0.05):
            eta, phi, Vex = _manufactured(g, h, eps)
            s = Solver(g, np.full((1, 128), h), mode="sa", order=L)
            W, _ = s.vertical_velocity(eta, phi)
            errs.append(np.abs(W - Vex).max())
        sl = math.log(errs[1] / errs[0]) / math.log(2)
        assert abs(sl - L) < 0.35, (L, sl)


# ---------------------------------------------------------------------------
# Two independent codings of the successive approximation agree (variable depth)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ny", [1, 16])
def test_general_recursion_equals_appendix_c(ny):
    g = Grid(32, ny, 4 * np.pi, 2 * np.pi)
    eta = _rand_band(g, 7, amp=0.1)
    phi = _rand_band(g, 8, amp=0.6)
    x = np.arange(32) * g.lx / 32
    y = np.arange(ny) * g.ly / ny if ny > 1 else np.zeros(1)
    X, Y = np.meshgrid(x, y)
    depth = 1.0 - 0.25 * np.exp(-((X - 6) ** 2 + (Y - 3) ** 2) / 4)
    s = Solver(g, depth, h_ref=1.0, mode="sa")
    W1, _ = s.vertical_velocity(eta, phi)
    W2 = w_sa_appc(s, eta, phi)
    assert np.abs(W1 - W2).max() < 1e-13 * np.abs(W1).max()
    for L in (2, 3, 5):
        s.L = L
        assert np.abs(s.vertical_velocity(eta, phi)[0] - w_sa_appc(s, eta, phi, L)).max() < 1e-13


def test_iteration_reaches_sa_to_truncation_order():
    g = Grid(64, 1, 4 * np.pi)
    h = 1.0
    diffs = []
    for eps in (0.02, 0.04):
        eta = eps * np.cos(2 * np.pi * np.arange(64) / 64 * 2)[None, :]
        phi = _rand_band(g, 9, nmodes=4)
        s_sa = Solver(g, np.full((1, 64), h), mode="sa")
        s_it = Solver(g, np.full((1, 64), h), mode="iter", max_sweeps=200)
        W1, _ = s_sa.vertical_velocity(eta, phi)
        W2, info = s_it.vertical_velocity(eta, phi, tol=1e-15)
        diffs.append(np.abs(W1 - W2).max())
    sl = math.log(diffs[1] / diffs[0]) / math.log(2)
    assert sl > 6.5, (diffs, sl)


# ---------------------------------------------------------------------------
# Symmetry: a 2D field constant in y reproduces the 1D result; x<->y swap
# ---------------------------------------------------------------------------
def test_2d_constant_in_y_equals_1d():
    g1 = Grid(32, 1, 4 * np.pi)
    g2 = Grid(32, 8, 4 * np.pi, 3.0)
    eta = _rand_band(g1, 11, amp=0.08)
    phi = _rand_band(g1, 12)
    depth = 1.0 - 0.2 * np.exp(-((np.arange(32) - 16) / 5.0) ** 2)[None, :]
    W1, _ = Solver(g1, depth, h_ref=1.0, mode="sa").vertical_velocity(eta, phi)
    W2, _ = Solver(g2, np.repeat(depth, 8, 0), h_ref=1.0, mode="sa").vertical_velocity(
        np.repeat(eta, 8, 0), np.repeat(phi, 8, 0))
    assert np.abs(W2 - W1).max() < 1e-13


def test_xy_swap():
    g = Grid(16, 16, 2 * np.pi, 2 * np.pi)
    eta = _rand_band(g, 13, amp=0.08)
    phi = _rand_band(g, 14)
    X, Y = np.meshgrid(np.arange(16), np.arange(16))
    depth = 1.0 - 0.2 * np.exp(-((X - 5) ** 2 + (Y - 9) ** 2) / 6.0)
    s = Solver(g, depth, h_ref=1.0, mode="sa")
    W, _ = s.vertical_velocity(eta, phi)
    Wt, _ = Solver(g, depth.T, h_ref=1.0, mode="sa").vertical_velocity(eta.T, phi.T)
    assert np.abs(W.T - Wt).max() < 1e-13


# ---------------------------------------------------------------------------
# Status logic
# ---------------------------------------------------------------------------
def test_status_codes():
    g = Grid(32, 1, 4 * np.pi)
    eta = _rand_band(g, 15, amp=0.1)
    phi = _rand_band(g, 16)
    s = Solver(g, np.full((1, 32), 1.0), mode="iter", max_sweeps=1)
    _, info = s.vertical_velocity(eta, phi, tol=1e-12)
    assert info.status == so.WARN_NOT_CONVERGED and info.sweeps == 1
    eta2 = eta.copy()
    eta2[0, 3] = np.nan
    s = Solver(g, np.full((1, 32), 1.0), mode="iter")
    _, info = s.vertical_velocity(eta2, phi, tol=1e-12)
    assert info.status == so.ERR_NONFINITE
    # relaxation factor: 1 for eta = 0, < 1 for a steep crest
    assert s.relax_factor(np.zeros((1, 32))) == 1.0
    assert s.relax_factor(eta * 5) < 1.0


# ---------------------------------------------------------------------------
# Previous-solve seed: the same fixed point, reached in fewer sweeps
# ---------------------------------------------------------------------------
def _vd_case(seed=21):
    g = Grid(32, 16, 4 * np.pi, 2 * np.pi)
    X, Y = np.meshgrid(np.arange(32), np.arange(16))
    depth = 1.0 - 0.25 * np.exp(-((X - 12) ** 2 / 30.0 + (Y - 7) ** 2 / 12.0))
    return g, _rand_band(g, seed, amp=0.06), _rand_band(g, seed + 1, amp=0.3), depth


def test_prev_seed_repeat_solve_is_one_sweep():
    g, eta, phi, depth = _vd_case()
    s = Solver(g, depth, h_ref=1.0, mode="iter", seed="prev")
    W1, i1 = s.vertical_velocity(eta, phi, tol=1e-11)
    assert i1.status == 0 and i1.sweeps > 5
    # seeded with the converged (V, phi_b) of the same state, one sweep meets tol
    W2, i2 = s.vertical_velocity(eta, phi, tol=1e-11)
    assert i2.status == 0 and i2.sweeps == 1
    assert np.abs(W2 - W1).max() < 1e-10 * np.abs(W1).max()
    # the linear-seed solver is unaffected by history
    s0 = Solver(g, depth, h_ref=1.0, mode="iter")
    s0.vertical_velocity(eta, phi, tol=1e-11)
    _, i3 = s0.vertical_velocity(eta, phi, tol=1e-11)
    assert i3.sweeps == i1.sweeps


def test_prev_seed_steps_match_linear_seed_with_fewer_sweeps():
    g, eta, phi, depth = _vd_case(23)
    sl = Solver(g, depth, h_ref=1.0, mode="iter")
    sp = Solver(g, depth, h_ref=1.0, mode="iter", seed="prev")
    el, pl, stl = sl.step(eta, phi, 0.1, 3, tol=1e-12)
    ep, pp, stp = sp.step(eta, phi, 0.1, 3, tol=1e-12)
    assert all(s.status == 0 for s in stl + stp)
    assert np.abs(ep - el).max() < 1e-10 * np.abs(el).max()
    assert np.abs(pp - pl).max() < 1e-10 * np.abs(pl).max()
    nl = sum(s.sweeps for s in stl)
    npv = sum(s.sweeps for s in stp)
    assert stp[0].sweeps == stl[0].sweeps      # first solve has no history
    assert npv < 0.9 * nl
    # the third stage sits at the same time level as the second: its seed is
    # closest there, and every step saves sweeps on it
    for k in range(3):
        assert stp[4 * k + 2].sweeps < stl[4 * k + 2].sweeps - 3
