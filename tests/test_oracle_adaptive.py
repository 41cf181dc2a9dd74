"""Pins of the oracle's adaptive step (Sec. 2.2: a six-stage fifth-order
Runge-Kutta pair with an embedded fourth-order solution, in the
integrating-factor form of Eq. (prognostic), with step-size control)."""
import cmath
import math
from fractions import Fraction

import numpy as np

from oracle import Grid, Solver
from oracle.sbi_oracle import CK_A, CK_B4, CK_B5, CK_C, WARN_STEP_LIMIT, lawson_rk54
import sbi_inputs as si


# -- the coefficient table against the Runge-Kutta order conditions ----------
def _trees(order):
    """Rooted trees with `order` vertices, each a sorted tuple of its subtrees."""
    if order == 1:
        return [()]
    out = set()

    def forests(n, max_tree):
        # multisets of trees with n vertices in total, trees in non-increasing order
        if n == 0:
            yield ()
            return
        for m in range(n, 0, -1):
            for t in _trees(m):
                if max_tree is not None and (m, t) > max_tree:
                    continue
                for rest in forests(n - m, (m, t)):
                    yield ((m, t),) + rest

    for f in forests(order - 1, None):
        out.add(tuple(sorted(t for _, t in f)))
    return sorted(out)


def _size(t):
    return 1 + sum(_size(s) for s in t)


def _gamma(t):
    return _size(t) * math.prod(_gamma(s) for s in t)


def _phi(t, A):
    """Elementary weight vector Phi_i(t) = prod over subtrees of (A Phi(s))_i."""
    n = len(A)
    v = np.ones(n)
    for s in t:
        v = v * (A @ _phi(s, A))
    return v


def _tableau():
    A = np.zeros((6, 6))
    for i, row in enumerate(CK_A):
        A[i, :len(row)] = row
    return A, np.array(CK_B5), np.array(CK_B4), np.array(CK_C)


def test_tree_enumeration_counts():
    # number of rooted trees with 1..6 vertices (OEIS A000081)
    assert [len(_trees(n)) for n in range(1, 7)] == [1, 1, 2, 4, 9, 20]


def test_pair_satisfies_order_conditions():
    A, b5, b4, c = _tableau()
    assert np.allclose(A.sum(axis=1), c, rtol=0, atol=1e-15)          # nodes are row sums
    for order in range(1, 6):
        for t in _trees(order):
            assert abs(b5 @ _phi(t, A) - 1.0 / _gamma(t)) < 1e-15, (order, t)
            if order <= 4:
                assert abs(b4 @ _phi(t, A) - 1.0 / _gamma(t)) < 1e-15, (order, t)
    # the embedded solution is of order exactly four, the main one of order five only
    assert max(abs(b4 @ _phi(t, A) - 1.0 / _gamma(t)) for t in _trees(5)) > 1e-4
    assert max(abs(b5 @ _phi(t, A) - 1.0 / _gamma(t)) for t in _trees(6)) > 1e-5


def test_coefficients_are_the_rationals_of_the_pair():
    # every coefficient equals a rational with a small denominator (a mistyped
    # digit in a float literal would not)
    for v in list(CK_C) + [a for r in CK_A for a in r] + list(CK_B5) + list(CK_B4):
        fr = Fraction(v).limit_denominator(200000)
        assert float(fr) == v and fr.denominator <= 110592, v


# -- the Lawson form on a scalar equation with a closed-form solution --------
ALPHA, BETA, Y0 = -0.3 + 2.0j, 0.4, 0.5


def _bernoulli(t):
    # y' = alpha y + beta y^2
    e = cmath.exp(ALPHA * t)
    return ALPHA * Y0 * e / (ALPHA + BETA * Y0 * (1 - e))


def _run(n, which, T=2.0):
    h = T / n
    y = (np.array([Y0], dtype=complex),)
    f = lambda u, tau: (BETA * u[0] * u[0],)
    E = lambda u, tau: (np.exp(ALPHA * tau) * u[0],)
    for _ in range(n):
        y5, y4 = lawson_rk54(y, h, f, E)
        y = y5 if which == 5 else y4
    return abs(y[0][0] - _bernoulli(T))


def test_lawson_pair_converges_at_orders_five_and_four():
    for which, lo, hi in ((5, 4.7, 5.4), (4, 3.7, 4.4)):
        e = [_run(n, which) for n in (10, 20, 40)]
        rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(lo < r < hi for r in rates), (which, e, rates)


def test_lawson_pair_is_exact_without_nonlinear_term():
    y = (np.array([Y0], dtype=complex),)
    f = lambda u, tau: (0.0 * u[0],)
    E = lambda u, tau: (np.exp(ALPHA * tau) * u[0],)
    y5, y4 = lawson_rk54(y, 0.9, f, E)
    assert y5[0][0] == y4[0][0] == np.exp(ALPHA * 0.9) * Y0


def test_local_error_estimate_scales_as_h5():
    y = (np.array([Y0], dtype=complex),)
    f = lambda u, tau: (BETA * u[0] * u[0],)
    E = lambda u, tau: (np.exp(ALPHA * tau) * u[0],)
    d = []
    for h in (0.2, 0.1):
        y5, y4 = lawson_rk54(y, h, f, E)
        d.append(abs(y5[0][0] - y4[0][0]))
    assert 4.6 < math.log2(d[0] / d[1]) < 5.4, d


# -- the wave problem --------------------------------------------------------
def _c1_solver(**kw):
    cfg = si.config_c1()
    gs = cfg["grid"]
    g = Grid(gs.nx, 1, gs.lx)
    return cfg, g, Solver(g, cfg["depth"], h_ref=cfg["h_ref"], mode="sa", **kw)


def test_linear_energy_norm_of_a_mode():
    # eta = a cos(kx), phi = b sin(kx):  sum eta^2 + phi D phi = N (a^2 + k tanh(kh) b^2) / 2
    g = Grid(64, 1, 4 * np.pi)
    s = Solver(g, np.full((1, 64), 0.8), mode="sa")
    k = 2 * np.pi * 3 / g.lx
    x = np.arange(64) * g.lx / 64
    a, b = 0.3, 0.7
    E = s.linear_energy(g.MF(a * np.cos(k * x)[None]), g.MF(b * np.sin(k * x)[None]))
    assert abs(E - 32 * (a * a + k * math.tanh(0.8 * k) * b * b)) < 1e-12


def test_fifth_order_self_convergence_on_waves():
    cfg, g, s = _c1_solver()
    Tp = cfg["period"]
    eh0, ph0 = g.MF(cfg["eta"]), g.MF(cfg["phi"])
    res = {}
    for n in (4, 8, 16):
        eh, ph = eh0, ph0
        for _ in range(n):
            eh, ph, _ = s.step_rk54_hat(eh, ph, Tp / n, 1e-13)
        res[n] = g.ifft(eh)
    d1 = np.abs(res[4] - res[8]).max()
    d2 = np.abs(res[8] - res[16]).max()
    assert math.log2(d1 / d2) > 4.6, (d1, d2)


def test_linear_waves_take_growing_steps_and_stay_exact():
    g = Grid(64, 1, 4 * np.pi)
    h = 0.8
    x = np.arange(64) * g.lx / 64
    a, m = 1e-9, 3
    k = 2 * np.pi * m / g.lx
    om = math.sqrt(k * math.tanh(k * h))
    s = Solver(g, np.full((1, 64), h), mode="sa")
    e, p, info = s.step_adaptive(a * np.cos(k * x)[None], (a / om) * np.sin(k * x)[None], 0.0, 10.0, 0.01, 1e-6)
    hs = [r[0] for r in info["history"]]
    assert info["rejected"] == 0 and info["t"] == 10.0
    assert all(abs(hs[i + 1] / hs[i] - 5.0) < 1e-12 for i in range(len(hs) - 2))   # the largest growth each time
    assert np.abs(e - a * np.cos(k * x - om * 10.0)).max() < 1e-17


def test_adaptive_run_lands_on_t_end_and_controls_the_error():
    cfg, g, s = _c1_solver()
    Tp = cfg["period"]
    ref_e, _, _ = s.step(cfg["eta"], cfg["phi"], Tp / 256, 256, tol=1e-13)  # RK4 at 256 steps per period
    errs = []
    for rk_tol in (1e-5, 1e-8):
        e, p, info = s.step_adaptive(cfg["eta"], cfg["phi"], 0.0, Tp, Tp / 4, rk_tol, tol=1e-13)
        assert info["t"] == Tp and info["status"] == 0
        for hs, err, ok in info["history"]:
            assert ok == (err <= rk_tol)
        assert info["rejected"] >= 1          # T/4 is far too long a first step
        errs.append(np.abs(e - ref_e).max() / np.abs(ref_e).max())
    assert errs[1] < errs[0] / 30 and errs[1] < 1e-7, errs


def test_no_growth_right_after_a_rejection():
    cfg, g, s = _c1_solver()
    _, _, info = s.step_adaptive(cfg["eta"], cfg["phi"], 0.0, cfg["period"], cfg["period"], 1e-7, tol=1e-13)
    h = info["history"]
    for i in range(1, len(h) - 1):
        if not h[i - 1][2] and h[i][2]:       # accepted right after a rejection
            assert h[i + 1][0] <= h[i][0] * (1 + 1e-15) or i + 1 == len(h) - 1


def test_step_limit_stops_early_with_a_warning():
    cfg, g, s = _c1_solver()
    _, _, info = s.step_adaptive(cfg["eta"], cfg["phi"], 0.0, cfg["period"], cfg["period"] / 64, 1e-6,
                                 tol=1e-13, max_steps=2)
    assert info["status"] == WARN_STEP_LIMIT and info["accepted"] + info["rejected"] == 2
    assert 0.0 < info["t"] < cfg["period"]
