"""Pins of the learned history seed (oracle.history_seed): the layer's
prediction, its loss gradient, Adam, and its use in fixed-step stepping."""
import math

import numpy as np
import pytest

import sbi_inputs as si
from oracle import Grid, Solver
from oracle import history_seed as hs


def _grid():
    return Grid(32, 16, 4 * math.pi, 2 * math.pi)


def test_prediction_is_newton_backward_extrapolation():
    # history h_q = p(-q) for a polynomial p of degree < K in time (random
    # coefficients per mode); weights C(r + q - 1, q) on the backward
    # differences give p(r) exactly (Newton's backward-difference formula),
    # here with r = 1 in some bins and r = 2 in others
    g = _grid()
    rng = np.random.Generator(np.random.PCG64(3))
    K, nb = 4, 6
    dk = g.kband / nb * 1.0001
    b = hs.bins(g, dk, nb)
    r_of_bin = np.array([1, 2, 1, 2, 2, 1])
    W = np.zeros((2, hs.STAGES, nb, K), complex)
    for bb in range(nb):
        for q in range(K):
            W[:, 2, bb, q] = math.comb(int(r_of_bin[bb]) + q - 1, q)
    coef = [rng.normal(size=g.k.shape) + 1j * rng.normal(size=g.k.shape) for _ in range(K)]
    hist = [(sum(coef[p] * float(-q) ** p for p in range(K)), None) for q in range(K)]
    pV, pB = hs.predict(W, hist, 2, b)
    r = r_of_bin[b].astype(float)
    exact = sum(coef[p] * r ** p for p in range(K))
    assert pB is None
    assert np.abs(pV - exact).max() < 1e-11 * np.abs(exact).max()


def test_gradient_matches_finite_differences():
    g = _grid()
    rng = np.random.Generator(np.random.PCG64(5))
    K, nb = 3, 5
    b = hs.bins(g, g.kband / nb * 1.0001, nb)
    c = hs.mode_weights(g)
    W = (rng.normal(size=(2, 4, nb, K)) + 1j * rng.normal(size=(2, 4, nb, K))) * 0.3
    hist = [tuple(g.mask * (rng.normal(size=g.k.shape) + 1j * rng.normal(size=g.k.shape)) for _ in range(2))
            for _ in range(K)]
    target = tuple(g.mask * (rng.normal(size=g.k.shape) + 1j * rng.normal(size=g.k.shape)) for _ in range(2))
    stage = 1
    L0, G, _ = hs.loss_grad(W, hist, target, stage, b, c, nb)
    eps = 1e-6
    for P, bb, q in [(0, 0, 0), (1, 3, 2), (0, 4, 1), (1, 2, 0)]:
        for part, unit in ((0, 1.0), (1, 1j)):
            Wp = W.copy()
            Wm = W.copy()
            Wp[P, stage, bb, q] += eps * unit
            Wm[P, stage, bb, q] -= eps * unit
            fd = (hs.loss_grad(Wp, hist, target, stage, b, c, nb)[0] -
                  hs.loss_grad(Wm, hist, target, stage, b, c, nb)[0]) / (2 * eps)
            an = G[P, bb, q].real if part == 0 else G[P, bb, q].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (P, bb, q, part, fd, an)
    # the loss is 0 for a perfect prediction and 1 (per part) for a zero one
    assert abs(hs.loss_grad(np.zeros_like(W), hist, target, stage, b, c, nb)[0] - 2.0) < 1e-12


def test_newton_step_lands_on_the_least_squares_weights():
    # per bin the loss summed over samples is a weighted least-squares problem
    # in the weights: numpy's lstsq on the sqrt(c/D)-scaled difference columns
    # gives its minimiser; one Newton step from any start lands there, and the
    # accumulated gradient vanishes there
    g = _grid()
    rng = np.random.Generator(np.random.PCG64(7))
    K, nb = 3, 4
    b = hs.bins(g, g.kband / nb * 1.0001, nb)
    c = hs.mode_weights(g)
    samples = []
    for _ in range(3):
        hist = [(g.mask * (rng.normal(size=g.k.shape) + 1j * rng.normal(size=g.k.shape)), None) for _ in range(K)]
        y = g.mask * (rng.normal(size=g.k.shape) + 1j * rng.normal(size=g.k.shape))
        samples.append((hist, (y, None)))
    W_ls = np.zeros((2, 4, nb, K), complex)
    for bb in range(nb):
        rows, rhs = [], []
        for hist, (y, _) in samples:
            D = np.sum(c * np.abs(y) ** 2)
            m = (b == bb) & (c > 0)
            sw = np.sqrt(c[m] / D)
            d = hs.differences(hist, 0)
            rows.append(np.stack([d[q][m] * sw for q in range(K)], 1))
            rhs.append(y[m] * sw)
        W_ls[0, 0, bb] = np.linalg.lstsq(np.concatenate(rows), np.concatenate(rhs), rcond=None)[0]
    G = sum(hs.loss_grad(W_ls, h, t, 0, b, c, nb)[1] for h, t in samples)
    assert np.abs(G[0]).max() < 1e-10
    W0 = (rng.normal(size=(2, 4, nb, K)) + 1j * rng.normal(size=(2, 4, nb, K)))
    gsum = np.zeros((2, 4, nb, K), complex)
    msum = np.zeros((2, 4, nb, K, K), complex)
    for h, t in samples:
        _, gr, gm = hs.loss_grad(W0, h, t, 0, b, c, nb)
        gsum[:, 0] += gr
        msum[:, 0] += gm
    W1 = hs.newton(W0, gsum, msum, 0.0)
    assert np.abs(W1[0, 0] - W_ls[0, 0]).max() < 1e-10
    assert np.array_equal(W1[:, 1:], W0[:, 1:])  # no samples at other stages: untouched


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    th = np.array([0.5, -1.0, 2.0])
    gr = np.array([3.0, -0.2, 1e-3])
    t1, m, v = hs.adam_step(th, np.zeros(3), np.zeros(3), gr, 1, 0.01)
    assert np.allclose(t1, th - 0.01 * np.sign(gr), atol=1e-7)


def _stepper(seed_mode, hist=None):
    cfg = si.config_c5(seed=2, n=64)
    g = cfg["grid"]
    G = Grid(g.nx, g.ny, g.lx, g.ly)
    return cfg, Solver(G, cfg["depth"], mode="iter", max_sweeps=200, accel="anderson", seed=seed_mode, hist=hist)


def test_identity_weights_are_the_previous_solve_seed():
    K, nb = 3, 8
    cfg, o_prev = _stepper("prev")
    _, o_hist = _stepper("net", hist=(K, nb, 0.5, hs.identity(K, nb)))
    e1, p1, s1 = o_prev.step(cfg["eta"], cfg["phi"], cfg["dt"], 3, tol=1e-9)
    e2, p2, s2 = o_hist.step(cfg["eta"], cfg["phi"], cfg["dt"], 3, tol=1e-9)
    assert [x.sweeps for x in s1] == [x.sweeps for x in s2]
    assert np.abs(e1 - e2).max() < 1e-13 and np.abs(p1 - p2).max() < 1e-13


def _record(seed, steps, K):
    """(history, target, stage) of every fixed-step solve with K solves behind
    it, from stepping a 64^2 sea of the benchmark recipe with the
    previous-solve seed."""
    cfg = si.config_c5(seed=seed, n=64)
    g = cfg["grid"]
    o = Solver(Grid(g.nx, g.ny, g.lx, g.ly), cfg["depth"], mode="iter", max_sweeps=200, accel="anderson",
               seed="prev")
    parts = []
    orig = o.w_iter_hat

    def spy(eta, ph, tol, seed_hat=None, seed_b_hat=None, stage=None):
        Vh, info = orig(eta, ph, tol, seed_hat, seed_b_hat, stage)
        parts.append((o._prev[0], o._prev[1], stage))
        return Vh, info

    o.w_iter_hat = spy
    o.step(cfg["eta"], cfg["phi"], cfg["dt"], steps, tol=1e-10)
    out = []
    for i in range(K, len(parts)):
        hist = [(parts[i - 1 - q][0], parts[i - 1 - q][1]) for q in range(K)]
        out.append((hist, (parts[i][0], parts[i][1]), parts[i][2]))
    return o.g, out


def test_adam_step_lowers_the_loss_on_its_samples():
    K, nb, dk = 4, 8, 0.6
    g, samples = _record(2, 4, K)
    b = hs.bins(g, dk, nb)
    c = hs.mode_weights(g)
    th = hs.identity(K, nb).astype(np.float64)

    def total(theta):
        W = hs.to_complex(theta, K, nb)
        L, G = 0.0, np.zeros((2, 4, nb, K), complex)
        for h, t, st in samples:
            l_, g_, _ = hs.loss_grad(W, h, t, st, b, c, nb)
            L += l_
            G[:, st] += g_
        return L / len(samples), G / len(samples)

    L0, G = total(th)
    gflat = np.stack([G.real, G.imag], axis=-1).ravel()
    th1, _, _ = hs.adam_step(th, np.zeros_like(th), np.zeros_like(th), gflat, 1, 1e-3)
    L1, _ = total(th1)
    assert L1 < L0, (L0, L1)


def test_trained_history_layer_saves_sweeps_on_another_sea():
    # trained by the oracle's own Gauss-Newton step on one sea, the layer
    # steps a second sea (other depth and phases) in fewer sweeps than the
    # previous-solve seed
    K, nb, dk = 6, 10, 0.4
    cfg, o = _stepper("net", hist=(K, nb, dk, hs.identity(K, nb)))
    o.hist_train = True
    eta, phi, _ = o.step(cfg["eta"], cfg["phi"], cfg["dt"], 10, tol=1e-10)
    loss0 = o._hist_acc["loss"] / o._hist_acc["n"]
    o.hist_newton(1e-9)
    o.step(eta, phi, cfg["dt"], 2, tol=1e-10, t0=10 * cfg["dt"])
    loss1 = o._hist_acc["loss"] / o._hist_acc["n"]
    assert loss1 < 0.05 * loss0, (loss0, loss1)
    cfg2 = si.config_c5(seed=3, n=64)
    g2 = cfg2["grid"]
    G2 = Grid(g2.nx, g2.ny, g2.lx, g2.ly)
    oh = Solver(G2, cfg2["depth"], mode="iter", max_sweeps=200, accel="anderson", seed="net",
                hist=(K, nb, dk, o.hist["theta"]))
    op = Solver(G2, cfg2["depth"], mode="iter", max_sweeps=200, accel="anderson", seed="prev")
    _, _, sh = oh.step(cfg2["eta"], cfg2["phi"], cfg2["dt"], 6, tol=1e-8)
    _, _, sp = op.step(cfg2["eta"], cfg2["phi"], cfg2["dt"], 6, tol=1e-8)
    nh = sum(x.sweeps for x in sh[K:])
    npv = sum(x.sweeps for x in sp[K:])
    assert nh < 0.85 * npv, (nh, npv)
