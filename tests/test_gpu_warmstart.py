"""The learned warm start on the GPU against its FP64 oracle (oracle/warmstart.py).

Tolerances:
* features (FP32 output of an FP64 spectral computation): 2e-7 relative to each
  channel's max;
* training forward / loss / gradient (FP32 kernels, BF16-rounded weights):
  1e-4 relative in max norm per parameter tensor (FP32 sums over the points);
* Adam: 1e-6 relative;
* matrix-core inference (BF16 activations, FP32 accumulation) against the
  oracle that rounds the same activations to BF16: a rounding decision flips
  where the FP32 and FP64 sums straddle a BF16 boundary (about one element in
  2^9 scaled by the sum's relative error), each flip moving an activation by
  one BF16 ulp (2^-8 relative); the bound 1e-2 of max|y| on the worst point
  and 1e-3 on the 99th percentile covers that with margin.
"""
import math
import sys

import numpy as np
import pytest

import sbi_inputs as si

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n=64, seed=3):
    from oracle import Grid, Solver
    gs = si.GridSpec(n, n, 8 * 2 * math.pi, 8 * 2 * math.pi)
    eta, phi = si.jonswap_crossing_sea(gs, 1.5, seed=seed, hs_half=0.1)
    depth = si.random_bumps_depth(gs, 1.5, 40 + seed)
    o = Solver(Grid(n, n, gs.lx, gs.ly), depth, h_ref=1.5, mode="iter", max_sweeps=300)
    return gs, eta, phi, depth, o


def _solver(gpu, gs, depth, batch=1, **kw):
    from paper_2310_19840_amd import Solver
    return Solver(gs.nx, gs.ny, gs.lx, gs.ly, depth, h_ref=1.5, batch=batch, device=gpu, **kw)


def _theta(seed, w4=0.2):
    from oracle import warmstart as ws
    th = ws.init_params(seed)
    p = ws.unpack(th.copy())
    rng = np.random.default_rng(seed + 100)
    p["W4"] = rng.standard_normal((2, 32)) * w4
    p["b1"] = rng.standard_normal(32) * 0.1
    p["b2"] = rng.standard_normal(32) * 0.1
    p["b3"] = rng.standard_normal(32) * 0.1
    p["b4"] = np.array([0.05, -0.03])
    return ws.pack(p).astype(np.float32)


SCALES = np.array([8.0, 4.0, 3.0, 3.0, 2.0, 2.0, 1.5, 20.0], dtype=np.float32)


def test_features_match_oracle(gpu):
    import torch
    from oracle import warmstart as ws
    from paper_2310_19840_amd import net_blob
    gs, eta, phi, depth, o = _case()
    _say("features", gs.nx)
    s = _solver(gpu, gs, depth)
    s.net_load(net_blob(_theta(0), SCALES, (0.5, 0.3)))
    e = torch.tensor(eta[None], dtype=torch.float64, device=gpu)
    p = torch.tensor(phi[None], dtype=torch.float64, device=gpu)
    feat, wlin = s.net_features(e, p)
    fo, wo = ws.features(o, eta, phi)
    fo = fo * SCALES.astype(np.float64)
    fg = feat.cpu().numpy()[0].astype(np.float64)
    for c in range(8):
        scale = max(np.abs(fo[..., c]).max(), 1e-30)
        assert np.abs(fg[..., c] - fo[..., c]).max() <= 2e-7 * scale, c
    assert np.abs(wlin.cpu().numpy()[0] - wo).max() < 1e-12 * np.abs(wo).max()


def _train_inputs(n=64, batch=2, seed=5):
    rng = np.random.default_rng(seed)
    # smooth random features: sums of a few periodic modes per channel
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = np.zeros((batch, n, n, 8))
    for b in range(batch):
        for c in range(8):
            for _ in range(4):
                kx, ky = rng.integers(-6, 7, 2)
                f[b, :, :, c] += rng.standard_normal() * np.cos(2 * np.pi * (kx * x + ky * y) / n + rng.uniform(0, 6.3))
    t = np.stack([0.3 * np.tanh(f[..., 0] * f[..., 1]) + 0.1 * f[..., 2] - 0.05 * f[..., 7],
                  0.2 * np.tanh(f[..., 6] * f[..., 3])], axis=-1)
    return f.astype(np.float32), t.astype(np.float32)


def test_trainer_gradient_and_adam_match_oracle(gpu):
    import torch
    from oracle import warmstart as ws
    from paper_2310_19840_amd import NetTrainer
    f, t = _train_inputs()
    th = _theta(1)
    _say("trainer gradient")
    tr = NetTrainer(2, 64, 64, th, device=gpu)
    fd = torch.tensor(f, device=gpu)
    td = torch.tensor(t, device=gpu)
    y = tr.forward(fd).cpu().numpy().astype(np.float64)
    yo = ws.forward(th.astype(np.float64), f.astype(np.float64), bf16_weights=True)
    assert np.abs(y - yo).max() < 1e-4 * np.abs(yo).max()
    loss, g = tr.gradient(fd, td, want_grad=True)
    lo, go = ws.loss_and_grad(th.astype(np.float64), f.astype(np.float64), t.astype(np.float64), bf16_weights=True)
    assert abs(loss - lo) < 1e-4 * lo
    off = 0
    for name, shp in ws.SHAPES:
        k = int(np.prod(shp))
        a, b = g[off:off + k].astype(np.float64), go[off:off + k]
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max() + 1e-12, name
        off += k
    # one Adam step from zero moments, on the device's gradient
    tr.adam(1e-3)
    tho, _, _ = ws.adam_step(th.astype(np.float64), np.zeros(ws.PARAM_COUNT), np.zeros(ws.PARAM_COUNT),
                             g.astype(np.float64), 1, lr=1e-3)
    assert np.abs(tr.params() - tho).max() < 1e-6 * np.abs(tho).max()


def test_inference_matches_oracle(gpu):
    import torch
    from oracle import warmstart as ws
    from paper_2310_19840_amd import net_blob
    gs, eta, phi, depth, o = _case(64, 7)
    th = _theta(2, w4=0.5)
    _say("inference")
    s = _solver(gpu, gs, depth)
    osc = (0.25, 0.125)
    s.net_load(net_blob(th, SCALES, osc))
    e = torch.tensor(eta[None], dtype=torch.float64, device=gpu)
    p = torch.tensor(phi[None], dtype=torch.float64, device=gpu)
    feat, wlin = s.net_features(e, p)
    seed, db = s.net_infer(feat, wlin)
    seed, db = seed.cpu().numpy()[0], db.cpu().numpy()[0]
    x = feat.cpu().numpy().astype(np.float64)
    yo = ws.forward(th.astype(np.float64), x, bf16_weights=True, bf16_acts=True)[0]
    ys = [(seed - wlin.cpu().numpy()[0]) / osc[0], db / osc[1]]
    for k in range(2):
        err = np.abs(ys[k] - yo[..., k])
        ymax = np.abs(yo[..., k]).max()
        assert err.max() <= 1e-2 * ymax, k
        assert np.quantile(err, 0.99) <= 1e-3 * ymax, k
    # and the oracle's seeds of the same state (features computed by the oracle)
    so, dbo = ws.seed(th.astype(np.float64), SCALES, osc, o, eta, phi)
    assert np.abs(seed - so).max() <= 1e-2 * osc[0] * np.abs(yo[..., 0]).max() + 1e-6 * np.abs(so).max()
    assert np.abs(db - dbo).max() <= 1e-2 * osc[1] * np.abs(yo[..., 1]).max()


def test_net_seed_converges_to_the_same_w(gpu):
    import torch
    from paper_2310_19840_amd import net_blob
    gs, eta, phi, depth, o = _case(64, 9)
    _say("net seed solve")
    e = torch.tensor(eta[None], dtype=torch.float64, device=gpu)
    p = torch.tensor(phi[None], dtype=torch.float64, device=gpu)
    sl = _solver(gpu, gs, depth, mode="iter", max_sweeps=300)
    Wl, stl, il = sl.vertical_velocity(e, p, tol=1e-11)
    sn = _solver(gpu, gs, depth, mode="iter", seed="net", max_sweeps=300)
    sn.net_load(net_blob(_theta(3, w4=0.05), SCALES, (0.05, 0.05)))
    Wn, stn, inn = sn.vertical_velocity(e, p, tol=1e-11)
    assert stl == 0 and stn == 0 and inn[0][1] == 0
    Wo, oi = o.vertical_velocity(eta, phi, tol=1e-11)
    assert il[0][0] == oi.sweeps
    scale = np.abs(Wo).max()
    assert np.abs(Wl.cpu().numpy()[0] - Wo).max() < 1e-10 * scale
    assert np.abs(Wn.cpu().numpy()[0] - Wo).max() < 1e-9 * scale


def test_failed_net_seed_falls_back_to_linear(gpu):
    import torch
    from paper_2310_19840_amd import _lib, net_blob
    gs, eta, phi, depth, o = _case(64, 11)
    _say("net seed fallback (FP32 overflow of the seed)")
    e = torch.tensor(eta[None], dtype=torch.float32, device=gpu)
    p = torch.tensor(phi[None], dtype=torch.float32, device=gpu)
    sl = _solver(gpu, gs, depth, mode="iter", precision="fp32", max_sweeps=100)
    Wl, stl, il = sl.vertical_velocity(e, p, tol=1e-5)
    sn = _solver(gpu, gs, depth, mode="iter", precision="fp32", seed="net", max_sweeps=100)
    # out_scale near FLT_MAX turns the FP32 seed into +-inf: the solve from it
    # is non-finite and is redone from the linear guess
    sn.net_load(net_blob(_theta(4, w4=2.0), SCALES, (3.0e38, 3.0e38)))
    Wn, stn, inn = sn.vertical_velocity(e, p, tol=1e-5)
    assert stn == _lib.SBI_WARN_FALLBACK_USED
    assert inn[0][0] == il[0][0]
    assert np.array_equal(Wn.cpu().numpy(), Wl.cpu().numpy())


def test_trained_net_saves_sweeps(gpu):
    """What the trained network gains: fewer sweeps to the same tolerance on
    states it was not trained on (the iteration's residual still decides)."""
    from paper_2310_19840_amd import warmstart as wst
    _say("train warm start: 32 states at 128^2")
    feat, dv, db, _ = wst.make_samples(range(100, 132), 128, gpu)
    blob, hist = wst.fit(feat, dv, db, steps=400, batch=4, lr=3e-3, device=gpu)
    _say("loss", hist[:5].mean(), "->", hist[-20:].mean())
    assert hist[-20:].mean() < 0.3 * hist[:5].mean()
    held = range(900, 906)
    lin = wst.sweeps_with(blob, held, 128, gpu, seed_mode="linear")
    net = wst.sweeps_with(blob, held, 128, gpu, seed_mode="net")
    _say("held-out sweeps linear", lin, "net", net)
    assert all(st == 0 for _, st in lin + net)
    assert np.mean([s for s, _ in net]) < np.mean([s for s, _ in lin])


def test_labels_match_oracle(gpu):
    """sbi_last_correction: the nonlinear parts of a converged solve."""
    import torch
    from oracle import warmstart as ws
    gs, eta, phi, depth, o = _case(64, 13)
    _say("labels")
    s = _solver(gpu, gs, depth, mode="iter", seed="prev", max_sweeps=300)
    e = torch.tensor(eta[None], dtype=torch.float64, device=gpu)
    p = torch.tensor(phi[None], dtype=torch.float64, device=gpu)
    _, st, info = s.vertical_velocity(e, p, tol=1e-11)
    dv, db = s.last_correction()
    dvo, dbo, oi = ws.labels(o, eta, phi, tol=1e-11)
    assert info[0][0] == oi.sweeps
    assert np.abs(dv.cpu().numpy()[0] - dvo).max() < 1e-10 * np.abs(dvo).max()
    assert np.abs(db.cpu().numpy()[0] - dbo).max() < 1e-10 * np.abs(dbo).max()
