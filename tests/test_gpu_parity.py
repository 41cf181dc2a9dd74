"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Tolerances: FP64 runs 1e-10 relative in max norm (observed ~1e-13), FP32 runs
1e-5 relative, for W and for eta after the stated steps.  Iteration sweep
counts must match the oracle exactly.
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


def _oracle():
    from oracle import Grid, Solver
    return Grid, Solver


def _t(x, dtype, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _fields(nx, ny, lx, ly, seed, amp_eta=0.05, amp_phi=0.5, bump=0.2, h=1.0):
    gs = si.GridSpec(nx, ny, lx, ly)
    eta = si.band_limited_random(gs, seed, amp=amp_eta, slope=2.5)
    phi = si.band_limited_random(gs, seed + 100, amp=amp_phi, slope=2.0)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = h - bump * np.exp(-((X - lx / 3) ** 2 + ((Y - ly / 2) ** 2 if ny > 1 else 0)) / (0.05 * lx * lx))
    return eta, phi, depth


def _solver(gpu, nx, ny, lx, ly, depth, batch=1, **kw):
    from paper_2310_19840_amd import Solver
    return Solver(nx, ny, lx, ly, depth, batch=batch, device=gpu, **kw)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nx,ny", [(64, 1), (256, 1), (32, 16), (64, 64)])
def test_linear_flat_limit_gpu(gpu, nx, ny):
    import torch
    lx, ly = 4 * math.pi, 2 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    X, Y = np.meshgrid(gs.x(), gs.y())
    mx, my = 3, (2 if ny > 1 else 0)
    kx, ky = 2 * math.pi * mx / lx, 2 * math.pi * my / ly
    k = math.hypot(kx, ky)
    h = 1.3
    phi = np.cos(kx * X + ky * Y + 0.4)
    for mode in ("sa", "iter"):
        _say("linear flat", nx, ny, mode)
        s = _solver(gpu, nx, ny, lx, ly, np.full((ny, nx), h), mode=mode)
        W, st, info = s.vertical_velocity(_t(np.zeros((ny, nx)), torch.float64, gpu), _t(phi, torch.float64, gpu),
                                          tol=1e-14)
        W = W.cpu().numpy()[0]
        assert np.abs(W - k * math.tanh(k * h) * phi).max() < 1e-13
        if mode == "iter":
            assert info[0][0] == 1 and info[0][2] == 0.0


@pytest.mark.parametrize("nx,ny,vd", [(64, 1, True), (256, 1, True), (32, 16, True), (64, 32, True),
                                      (128, 64, False), (64, 128, True)])
def test_sa_vertical_velocity_matches_oracle(gpu, nx, ny, vd):
    import torch
    Grid, Solver = _oracle()
    lx, ly = 4 * math.pi, 3 * math.pi
    eta, phi, depth = _fields(nx, ny, lx, ly, seed=nx + ny, bump=0.2 if vd else 0.0)
    _say("SA W", nx, ny, vd)
    s = _solver(gpu, nx, ny, lx, ly, depth, h_ref=1.0, mode="sa")
    W, st, _ = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu))
    o = Solver(Grid(nx, ny, lx, ly), depth, h_ref=1.0, mode="sa")
    Wo, _ = o.vertical_velocity(eta, phi)
    assert _rel(W.cpu().numpy()[0], Wo) < 1e-12


@pytest.mark.parametrize("nx,ny,vd", [(64, 1, True), (256, 1, False), (32, 16, True), (64, 64, True),
                                      (128, 32, False)])
def test_iter_vertical_velocity_matches_oracle(gpu, nx, ny, vd):
    import torch
    Grid, Solver = _oracle()
    lx, ly = 4 * math.pi, 3 * math.pi
    eta, phi, depth = _fields(nx, ny, lx, ly, seed=7 * nx + ny, bump=0.2 if vd else 0.0)
    _say("ITER W", nx, ny, vd)
    s = _solver(gpu, nx, ny, lx, ly, depth, h_ref=1.0, mode="iter", max_sweeps=200)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
    o = Solver(Grid(nx, ny, lx, ly), depth, h_ref=1.0, mode="iter", max_sweeps=200)
    Wo, oi = o.vertical_velocity(eta, phi, tol=1e-12)
    assert info[0][0] == oi.sweeps, (info, oi.sweeps, oi.history[-3:])
    assert info[0][1] == oi.status
    assert abs(info[0][3] - oi.omega) < 1e-14
    assert _rel(W.cpu().numpy()[0], Wo) < 1e-11


@pytest.mark.parametrize("mode", ["sa", "iter"])
def test_fp32_vertical_velocity(gpu, mode):
    import torch
    Grid, Solver = _oracle()
    nx, ny = 128, 64
    lx, ly = 8 * math.pi, 4 * math.pi
    eta, phi, depth = _fields(nx, ny, lx, ly, seed=31)
    _say("FP32 W", mode)
    s = _solver(gpu, nx, ny, lx, ly, depth, h_ref=1.0, mode=mode, precision="fp32", max_sweeps=200)
    W, st, info = s.vertical_velocity(_t(eta, torch.float32, gpu), _t(phi, torch.float32, gpu), tol=1e-6)
    o = Solver(Grid(nx, ny, lx, ly), depth, h_ref=1.0, mode=mode, max_sweeps=200)
    Wo, _ = o.vertical_velocity(eta.astype(np.float32).astype(np.float64), phi.astype(np.float32).astype(np.float64),
                                tol=1e-12)
    assert _rel(W.cpu().numpy()[0].astype(np.float64), Wo) < 1e-5


def test_step_1d_c1_window(gpu):
    """C1 geometry (1D N=256, Gaussian bump, Stokes), iteration tol 1e-10, FP64."""
    import torch
    Grid, Solver = _oracle()
    cfg = si.config_c1()
    g = cfg["grid"]
    n = 4
    _say("step C1 window", n)
    s = _solver(gpu, g.nx, 1, g.lx, 1.0, cfg["depth"], h_ref=cfg["h_ref"], mode="iter", max_sweeps=200)
    e = _t(cfg["eta"], torch.float64, gpu)
    p = _t(cfg["phi"], torch.float64, gpu)
    st, info = s.step(e, p, cfg["dt"], n, tol=cfg["tol"])
    o = Solver(Grid(g.nx, 1, g.lx), cfg["depth"], h_ref=cfg["h_ref"], mode="iter", max_sweeps=200)
    eo, po, stats = o.step(cfg["eta"], cfg["phi"], cfg["dt"], n, tol=cfg["tol"])
    assert info["sweeps_total"] == sum(x.sweeps for x in stats)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


@pytest.mark.parametrize("mode", ["sa", "iter"])
def test_step_2d_variable_depth(gpu, mode):
    import torch
    Grid, Solver = _oracle()
    nx, ny = 64, 32
    lx, ly = 8 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 1.0, seed=5, hs_half=0.03)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.0 - 0.15 * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 2) ** 2) / 20.0)
    dt = 2 * math.pi / math.sqrt(math.tanh(1.0)) / 64
    n = 3
    _say("step 2D", mode)
    s = _solver(gpu, nx, ny, lx, ly, depth, mode=mode, max_sweeps=200)
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    s.step(e, p, dt, n, tol=1e-11)
    o = Solver(Grid(nx, ny, lx, ly), depth, mode=mode, max_sweeps=200)
    eo, po, _ = o.step(eta, phi, dt, n, tol=1e-11)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


@pytest.mark.parametrize("nx,ny", [(64, 1), (64, 32)])
def test_prev_seed_matches_oracle(gpu, nx, ny):
    """Previous-solve seed: same states as the oracle, same sweep count per solve."""
    import torch
    Grid, Solver = _oracle()
    lx, ly = 8 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    X, Y = np.meshgrid(gs.x(), gs.y())
    if ny > 1:
        eta, phi = si.jonswap_crossing_sea(gs, 1.0, seed=9, hs_half=0.03)
        depth = 1.0 - 0.15 * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 2) ** 2) / 20.0)
    else:
        eta, phi, _ = si.stokes2_finite_depth(gs, 0.03, 1.0, k0=1.0)
        depth = 1.0 - 0.2 * np.exp(-((X - lx / 2) ** 2) / 8.0)
    dt = 2 * math.pi / math.sqrt(math.tanh(1.0)) / 64
    _say("prev seed", nx, ny)
    s = _solver(gpu, nx, ny, lx, ly, depth, mode="iter", seed="prev", max_sweeps=200)
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    _, info = s.step(e, p, dt, 3, tol=1e-11)
    o = Solver(Grid(nx, ny, lx, ly), depth, mode="iter", seed="prev", max_sweeps=200)
    eo, po, so_ = o.step(eta, phi, dt, 3, tol=1e-11)
    assert info["sweeps_total"] == sum(x.sweeps for x in so_)
    assert info["sweeps_max"] == max(x.sweeps for x in so_)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10
    # a repeated solve at one state is seeded with its own answer: one sweep
    W1, _, i1 = s.vertical_velocity(e, p, tol=1e-11)
    W2, _, i2 = s.vertical_velocity(e, p, tol=1e-11)
    assert i2[0][0] == 1 and i2[0][1] == 0
    assert _rel(W2.cpu().numpy(), W1.cpu().numpy()) < 1e-10


def test_diagnostics_match_oracle(gpu):
    import torch
    Grid, Solver = _oracle()
    nx, ny = 64, 32
    lx, ly = 8 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 2.0, seed=9, hs_half=0.04)
    eta = eta + 0.003
    depth = np.full((ny, nx), 2.0)
    _say("diagnostics")
    s = _solver(gpu, nx, ny, lx, ly, depth, mode="sa")
    m, E = s.diagnostics(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu))
    o = Solver(Grid(nx, ny, lx, ly), depth, mode="sa")
    mo, Eo = o.diagnostics(eta, phi)
    assert abs(m[0] - mo) < 1e-12 * max(1, abs(mo))
    assert abs(E[0] - Eo) < 1e-12 * abs(Eo)


def test_batch_member_equals_single_run(gpu):
    import torch
    nx, ny = 64, 32
    lx, ly = 8 * math.pi, 4 * math.pi
    etas, phis, depths = [], [], []
    for b in range(3):
        e, p, d = _fields(nx, ny, lx, ly, seed=50 + b, bump=0.1 * (b + 1))
        etas.append(e)
        phis.append(p)
        depths.append(d)
    _say("batch vs single")
    sb = _solver(gpu, nx, ny, lx, ly, np.stack(depths), batch=3, mode="iter", max_sweeps=100)
    Wb, st, infos = sb.vertical_velocity(_t(np.stack(etas), torch.float64, gpu), _t(np.stack(phis), torch.float64, gpu),
                                         tol=1e-11)
    for b in range(3):
        s1 = _solver(gpu, nx, ny, lx, ly, depths[b], mode="iter", max_sweeps=100)
        W1, _, i1 = s1.vertical_velocity(_t(etas[b], torch.float64, gpu), _t(phis[b], torch.float64, gpu), tol=1e-11)
        assert infos[b][0] == i1[0][0]
        assert torch.equal(Wb[b], W1[0])


def test_status_codes_gpu(gpu):
    import torch
    from paper_2310_19840_amd import SBIError, _lib
    nx, ny = 64, 1
    lx = 4 * math.pi
    eta, phi, depth = _fields(nx, ny, lx, 1.0, seed=3)
    _say("status codes")
    s = _solver(gpu, nx, ny, lx, 1.0, depth, mode="iter", max_sweeps=1)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-13)
    assert st == _lib.SBI_WARN_NOT_CONVERGED and info[0][0] == 1
    s2 = _solver(gpu, nx, ny, lx, 1.0, depth, mode="iter")
    e2 = eta.copy()
    e2[0, 5] = np.nan
    with pytest.raises(SBIError) as ex:
        s2.vertical_velocity(_t(e2, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
    assert ex.value.code == _lib.SBI_ERR_NONFINITE


def test_user_seed_converged_w_takes_one_sweep(gpu):
    import torch
    nx, ny = 64, 32
    lx, ly = 8 * math.pi, 4 * math.pi
    eta, phi, depth = _fields(nx, ny, lx, ly, seed=77, bump=0.0)
    _say("user seed")
    s = _solver(gpu, nx, ny, lx, ly, depth, mode="iter", max_sweeps=100)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-13)
    su = _solver(gpu, nx, ny, lx, ly, depth, mode="iter", max_sweeps=100, seed="user")
    W2, st2, info2 = su.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12,
                                          w_seed=W)
    assert info2[0][0] <= 2 < info[0][0]
    assert _rel(W2.cpu().numpy(), W.cpu().numpy()) < 1e-12


def test_relaxation_zone_matches_oracle(gpu):
    import torch
    Grid, Solver = _oracle()
    cfg = si.config_c2(case=2, nx=512, steps=6)
    g = cfg["grid"]
    rz = cfg["relax"]
    _say("relaxation zone")
    s = _solver(gpu, g.nx, 1, g.lx, 1.0, cfg["depth"], h_ref=cfg["h_ref"], mode="sa")
    s.set_relaxation(rz["a"], rz["k"], rz["omega"], rz["gen_len"], rz["abs_len"], rz["ramp_periods"])
    e = _t(cfg["eta"], torch.float64, gpu)
    p = _t(cfg["phi"], torch.float64, gpu)
    dt = cfg["dt"] * 8
    s.step(e, p, dt, cfg["steps"])
    o = Solver(Grid(g.nx, 1, g.lx), cfg["depth"], h_ref=cfg["h_ref"], mode="sa", relaxation_zone=rz)
    eo, po, _ = o.step(cfg["eta"], cfg["phi"], dt, cfg["steps"])
    assert np.abs(eo).max() > 1e-4
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10


def _steep_1d():
    nx = 64
    lx = 4 * math.pi
    x = np.arange(nx) * lx / nx
    eta = (0.15 * np.cos(2 * math.pi * 3 * x / lx) + 0.02 * np.cos(2 * math.pi * 11 * x / lx + 1.0))[None]
    phi = (0.5 * np.sin(2 * math.pi * 3 * x / lx) + 0.1 * np.sin(2 * math.pi * 7 * x / lx))[None]
    return nx, lx, eta, phi


@pytest.mark.parametrize("accel", [None, "anderson"])
def test_divergence_status_matches_oracle(gpu, accel):
    """Plain sweeps (relax off) on a crest beyond the contraction range: the
    residual first falls, then grows from round-off in the short waves; both
    sides stop with SBI_ERR_DIVERGED at the same sweep (or, mixed, reach the
    same outcome)."""
    import torch
    from paper_2310_19840_amd import SBIError, _lib
    Grid, Solver = _oracle()
    nx, lx, eta, phi = _steep_1d()
    depth = np.full((1, nx), 1.0)
    _say("divergence", accel)
    o = Solver(Grid(nx, 1, lx), depth, mode="iter", max_sweeps=500, relax=False, accel=accel)
    Wo, oi = o.vertical_velocity(eta, phi, tol=1e-12)
    s = _solver(gpu, nx, 1, lx, 1.0, depth, mode="iter", max_sweeps=500, relax=False, accel=accel)
    if oi.status < 0:
        with pytest.raises(SBIError) as ex:
            s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
        assert ex.value.code == oi.status == _lib.SBI_ERR_DIVERGED
        assert ex.value.info[0][0] == oi.sweeps, (ex.value.info, oi.sweeps)
    else:
        W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
        assert info[0][0] == oi.sweeps and info[0][1] == oi.status
        assert _rel(W.cpu().numpy()[0], Wo) < 1e-10
    if accel is None:
        assert oi.status == _lib.SBI_ERR_DIVERGED
    # a step that meets a diverged solve reports the error and leaves the state untouched
    if oi.status < 0:
        e = _t(eta, torch.float64, gpu)
        p = _t(phi, torch.float64, gpu)
        e0, p0 = e.clone(), p.clone()
        with pytest.raises(SBIError) as ex:
            s.step(e, p, 0.05, 1, tol=1e-12)
        assert ex.value.code == _lib.SBI_ERR_DIVERGED
        assert torch.equal(e, e0) and torch.equal(p, p0)


def test_depth_criterion_warning_matches_oracle(gpu):
    """Sec. 5: k_band max|delta| > 2.4 makes sbi_init warn (context usable),
    exactly where the oracle sets its depth warning."""
    import torch
    from paper_2310_19840_amd import _lib
    Grid, Solver = _oracle()
    nx = 64
    lx = 8 * math.pi
    g = Grid(nx, 1, lx)
    x = np.arange(nx) * lx / nx
    bump = np.exp(-((x - lx / 2) / 2.0) ** 2)[None]
    eta = 0.01 * np.cos(2 * math.pi * 4 * x / lx)[None]
    phi = 0.05 * np.sin(2 * math.pi * 4 * x / lx)[None]
    _say("depth criterion")
    for kd, warn in ((2.3, False), (2.5, True)):
        depth = 2.0 - (kd / g.kband) * bump
        o = Solver(g, depth, h_ref=2.0, mode="sa")
        assert o.depth_warning == warn
        s = _solver(gpu, nx, 1, lx, 1.0, depth, h_ref=2.0, mode="sa")
        assert s.init_status == (_lib.SBI_WARN_DEPTH_CRITERION if warn else _lib.SBI_OK)
        W, st, _ = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu))
        Wo, _ = o.vertical_velocity(eta, phi)
        assert _rel(W.cpu().numpy()[0], Wo) < 1e-12
        # a new depth passed to the solve re-checks the criterion
        W, st, _ = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), h=depth)
        assert st == (_lib.SBI_WARN_DEPTH_CRITERION if warn else _lib.SBI_OK)
