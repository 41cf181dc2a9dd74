"""Parity of the numerical wave tank of Sec. 3.2 (pneumatic wavemaker p_g and
damping pressure p_d of Eq. (pd), sbi_set_wavemaker) with the FP64 oracle,
under the fixed RK4 step and the adaptive pair.  Tolerances: FP64 1e-10
relative in max norm, FP32 1e-5."""
import math
import sys

import numpy as np
import pytest

import sbi_inputs as si

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(x, dtype, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _tank_1d(h=1.0, nx=512, nlam=32):
    L = nlam * 2 * math.pi
    x = np.arange(nx) * L / nx
    # a gentle shoal in the middle of the tank
    depth = h - 0.3 * h * np.exp(-((x - 0.45 * L) / (0.06 * L)) ** 2)
    om = math.sqrt(math.tanh(h))
    comps = [(0.02, 1.0, om, 0.3), (0.006, 1.6, math.sqrt(1.6 * math.tanh(1.6 * h)), 1.1)]
    return L, depth[None], comps, dict(comps=comps, x0=7 * L / 8)


def _pair(gpu, nx, ny, lx, ly, depth, wm, mode="sa", precision="fp64", **kw):
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    s = Solver(nx, ny, lx, ly, depth, device=gpu, mode=mode, precision=precision, max_sweeps=200, **kw)
    s.set_wavemaker(wm.get("comps", ()), x0=wm.get("x0"), width=wm.get("width", 4 * math.pi), h=wm.get("h"))
    o = OSolver(Grid(nx, ny, lx, ly), depth, mode=mode, max_sweeps=200, wavemaker=wm, **kw)
    return s, o


@pytest.mark.parametrize("mode", ["sa", "iter"])
def test_tank_1d_rk4_from_rest(gpu, mode):
    import torch
    L, depth, comps, wm = _tank_1d()
    nx = depth.shape[1]
    s, o = _pair(gpu, nx, 1, L, 1.0, depth, wm, mode=mode)
    T = 2 * math.pi / comps[0][2]
    dt, n, t0 = T / 16, 48, 3.7
    _say("tank 1D rk4", mode)
    e = _t(np.zeros((1, nx)), torch.float64, gpu)
    p = _t(np.zeros((1, nx)), torch.float64, gpu)
    st, info = s.step(e, p, dt, n, tol=1e-12, t=t0)
    eo, po, _ = o.step(np.zeros((1, nx)), np.zeros((1, nx)), dt, n, tol=1e-12, t0=t0)
    assert np.abs(eo).max() > 5e-3           # waves have left the generator
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def test_tank_2d_variable_depth_iter(gpu):
    import torch
    nx, ny = 64, 32
    lx, ly = 16 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 1.0, seed=7, hs_half=0.03)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.0 - 0.15 * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 2) ** 2) / 20.0)
    wm = dict(comps=[(0.01, 1.0, math.sqrt(math.tanh(1.0)), 0.0)], x0=0.75 * lx, width=2.0, h=1.2)
    s, o = _pair(gpu, nx, ny, lx, ly, depth, wm, mode="iter")
    dt, n = 2 * math.pi / 32, 6
    _say("tank 2D")
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    s.step(e, p, dt, n, tol=1e-12, t=1.25)
    eo, po, _ = o.step(eta, phi, dt, n, tol=1e-12, t0=1.25)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


@pytest.mark.parametrize("which", ["damping only", "wavemaker only"])
def test_tank_pressures_separately(gpu, which):
    import torch
    nx, ny = 64, 16
    lx, ly = 16 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 1.0, seed=9, hs_half=0.03)
    if which == "damping only":
        wm = dict(comps=[], x0=0.5 * lx, width=6.0)
    else:
        wm = dict(comps=[(0.01, 1.0, 0.9, 0.2), (0.004, 2.0, 1.3, 0.0)])
    s, o = _pair(gpu, nx, ny, lx, ly, np.ones((ny, nx)), wm)
    dt, n = 2 * math.pi / 32, 8
    _say("tank", which)
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    s.step(e, p, dt, n)
    eo, po, _ = o.step(eta, phi, dt, n)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def test_tank_1d_adaptive(gpu):
    import torch
    L, depth, comps, wm = _tank_1d()
    nx = depth.shape[1]
    s, o = _pair(gpu, nx, 1, L, 1.0, depth, wm, mode="iter")
    T = 2 * math.pi / comps[0][2]
    _say("tank 1D adaptive")
    e = _t(np.zeros((1, nx)), torch.float64, gpu)
    p = _t(np.zeros((1, nx)), torch.float64, gpu)
    st, info = s.step_adaptive(e, p, 2.5 + 2 * T, T / 8, 1e-7, tol=1e-12, t=2.5)
    eo, po, oi = o.step_adaptive(np.zeros((1, nx)), np.zeros((1, nx)), 2.5, 2.5 + 2 * T, T / 8, 1e-7, tol=1e-12)
    assert oi["accepted"] >= 4
    assert (info["accepted"], info["rejected"]) == (oi["accepted"], oi["rejected"])
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def test_tank_fp32(gpu):
    import torch
    L, depth, comps, wm = _tank_1d()
    nx = depth.shape[1]
    s, o = _pair(gpu, nx, 1, L, 1.0, depth, wm, precision="fp32")
    T = 2 * math.pi / comps[0][2]
    _say("tank fp32")
    e = _t(np.zeros((1, nx)), torch.float32, gpu)
    p = _t(np.zeros((1, nx)), torch.float32, gpu)
    s.step(e, p, T / 16, 32)
    eo, _, _ = o.step(np.zeros((1, nx)), np.zeros((1, nx)), T / 16, 32)
    assert _rel(e.cpu().numpy().reshape(eo.shape).astype(np.float64), eo) < 1e-5


def test_tank_settings_checked(gpu):
    import torch
    from paper_2310_19840_amd import SBIError, Solver, _lib
    s = Solver(64, 1, 10.0, 1.0, np.ones((1, 64)), device=gpu, mode="sa")
    _say("tank settings")
    for comps in ([(0.01, 0.0, 1.0, 0.0)], [(0.01, 1.0, -1.0, 0.0)], [(0.01, 1.0, 1.0, float("nan"))],
                  [(0.01, 1.0, 1.0, 0.0)] * 9):
        with pytest.raises(SBIError) as ex:
            s.set_wavemaker(comps)
        assert ex.value.code == _lib.SBI_ERR_INVALID_ARG
    # removing the pressures restores the plain step
    e = _t(np.zeros((1, 64)), torch.float64, gpu)
    p = _t(np.zeros((1, 64)), torch.float64, gpu)
    s.set_wavemaker([(0.01, 1.0, 0.8, 0.0)], x0=8.0, width=2.0)
    s.set_wavemaker([], x0=None)
    s.step(e, p, 0.1, 4)
    assert float(e.abs().max()) == 0.0


def test_tank_2d_with_anderson_mixed_solves(gpu):
    import torch
    nx, ny = 64, 32
    lx, ly = 16 * math.pi, 4 * math.pi
    gs = si.GridSpec(nx, ny, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 1.0, seed=7, hs_half=0.03)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.0 - 0.15 * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 2) ** 2) / 20.0)
    wm = dict(comps=[(0.01, 1.0, math.sqrt(math.tanh(1.0)), 0.0)], x0=0.75 * lx, width=2.0)
    s, o = _pair(gpu, nx, ny, lx, ly, depth, wm, mode="iter", accel="anderson")
    dt = 2 * math.pi / 32
    _say("tank 2D anderson")
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    st, info = s.step(e, p, dt, 4, tol=1e-12, t=0.5)
    eo, po, stats = o.step(eta, phi, dt, 4, tol=1e-12, t0=0.5)
    assert info["sweeps_total"] == sum(x.sweeps for x in stats)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
