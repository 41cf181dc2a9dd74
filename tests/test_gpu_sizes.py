"""Every transform size the kernels are instantiated for, against the FP64
oracle: row passes for nx = 16 .. 8192 (1D grids) and column passes for
ny = 16 .. 2048 (2D grids, with the quarter-band variant where it applies),
each with a variable bed, in SA mode, in the Anderson-mixed iteration (same
sweep count) and over one time step with the wave tank's pressures (1D) or
with the relaxation zone (1D, second step).  FP64 within 1e-10 (W: 1e-11),
FP32 within 1e-5.
"""
import math
import sys

import numpy as np
import pytest

import sbi_inputs as si

pytestmark = pytest.mark.gpu

NX_ALL = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]
NY_ALL = [16, 32, 64, 128, 256, 512, 1024, 2048]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(x, dtype, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case(nx, ny):
    # a random sea around k = 1 (16 points per wavelength, nx/16 wavelengths)
    lx = 2 * math.pi * max(nx, 16) / 16
    ly = 2 * math.pi * max(ny, 16) / 16 if ny > 1 else 1.0
    gs = si.GridSpec(nx, ny, lx, ly)
    eta = si.narrowband_random(gs, nx + 7 * ny, amp=0.06)
    phi = si.narrowband_random(gs, nx + 7 * ny + 1, amp=0.3)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.5 - 0.3 * np.exp(-((X - lx / 3) ** 2 / (0.02 * lx * lx) + ((Y - ly / 2) ** 2 / (0.02 * ly * ly)
                                                                        if ny > 1 else 0.0)))
    return lx, ly, eta, phi, depth


def _check_w(gpu, nx, ny):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    lx, ly, eta, phi, depth = _case(nx, ny)
    g = Grid(nx, ny, lx, ly)
    for mode, accel in (("sa", None), ("iter", "anderson")):
        o = OSolver(g, depth, mode=mode, max_sweeps=200, accel=accel)
        Wo, oi = o.vertical_velocity(eta, phi, tol=1e-12)
        s = Solver(nx, ny, lx, ly, depth, device=gpu, mode=mode, max_sweeps=200, accel=accel)
        W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
        err = _rel(W.cpu().numpy()[0], Wo)
        _say(f"   {mode:4s} W err {err:.2e}" + (f" sweeps {info[0][0]}/{oi.sweeps}" if mode == "iter" else ""))
        assert err < 1e-11
        if mode == "iter":
            assert info[0][0] == oi.sweeps
        # FP32: against the oracle on the same FP32-rounded inputs
        e32 = eta.astype(np.float32)
        p32 = phi.astype(np.float32)
        Wo32, _ = OSolver(g, depth, mode=mode, max_sweeps=200, accel=accel).vertical_velocity(
            e32.astype(np.float64), p32.astype(np.float64), tol=1e-12)
        s32 = Solver(nx, ny, lx, ly, depth, device=gpu, mode=mode, max_sweeps=200, accel=accel, precision="fp32")
        W32, _, _ = s32.vertical_velocity(_t(e32, torch.float32, gpu), _t(p32, torch.float32, gpu), tol=1e-6)
        err32 = _rel(W32.cpu().numpy()[0].astype(np.float64), Wo32)
        _say(f"   {mode:4s} FP32 W err {err32:.2e}")
        assert err32 < 1e-5


@pytest.mark.parametrize("nx", NX_ALL)
def test_row_sizes_1d(gpu, nx):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    _say("1D nx", nx)
    _check_w(gpu, nx, 1)
    # one SA step inside the wave tank (pneumatic wavemaker + damping), then
    # one with the relaxation zone
    lx, _, eta, phi, depth = _case(nx, 1)
    g = Grid(nx, 1, lx)
    h = 1.5
    om = math.sqrt(math.tanh(h))
    dt = 2 * math.pi / om / 32
    wm = dict(comps=[(0.01, 1.0, om, 0.2)], x0=7 * lx / 8, width=lx / 16)
    o = OSolver(g, depth, mode="sa", wavemaker=wm)
    eo, po, _ = o.step(eta, phi, dt, 1, t0=0.3)
    s = Solver(nx, 1, lx, 1.0, depth, device=gpu, mode="sa")
    s.set_wavemaker(wm["comps"], x0=wm["x0"], width=wm["width"])
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    s.step(e, p, dt, 1, t=0.3)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10
    lam = 2 * math.pi
    rz = dict(a=0.01, k=1.0, omega=om, gen_len=min(2 * lam, lx / 4), abs_len=min(3 * lam, lx / 4),
              ramp_periods=1.0)
    o2 = OSolver(g, depth, mode="sa", relaxation_zone=rz)
    eo2, po2, _ = o2.step(eta, phi, dt, 1, t0=0.7)
    s2 = Solver(nx, 1, lx, 1.0, depth, device=gpu, mode="sa")
    s2.set_relaxation(rz["a"], rz["k"], rz["omega"], rz["gen_len"], rz["abs_len"], rz["ramp_periods"])
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    s2.step(e, p, dt, 1, t=0.7)
    assert _rel(e.cpu().numpy().reshape(eo2.shape), eo2) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po2.shape), po2) < 1e-10


@pytest.mark.parametrize("ny", NY_ALL)
def test_column_sizes_2d(gpu, ny):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 32
    _say("2D ny", ny)
    _check_w(gpu, nx, ny)
    lx, ly, eta, phi, depth = _case(nx, ny)
    dt = 2 * math.pi / math.sqrt(math.tanh(1.5)) / 32
    o = OSolver(Grid(nx, ny, lx, ly), depth, mode="iter", accel="anderson", max_sweeps=200)
    eo, po, st = o.step(eta, phi, dt, 1, tol=1e-11)
    s = Solver(nx, ny, lx, ly, depth, device=gpu, mode="iter", accel="anderson", max_sweeps=200)
    e = _t(eta, torch.float64, gpu)
    p = _t(phi, torch.float64, gpu)
    _, info = s.step(e, p, dt, 1, tol=1e-11)
    assert info["sweeps_total"] == sum(x.sweeps for x in st)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10
