"""The fully nonlinear W solve (SBI_MODE_FULL: the boundary-integral
equations with the remaining integrals I^(S) kept, and I^(B) over a variable
bed; one dimension) on the GPU against the oracle (oracle/full_bie.py): W with
the same sweep count (FP64 within 1e-11, FP32 within 1e-5 of the oracle fed
FP32-rounded inputs), exact Stokes waves, time steps, and what the mode
refuses."""
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


def _sea(nx, seed, amp):
    lx = 2 * math.pi * nx / 32          # 32 points per wavelength of the peak (k = 1)
    gs = si.GridSpec(nx, 1, lx, 1.0)
    eta = si.narrowband_random(gs, seed, amp=amp)
    phi = si.narrowband_random(gs, seed + 1, amp=2 * amp)
    return lx, eta, phi


@pytest.mark.parametrize("nx", [64, 256, 1024, 4096])
@pytest.mark.parametrize("depth", [1.0, 50.0])
def test_full_w_matches_oracle(gpu, nx, depth):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    lx, eta, phi = _sea(nx, nx + 3, 0.12)
    _say("full W", nx, "depth", depth)
    g = Grid(nx, 1, lx)
    dep = np.full((1, nx), depth)
    o = OSolver(g, dep, mode="full", max_sweeps=100)
    Wo, oi = o.vertical_velocity(eta, phi, tol=1e-12)
    s = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=100)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
    err = _rel(W.cpu().numpy()[0], Wo)
    _say(f"   W err {err:.2e}, sweeps {info[0][0]}/{oi.sweeps}")
    assert st == 0 and info[0][0] == oi.sweeps
    assert err < 1e-11
    # FP32 against the oracle on the same FP32-rounded inputs
    e32, p32 = eta.astype(np.float32), phi.astype(np.float32)
    Wo32, _ = OSolver(g, dep, mode="full", max_sweeps=100).vertical_velocity(
        e32.astype(np.float64), p32.astype(np.float64), tol=1e-12)
    s32 = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=100, precision="fp32")
    W32, st32, _ = s32.vertical_velocity(_t(e32, torch.float32, gpu), _t(p32, torch.float32, gpu), tol=1e-6)
    err32 = _rel(W32.cpu().numpy()[0].astype(np.float64), Wo32)
    _say(f"   FP32 W err {err32:.2e}")
    assert st32 >= 0 and err32 < 1e-5


@pytest.mark.parametrize("eps,bar", [(0.3, 1e-10), (0.35, 5e-9)])
def test_full_w_of_exact_stokes_waves(gpu, eps, bar):
    """Deep-water Stokes waves from the stream-function method: the GPU's
    fully nonlinear W equals the exact one on the kept band (all modes but
    Nyquist), where the expansion of order 7 is off by 1e-5 (eps = 0.3) and
    7e-4 (eps = 0.35)."""
    import torch
    from oracle import Grid
    from oracle.fenton import SteadyWave
    from paper_2310_19840_amd import Solver
    w = SteadyWave(2 * eps)
    x = np.arange(64) * 2 * math.pi / 64
    eta, _, phi, V = w.surface(x)
    g = Grid(64, 1, 2 * math.pi, dealias=0.99)
    Vm = g.ifft(g.MF(V[None]))[0]
    s = Solver(64, 1, 2 * math.pi, 1.0, np.full((1, 64), 60.0), device=gpu, mode="full", max_sweeps=100,
               dealias=0.99)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-13)
    err = _rel(W.cpu().numpy()[0], Vm)
    sa = Solver(64, 1, 2 * math.pi, 1.0, np.full((1, 64), 60.0), device=gpu, mode="sa")
    W7, _, _ = sa.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu))
    err7 = _rel(W7.cpu().numpy()[0], V)
    _say(f"eps {eps}: full {err:.2e} ({info[0][0]} sweeps), order 7 {err7:.2e}")
    assert st == 0 and err < bar and err7 > 1e3 * err


@pytest.mark.parametrize("depth", [1.0, 50.0])
def test_full_steps_match_oracle(gpu, depth):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 256
    lx, eta, phi = _sea(nx, 17, 0.1)
    dep = np.full((1, nx), depth)
    om = math.sqrt(math.tanh(depth))
    dt = 2 * math.pi / om / 32
    o = OSolver(Grid(nx, 1, lx), dep, mode="full", max_sweeps=100)
    eo, po, sto = o.step(eta, phi, dt, 4, tol=1e-12)
    s = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=100)
    e = _t(eta[None], torch.float64, gpu)
    p = _t(phi[None], torch.float64, gpu)
    st, info = s.step(e, p, dt, 4, tol=1e-12)
    _say(f"full steps depth {depth}: sweeps {info['sweeps_total']}/{sum(i.sweeps for i in sto)}")
    assert st == 0 and info["solves"] == 16
    assert info["sweeps_total"] == sum(i.sweeps for i in sto)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def _bar(nx, lx, amp):
    x = np.arange(nx) * lx / nx
    # a smooth bar and a gentler second one (depth 1 away from them)
    return 1.0 - amp * (np.exp(-((x - 0.3 * lx) / (0.08 * lx)) ** 2) + 0.5 * np.exp(-((x - 0.7 * lx) / (0.12 * lx)) ** 2))


@pytest.mark.parametrize("nx", [64, 256, 1024])
def test_full_w_over_a_variable_bed_matches_oracle(gpu, nx):
    """The two-boundary solve (I^(B) kept) against the oracle's: the same
    sweeps and W within 1e-11 in FP64; FP32 within 1e-5 of the oracle fed the
    FP32-rounded inputs."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    lx, eta, phi = _sea(nx, nx + 9, 0.1)
    dep = _bar(nx, lx, 0.5)[None]
    g = Grid(nx, 1, lx)
    Wo, oi = OSolver(g, dep, mode="full", max_sweeps=200).vertical_velocity(eta, phi, tol=1e-12)
    s = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=200)
    W, st, info = s.vertical_velocity(_t(eta, torch.float64, gpu), _t(phi, torch.float64, gpu), tol=1e-12)
    err = _rel(W.cpu().numpy()[0], Wo)
    _say(f"bed W {nx}: err {err:.2e}, sweeps {info[0][0]}/{oi.sweeps}")
    assert st == 0 and info[0][0] == oi.sweeps and err < 1e-11
    e32, p32 = eta.astype(np.float32), phi.astype(np.float32)
    Wo32, _ = OSolver(g, dep, mode="full", max_sweeps=200).vertical_velocity(
        e32.astype(np.float64), p32.astype(np.float64), tol=1e-12)
    s32 = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=200, precision="fp32")
    W32, st32, _ = s32.vertical_velocity(_t(e32, torch.float32, gpu), _t(p32, torch.float32, gpu), tol=1e-6)
    err32 = _rel(W32.cpu().numpy()[0].astype(np.float64), Wo32)
    _say(f"   FP32 err {err32:.2e}")
    assert st32 >= 0 and err32 < 1e-5


def test_full_members_with_flat_variable_and_deep_beds(gpu):
    """One context: a flat bed (image form), a variable bed (two-boundary
    form) and a variable bed too deep to matter (image form without image),
    each equal to its own oracle solve with its sweep count."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 256
    lx, e0, p0 = _sea(nx, 61, 0.1)
    _, e1, p1 = _sea(nx, 71, 0.1)
    _, e2, p2 = _sea(nx, 81, 0.08)
    dep = np.stack([np.full((1, nx), 1.0), _bar(nx, lx, 0.4)[None], 500.0 * _bar(nx, lx, 0.2)[None]])
    s = Solver(nx, 1, lx, 1.0, dep, batch=3, device=gpu, mode="full", max_sweeps=200)
    E = np.stack([e0, e1, e2])
    P = np.stack([p0, p1, p2])
    W, st, info = s.vertical_velocity(_t(E, torch.float64, gpu), _t(P, torch.float64, gpu), tol=1e-12)
    assert st == 0
    for k in range(3):
        Wo, oi = OSolver(Grid(nx, 1, lx), dep[k], mode="full", max_sweeps=200).vertical_velocity(E[k], P[k], tol=1e-12)
        err = _rel(W.cpu().numpy()[k], Wo)
        _say(f"member {k}: err {err:.2e}, sweeps {info[k][0]}/{oi.sweeps}")
        assert info[k][0] == oi.sweeps and err < 1e-11


def test_full_steps_over_a_bar_match_oracle(gpu):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 256
    lx, eta, phi = _sea(nx, 23, 0.08)
    dep = _bar(nx, lx, 0.5)[None]
    dt = 2 * math.pi / math.sqrt(math.tanh(1.0)) / 32
    o = OSolver(Grid(nx, 1, lx), dep, mode="full", max_sweeps=200)
    eo, po, sto = o.step(eta, phi, dt, 3, tol=1e-12)
    s = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=200)
    e = _t(eta[None], torch.float64, gpu)
    p = _t(phi[None], torch.float64, gpu)
    st, info = s.step(e, p, dt, 3, tol=1e-12)
    _say(f"bed steps: sweeps {info['sweeps_total']}/{sum(i.sweeps for i in sto)}")
    assert st == 0 and info["sweeps_total"] == sum(i.sweeps for i in sto)
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def test_full_c1_over_one_period_matches_oracle(gpu):
    """The Gaussian-bump configuration (N = 256, bump 0.3 h0, Stokes wave
    k0 a = 0.05) stepped one wave period (64 RK4 steps) with the fully
    nonlinear W over its variable bed: the oracle's sweeps and end state."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    cfg = si.config_c1()
    g = cfg["grid"]
    dep = cfg["depth"].reshape(1, g.nx)
    o = OSolver(Grid(g.nx, 1, g.lx), dep, h_ref=cfg["h_ref"], mode="full", max_sweeps=200)
    eo, po, sto = o.step(cfg["eta"].reshape(1, -1), cfg["phi"].reshape(1, -1), cfg["dt"], 64, tol=1e-11)
    s = Solver(g.nx, 1, g.lx, 1.0, dep, h_ref=cfg["h_ref"], device=gpu, mode="full", max_sweeps=200)
    e = _t(cfg["eta"].reshape(1, 1, -1), torch.float64, gpu)
    p = _t(cfg["phi"].reshape(1, 1, -1), torch.float64, gpu)
    st, info = s.step(e, p, cfg["dt"], 64, tol=1e-11)
    err = _rel(e.cpu().numpy().reshape(eo.shape), eo)
    _say(f"C1 full, one period: sweeps {info['sweeps_total']}/{sum(i.sweeps for i in sto)}, eta err {err:.2e}")
    assert st == 0 and info["sweeps_total"] == sum(i.sweeps for i in sto)
    assert err < 1e-10 and _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10


def test_full_mode_refusals(gpu):
    from paper_2310_19840_amd import Batch, SBIError, Solver, _lib
    # two-dimensional grids: not a valid grid for the mode
    with pytest.raises(SBIError):
        Solver(32, 32, 10.0, 10.0, np.ones((32, 32)), device=gpu, mode="full")
    # ensembles
    with pytest.raises(SBIError) as ex:
        Batch([dict(nx=64, ny=1, lx=10.0, ly=1.0, depth=np.ones((1, 64)), mode="full")], device=gpu)
    assert ex.value.code == _lib.SBI_ERR_UNSUPPORTED


def test_full_two_members_with_their_own_depths(gpu):
    """One context of two members, one over a finite flat bed and one in deep
    water: each member's W equals its own oracle solve."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 512
    lx, e0, p0 = _sea(nx, 31, 0.12)
    _, e1, p1 = _sea(nx, 41, 0.08)
    dep = np.stack([np.full((1, nx), 1.0), np.full((1, nx), 1000.0)])
    s = Solver(nx, 1, lx, 1.0, dep, batch=2, device=gpu, mode="full", max_sweeps=100)
    W, st, info = s.vertical_velocity(_t(np.stack([e0, e1]), torch.float64, gpu), _t(np.stack([p0, p1]), torch.float64, gpu),
                                      tol=1e-12)
    assert st == 0
    for k, (e, p) in enumerate(((e0, p0), (e1, p1))):
        o = OSolver(Grid(nx, 1, lx), dep[k], mode="full", max_sweeps=100)
        Wo, oi = o.vertical_velocity(e, p, tol=1e-12)
        err = _rel(W.cpu().numpy()[k], Wo)
        _say(f"member {k}: W err {err:.2e}, sweeps {info[k][0]}/{oi.sweeps}")
        assert info[k][0] == oi.sweeps and err < 1e-11


def test_full_adaptive_pair_matches_oracle(gpu):
    """The adaptive fifth/fourth-order pair with the fully nonlinear W: the same
    accepted and rejected steps as the oracle and the end state within 1e-10."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    nx = 128
    lx, eta, phi = _sea(nx, 53, 0.1)
    dep = np.full((1, nx), 1.0)
    T = 2 * math.pi / math.sqrt(math.tanh(1.0))
    o = OSolver(Grid(nx, 1, lx), dep, mode="full", max_sweeps=100)
    eo, po, oinfo = o.step_adaptive(eta, phi, 0.0, T, T / 16, 1e-6, tol=1e-12)
    s = Solver(nx, 1, lx, 1.0, dep, device=gpu, mode="full", max_sweeps=100)
    e = _t(eta[None], torch.float64, gpu)
    p = _t(phi[None], torch.float64, gpu)
    st, info = s.step_adaptive(e, p, T, T / 16, 1e-6, tol=1e-12)
    _say(f"adaptive full: accepted {info['accepted']}/{oinfo['accepted']}, rejected {info['rejected']}/{oinfo['rejected']}")
    assert st >= 0
    assert (info["accepted"], info["rejected"]) == (oinfo["accepted"], oinfo["rejected"])
    assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
    assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10
