"""Parity of the HIP path (through the C interface) with the FP64 oracle at
each benchmark configuration's own size and window.

The oracle's end states come from tests/golden/make_config_goldens.py, which
runs only the oracle on the seeded inputs of sbi_inputs/: the whole state for
the 1D configurations, 4096 seeded sample points plus whole-field sums for
the 2D ones.  Bars: eta and phi within 1e-10 of the oracle's max |eta| (|phi|)
in FP64 and 1e-5 in FP32, after the stated steps; the iteration takes the
oracle's sweep counts.

Windows: C1 all 640 steps (10 periods); C2 all 20,000 steps of both incident
waves with the paper's low-pass filter, and 4000 steps without it (the
unfiltered tank amplifies round-off at the dealiasing edge: a 1e-13
perturbation grows past 1e-10 within ~3500 steps); C3 the first and the first ten of its 100 peak periods (the oracle
needs ~3 s per 512^2 step); C4 the 64-step window of a 128^2, a 256^2 and a
512^2 member, alone and together in one captured ragged ensemble; C5 two steps
at 1024^2 in SA mode and with the benchmark's iteration (Anderson-mixed
sweeps, tol 1e-8).
"""
import math
import os
import sys

import numpy as np
import pytest

import sbi_inputs as si

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gold(name):
    p = os.path.join(GOLD, name + ".npz")
    assert os.path.exists(p), f"missing golden {p}: run tests/golden/make_config_goldens.py"
    return np.load(p)


def _t(x, dtype, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _check_full(e, p, G, tol, prefix=""):
    ee, pp = G[prefix + "eta"], G[prefix + "phi"]
    ee = ee.reshape(e.shape)
    pp = pp.reshape(p.shape)
    de = np.abs(e - ee).max() / np.abs(ee).max()
    dp = np.abs(p - pp).max() / np.abs(pp).max()
    _say(f"   max|d eta|/max|eta| {de:.2e}  max|d phi|/max|phi| {dp:.2e}")
    assert de < tol and dp < tol, (de, dp)


def _check_sampled(e, p, G, tol, prefix=""):
    idx = G["idx"]
    ef = e.ravel()
    pf = p.ravel()
    de = np.abs(ef[idx] - G[prefix + "eta"]).max() / G[prefix + "eta_absmax"]
    dp = np.abs(pf[idx] - G[prefix + "phi"]).max() / G[prefix + "phi_absmax"]
    # whole-field properties: extrema, mean and mean square of eta
    n = ef.size
    dm = abs(np.abs(ef).max() - G[prefix + "eta_absmax"]) / G[prefix + "eta_absmax"]
    ds = abs(ef.sum() - G[prefix + "eta_sum"]) / (n * G[prefix + "eta_absmax"])
    dq = abs((ef * ef).sum() - G[prefix + "eta_sumsq"]) / G[prefix + "eta_sumsq"]
    _say(f"   sampled max|d eta| {de:.2e} |d phi| {dp:.2e}; max|eta| {dm:.2e} sum {ds:.2e} sumsq {dq:.2e}")
    assert de < tol and dp < tol, (de, dp)
    assert dm < tol and ds < tol and dq < 2 * tol, (dm, ds, dq)


def _run(gpu, cfg, steps, precision="fp64", chunks=None, **opts):
    import torch
    from paper_2310_19840_amd import Solver
    g = cfg["grid"]
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = Solver(g.nx, g.ny, g.lx, g.ly if g.ny > 1 else 1.0, cfg["depth"], h_ref=cfg["h_ref"], device=gpu,
               precision=precision, **opts)  # opts may carry filter_beta
    if "relax" in cfg and cfg["relax"] is not None and g.ny == 1 and opts.get("mode") == "sa":
        rz = cfg["relax"]
        s.set_relaxation(rz["a"], rz["k"], rz["omega"], rz["gen_len"], rz["abs_len"], rz["ramp_periods"])
    e = _t(cfg["eta"], dt, gpu)
    p = _t(cfg["phi"], dt, gpu)
    tol = cfg["tol"] if opts.get("mode") == "iter" else 0.0
    infos = []
    t = 0.0
    for n in (chunks or [steps]):
        st, info = s.step(e, p, cfg["dt"], n, tol=tol, t=t)
        t = info["t"]
        infos.append(info)
    return s, e, p, infos


# ---------------------------------------------------------------------------
def test_c1_all_640_steps(gpu):
    """C1: 1D N=256 over a Gaussian bump, Stokes wave, iteration tol 1e-10,
    FP64, 10 periods (640 steps): the whole state and the sweep totals."""
    G = _gold("c1_iter_640")
    cfg = si.config_c1()
    _say("C1 640 steps")
    s, e, p, infos = _run(gpu, cfg, 640, mode="iter", max_sweeps=200)
    info = infos[0]
    assert info["solves"] == 4 * 640
    assert info["sweeps_total"] == int(G["sweeps"].sum()), (info["sweeps_total"], int(G["sweeps"].sum()))
    assert info["sweeps_max"] == int(G["sweeps"].max())
    _check_full(e.cpu().numpy(), p.cpu().numpy(), G, 1e-10)


@pytest.mark.parametrize("case", [1, 2])
def test_c2_all_20000_steps(gpu, case):
    """C2: 1D N=4096 submerged trapezoidal bar, regular waves ramped in by the
    relaxation zone, SA mode, FP64, the paper's low-pass filter, all 20,000
    steps."""
    G = _gold(f"c2_case{case}_20000")
    cfg = si.config_c2(case=case)
    _say("C2 case", case, "20000 steps")
    s, e, p, _ = _run(gpu, cfg, 20000, mode="sa", chunks=[5000] * 4, filter_beta=cfg["filter_beta"])
    e, p = e.cpu().numpy(), p.cpu().numpy()
    assert np.abs(G["eta"]).max() > 0.5 * cfg["relax"]["a"]  # the wave has crossed the tank
    _check_full(e, p, G, 1e-10)


@pytest.mark.parametrize("case", [1, 2])
def test_c2_unfiltered_4000_steps(gpu, case):
    """C2 without the filter, over the 4000 steps in which its amplification
    of round-off at the dealiasing edge stays far below the bar."""
    G = _gold(f"c2_case{case}_nofilter_4000")
    cfg = si.config_c2(case=case)
    _say("C2 case", case, "unfiltered, 4000 steps")
    s, e, p, _ = _run(gpu, cfg, 4000, mode="sa", chunks=[2000] * 2)
    _check_full(e.cpu().numpy(), p.cpu().numpy(), G, 1e-10)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_c3_crossing_sea_512(gpu, precision, tol):
    """C3: 512^2 crossing JONSWAP seas over a flat bed, SA mode: one peak
    period (64 steps) and ten (640) in FP64 and FP32."""
    G = _gold("c3_sa_640")
    cfg = si.config_c3()
    _say("C3", precision)
    s, e, p, _ = _run(gpu, cfg, 640, precision=precision, mode="sa", chunks=[64])
    _check_sampled(e.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64), G, tol, "s64_")
    st, _ = s.step(e, p, cfg["dt"], 576, tol=0.0, t=64 * cfg["dt"])
    _check_sampled(e.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64), G, tol)


C4_MEMBERS = [5, 40, 90]  # 128^2, 256^2, 512^2


@pytest.mark.parametrize("member", C4_MEMBERS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_c4_member_64_steps(gpu, member, precision, tol):
    """C4: ensemble members with their own undulating bars (4-12 bars,
    0.1-0.25 h0), SA mode, the 64-step window."""
    G = _gold(f"c4_m{member}_sa_64")
    cfg = si.config_c4_member(member)
    _say("C4 member", member, cfg["grid"].nx, precision)
    s, e, p, _ = _run(gpu, cfg, 64, precision=precision, mode="sa")
    _check_sampled(e.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64), G, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_c4_ragged_graph_64_steps(gpu, precision, tol):
    """The same three members stepped together in one captured ragged
    ensemble (the C4 form), 64 steps."""
    import torch
    from paper_2310_19840_amd import Batch
    dt_ = torch.float64 if precision == "fp64" else torch.float32
    cfgs = [si.config_c4_member(m) for m in C4_MEMBERS]
    mems = []
    for c in cfgs:
        g = c["grid"]
        mems.append(dict(nx=g.nx, ny=g.ny, lx=g.lx, ly=g.ly, depth=c["depth"], precision=precision, mode="sa"))
    _say("C4 ragged graph", precision)
    b = Batch(mems, h_ref=3.0, device=gpu, graph=True)
    es = [_t(c["eta"], dt_, gpu) for c in cfgs]
    ps = [_t(c["phi"], dt_, gpu) for c in cfgs]
    b.step(es, ps, cfgs[0]["dt"], 64, tol=0.0)
    for m, e, p in zip(C4_MEMBERS, es, ps):
        _check_sampled(e.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64),
                       _gold(f"c4_m{m}_sa_64"), tol)


def test_c5_sa_two_steps_1024(gpu):
    """C5 at 1024^2 over random Gaussian bumps, SA mode (the paper's method),
    two steps: the 1024-row state pass, the nonlinear term and the stage
    updates elementwise at 4096 points and in whole-field sums."""
    G = _gold("c5_sa_2")
    cfg = si.config_c5()
    _say("C5 SA 2 steps")
    s, e, p, _ = _run(gpu, cfg, 2, mode="sa")
    _check_sampled(e.cpu().numpy(), p.cpu().numpy(), G, 1e-10)


def test_c5_benchmark_iteration_two_steps_1024(gpu):
    """C5 as the benchmark runs it: 1024^2, W iteration to tol 1e-8 with
    Anderson-mixed sweeps, FP64, two steps: the same sweep count in every
    solve and the state within 1e-10."""
    G = _gold("c5_iter_aa_2")
    cfg = si.config_c5()
    _say("C5 iteration 2 steps")
    s, e, p, infos = _run(gpu, cfg, 2, mode="iter", max_sweeps=400, accel="anderson")
    sw = G["sweeps"]
    assert infos[0]["solves"] == len(sw) == 8
    assert infos[0]["sweeps_total"] == int(sw.sum()), (infos[0], sw)
    assert infos[0]["sweeps_max"] == int(sw.max())
    _check_sampled(e.cpu().numpy(), p.cpu().numpy(), G, 1e-10)
