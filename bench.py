#!/usr/bin/env python3
"""Throughput of the SBI hot path on one MI355X.

Workload: 2D crossing JONSWAP seas on a 1024^2 periodic grid (128 peak
wavelengths, dx = lambda_p/8) over random Gaussian-bump bathymetry, reference
depth k_p h drawn in [0.8, 3]; each step is one integrating-factor RK4 step
with four W solves iterated to a relative residual of 1e-8 in FP64.  Metric:
grid-point RK4 steps per second (points x steps / wall seconds), inputs
resident in HBM before the timed region.

`value` is the plain form (one realisation, linear-guess seed, eager launches;
HIP events bracket the sweep kernels of the last timed step only), whose W
iteration mixes its relaxed sweeps by Anderson's method (same residual test
and fixed point, about half the sweeps; `--accel none` and the
"plain-relaxed" form give the relaxed sweeps alone).  `forms` adds, at the same tolerance, two
realisations stepped in one captured HIP graph with the previous-solve seed
("batched+prev") and with the learned warm start ("batched+learned": the
network starts the first solve and the trained history layer predicts every
later stepping solve from the last eight, its inference inside the timed
region); both graphs enqueue a speculative sweep budget (the largest recent
sweep count + 3, redone exactly with a larger budget if a solve outruns it),
with the plain form's sweep cap; the
plain step in FP32 (tolerance 1e-6, the FP32 floor), the plain step in mixed
precision ("plain-mixed": FP32 sweeps on the correction equation between FP64
residual sweeps, at the headline's tolerance 1e-8, with its end state and
energy against the FP64 form's), the adaptive
fifth/fourth-order pair over four peak periods ("adaptive", at the error bound
3e-7 that makes it at least as accurate as the fixed step; counted in
fixed-step equivalents of T_p/64), the 1D submerged-bar tank driven by
the pneumatic wavemaker and damping pressure ("c2-tank", beside relaxation
zones), the ragged C4
ensemble (96 members, SA mode, FP32) in one graph, the 512^2 flat
crossing sea in FP32 beside FP64 with the FP32 error (max |eta|, energy drift),
and the fully nonlinear W (remaining integrals kept) stepping a steep 1D sea of
4096 points over a flat bed ("full-1d") and over two bars ("full-1d-bed").

Prints ONE JSON line.  `roofline` is for the dominant kernel of the plain
form, its algorithmic bytes per launch divided by its average launch time from
HIP events recorded on the library's stream during the timed region.
`cpu_baseline` times the FP64 oracle in the headline's mode (Anderson-mixed
iteration, tol 1e-8) on a bounded sample of the same workload, on one core and
on one member per usable core (at most 16).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point RK4 steps/s at 1024^2, plain vs batched+learned, W residual<=1e-8"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(kind: str, nx: int, ny: int, Kx: int, Ky: int, csz: int, rsz: int, vd: bool, J: int,
                      two_d: bool, aa: bool = False) -> float:
    """Minimum HBM bytes of one working launch of a sweep kernel (one member).

    half-form array: ny*Kx complex; compact array: Ky*Kx complex; physical: nx*ny real.
    aa: the Anderson-mixed iteration, whose row pass also reads T(V_(n-1)) and
    whose column pass writes T_V(x_n), f_n and g_n (compact) and the residual's
    half forms, not the next iterate.
    """
    half = ny * Kx * csz
    comp = Ky * Kx * csz
    phys = nx * ny * rsz
    ncomp = (2 if two_d else 1) if vd else 0
    nprod = J * (1 + ncomp)
    if kind == "row_sweep":
        # read G_V, G_D [, G_T] (+ grad phi_b components) and eta (+ delta); write the products
        return (2 + (1 if aa else 0) + ncomp) * half + (1 + (1 if vd else 0)) * phys + nprod * half
    if kind == "col_sweep":
        # read the products and b_V, V_n (+ b_phi, phi_b,n); write G_V, G_D (+ grad phi_b)
        # and T(V_n), V_(n+1) (+ phi_b,(n+1))
        nin_c = 2 + (2 if vd else 0)
        if aa:
            # write T_V(x_n), the residual f_n and relaxed sweep g_n (compact, V and phi_b parts) and the half
            # forms of f_n and T_V(x_n)
            return nprod * half + nin_c * comp + 2 * half + (1 + 2 * (1 + (1 if vd else 0))) * comp
        nout_c = 2 + (1 if vd else 0)
        return nprod * half + nin_c * comp + (2 + ncomp) * half + nout_c * comp
    raise ValueError(kind)


KERNEL_SOURCES = ["paper_2310_19840_amd/csrc/sbi_kernels.hip", "paper_2310_19840_amd/csrc/sbi_fft.hpp",
                  "paper_2310_19840_amd/csrc/sbi_internal.hpp", "paper_2310_19840_amd/csrc/sbi_kernels.hpp",
                  "paper_2310_19840_amd/csrc/sbi_device.hpp"]
TRAFFIC_RECORD = "profiles/sweep_kernels_traffic_c5_1024.txt"


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the recorded rocprofv3 FETCH_SIZE/WRITE_SIZE passes,
    scaled by the copy-kernel calibration; None when the kernel sources changed since."""
    import hashlib
    try:
        rec = {}
        for line in open(os.path.join(ROOT, TRAFFIC_RECORD)):
            if ": " in line and not line.startswith(" "):
                k, v = line.strip().split(": ", 1)
                rec[k] = v
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if rec.get("src_sha256") != h.hexdigest():
            return None
        return (float(rec[f"{kernel}_fetch_kib"]) * 1024 * float(rec["fetch_factor"]) +
                float(rec[f"{kernel}_write_kib"]) * 1024 * float(rec["write_factor"]))
    except (OSError, KeyError, ValueError):
        return None


def _oracle_member_rate(job):
    """Worker of cpu_baseline: consecutive RK4 steps of one sample member with
    the oracle (single-threaded numpy) until `min_seconds` of work (at most
    `max_steps`).  Returns (grid-point-steps, seconds, steps, sweeps)."""
    seed, n, min_seconds, max_steps, accel = job
    from oracle import Grid, Solver as OSolver
    from sbi_inputs import config_c5

    cfg = config_c5(seed=seed, n=n)
    g = cfg["grid"]
    o = OSolver(Grid(g.nx, g.ny, g.lx, g.ly), cfg["depth"], mode="iter", max_sweeps=400, accel=accel)
    eta, phi = cfg["eta"], cfg["phi"]
    sweeps, steps = 0, 0
    t0 = time.perf_counter()
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        eta, phi, stats = o.step(eta, phi, cfg["dt"], 1, tol=cfg["tol"])
        sweeps += sum(s.sweeps for s in stats)
        steps += 1
    return g.nx * g.ny * steps, time.perf_counter() - t0, steps, sweeps


def _host_cpu():
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, os.cpu_count() or 1, usable


def cpu_baseline(n_sample: int = 256, min_seconds: float = 10.0, max_steps: int = 8, accel: str = "anderson",
                 max_workers: int = 16):
    """The FP64 oracle in the headline's mode (W iteration to tol 1e-8 with
    Anderson-mixed sweeps) on a bounded sample of the workload: 256^2 members
    of the same recipe (same dx, depth draw and sea statistics; 1/16 of the
    1024^2 points), each stepped for about `min_seconds`.  First one member on
    one core alone, then one member per usable core (at most `max_workers`
    processes, numpy single-threaded in each) at once; `value` is the
    all-core figure."""
    import multiprocessing as mp

    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    model, ncpu, usable = _host_cpu()
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of the GPU process is inherited
    with ctx.Pool(1) as pool:
        pts1, el1, st1, sw1 = pool.map(_oracle_member_rate, [(0, n_sample, min_seconds, max_steps, accel)])[0]
    workers = max(1, min(usable, max_workers))
    jobs = [(sd, n_sample, min_seconds, max_steps, accel) for sd in range(workers)]
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_member_rate, jobs)
    wall = time.perf_counter() - t0
    pts = sum(r[0] for r in res)
    span = max(r[1] for r in res)
    steps = sum(r[2] for r in res)
    sweeps = sum(r[3] for r in res)
    return {
        "value": pts / span,
        "unit": "grid-point-steps/s",
        "cores": workers,
        "kind": "oracle",
        "value_1core": pts1 / el1,
        "host": f"{model}; {ncpu} logical CPUs, {usable} usable by this process",
        "sample": (f"{workers} members at {n_sample}x{n_sample} (the 1024^2 recipe at 1/16 of the points: same dx, "
                   f"depth draw and sea statistics, seeds 0..{workers - 1}), each stepped alone in its own "
                   f"single-threaded process for ~{min_seconds:.0f} s: {steps} RK4 steps, {4 * steps} W solves, "
                   f"{sweeps} sweeps ({sweeps / max(4 * steps, 1):.1f} per solve), W iteration tol 1e-8 with "
                   f"Anderson-mixed sweeps as in the headline; value = all members' grid-point-steps / the "
                   f"longest member's time ({span:.1f} s; {wall:.1f} s with process start-up). One core alone: "
                   f"{st1} steps of member 0 in {el1:.1f} s ({sw1} sweeps) -> value_1core"),
    }


def c5_members(seeds, n):
    from sbi_inputs import config_c5
    return [config_c5(seed=sd, n=n) for sd in seeds]


def dominant(prof, sweeps_total, solves, g, vd, csz, rsz, aa=False):
    """Dominant sweep kernel and its algorithmic bandwidth from the live profile."""
    Mx = int(math.ceil(0.5 * g.nx / 2 - 1e-9)) - 1
    My = int(math.ceil(0.5 * g.ny / 2 - 1e-9)) - 1
    Kx, Ky = Mx + 1, 2 * My + 1
    cand = {}
    for kind in ("row_sweep", "col_sweep"):
        tot_ms, cnt = prof.get(kind, (0.0, 0))
        if tot_ms <= 0:
            continue
        working = sweeps_total + (solves if kind == "row_sweep" else 0)
        b = algorithmic_bytes(kind, g.nx, g.ny, Kx, Ky, csz, rsz, vd, 6, g.ny > 1, aa)
        avg_s = tot_ms * 1e-3 / max(working, 1)
        cand[kind] = (tot_ms, b, avg_s, cnt, working)
    dom = max(cand, key=lambda k: cand[k][0])
    tot_ms, b, avg_s, cnt, working = cand[dom]
    achieved = b / avg_s / 1e9
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": dom, "bytes_per_launch": b,
                 "avg_launch_us": round(avg_s * 1e6, 2), "launches_working": working, "launches_total": cnt}


def run_plain(args, dev, precision, tol, accel=None, keep_state=False):
    """One C5 member, linear-guess seed, eager steps.  The sweep kernels of the
    last timed step are bracketed by HIP events (each bracket idles the device
    for a few microseconds, so the other steps run without them).  keep_state:
    also return the end state and its energy (Eq. (energy), FP64, after the
    timed region)."""
    import numpy as np
    import torch

    from paper_2310_19840_amd import Solver

    cfg = c5_members([0], args.n)[0]
    g = cfg["grid"]
    dtype = torch.float32 if precision == "fp32" else torch.float64
    s = Solver(g.nx, g.ny, g.lx, g.ly, cfg["depth"], device=dev, mode="iter", precision=precision,
               max_sweeps=args.max_sweeps, accel=accel)
    # launch plan from the autotuner (set-up, before the timed region)
    plan = s.autotune() if args.autotune else s.plan()
    eta = torch.tensor(cfg["eta"][None], dtype=dtype, device=dev)
    phi = torch.tensor(cfg["phi"][None], dtype=dtype, device=dev)
    dt = cfg["dt"]
    if args.warmup > 0:
        s.step(eta, phi, dt, args.warmup, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st0, info0 = 0, None
    if args.steps > 1:
        st0, info0 = s.step(eta, phi, dt, args.steps - 1, tol=tol)
    s.profile(True, sweeps_only=True)
    st1, info1 = s.step(eta, phi, dt, 1, tol=tol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    st = max(st0, st1) if min(st0, st1) >= 0 else min(st0, st1)
    info = dict(info1)
    if info0 is not None:
        for k in ("solves", "sweeps_total", "fallbacks", "sweeps_fp32_total"):
            info[k] = info0[k] + info1[k]
        info["sweeps_max"] = max(info0["sweeps_max"], info1["sweeps_max"])
        info["max_residual"] = max(info0["max_residual"], info1["max_residual"])
    solves = max(info["solves"], 1)
    vd = bool(np.any(cfg["depth"] != cfg["depth"].max()))
    csz, rsz = (8, 4) if precision == "fp32" else (16, 8)
    if precision == "mixed":
        # the FP32 correction sweeps: a W solve of K FP64 sweeps runs K - 1
        # correction solves, each with one working row launch per sweep plus
        # the one whose column pass decides it
        sw32 = info1["sweeps_fp32_total"]
        corr = info1["sweeps_total"] - sw32 - info1["solves"]
        dom, roof = dominant({"row_sweep": prof.get("row_sweep_fp32", (0.0, 0))}, sw32, max(corr, 1), g, vd, 8, 4,
                             accel == "anderson")
        dom = "row_sweep_fp32"
        roof["kernel"] = dom
    else:
        # the profiled step's own launches decide which of them did work
        dom, roof = dominant(prof, info1["sweeps_total"], max(info1["solves"], 1), g, vd, csz, rsz,
                             accel == "anderson")
    out = dict(value=g.nx * g.ny * args.steps / el, ms_per_step=1e3 * el / max(args.steps, 1), status=st,
               sweeps_mean=info["sweeps_total"] / solves, sweeps_max=info["sweeps_max"],
               max_residual=info["max_residual"], roofline=roof, dominant=dom,
               kernel_ms={k: round(v[0], 3) for k, v in prof.items() if v[1] > 0}, plan=plan, cfg=cfg)
    if precision == "mixed":
        out["sweeps_fp32_mean"] = info["sweeps_fp32_total"] / solves
    if keep_state:
        _, energy = s.diagnostics(eta, phi, tol=tol)
        out["end"] = (eta.double().cpu().numpy(), float(energy[0]))
    return out


def run_batched(args, dev, seed_mode, members, accel=None):
    """B C5 realisations in one captured graph, with the previous-solve seed
    ("prev") or the learned warm start ("net": the network starts the first
    solve, the trained history layer predicts every later stepping solve, so
    the layer's inference runs inside the timed region)."""
    import torch

    from paper_2310_19840_amd import Batch, warmstart

    cfgs = c5_members(range(members), args.n)
    blob = hist = None
    if seed_mode == "net":
        path = os.path.join(ROOT, "paper_2310_19840_amd", "weights", "warmstart_c5.sbiw")
        if not os.path.exists(path) or not os.path.exists(warmstart.HISTORY_WEIGHTS):
            return dict(skipped="no trained weights under paper_2310_19840_amd/weights")
        blob = open(path, "rb").read()
        hist = warmstart.load_history()
    mem = [dict(nx=c["grid"].nx, ny=c["grid"].ny, lx=c["grid"].lx, ly=c["grid"].ly, depth=c["depth"],
                precision="fp64", mode="iter", seed=seed_mode, max_sweeps=args.batch_sweeps, accel=accel)
           for c in cfgs]
    b = Batch(mem, device=dev, graph=True, autotune=args.autotune)
    if blob is not None:
        b.net_load(blob)
        b.hist_load(*hist)
    etas = [torch.tensor(c["eta"], dtype=torch.float64, device=dev) for c in cfgs]
    phis = [torch.tensor(c["phi"], dtype=torch.float64, device=dev) for c in cfgs]
    dt = cfgs[0]["dt"]
    tol = cfgs[0]["tol"]
    first = []
    # warm-up: the first call starts from no history (captured once); the
    # second captures the steady graph that the timed call replays
    _, i1 = b.step(etas, phis, dt, 1, tol=tol)
    first = [x["sweeps_total"] / max(x["solves"], 1) for x in i1]
    b.step(etas, phis, dt, args.steps, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = b.step(etas, phis, dt, args.steps, tol=tol)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    npts = sum(c["grid"].nx * c["grid"].ny for c in cfgs)
    solves = sum(x["solves"] for x in info)
    budgets, redos = b.budgets()
    return dict(value=npts * args.steps / el, ms_per_step=1e3 * el / max(args.steps, 1), status=st, members=members,
                sweeps_mean=sum(x["sweeps_total"] for x in info) / max(solves, 1),
                sweeps_max=max(x["sweeps_max"] for x in info),
                max_residual=max(x["max_residual"] for x in info),
                first_step_sweeps_mean=sum(first) / len(first), sweep_budget=budgets, redone_calls=redos,
                plans=b.plans())


def run_adaptive(args, dev, rk_tol):
    """One C5 member advanced by the adaptive fifth/fourth-order pair over
    `adaptive_periods` peak periods after one untimed period that lets the
    controller reach its working step; same W tolerance.  `value` counts
    fixed-step equivalents (grid points x simulated time / (T_p/64) per wall
    second), comparable with the plain form's."""
    import torch

    from paper_2310_19840_amd import Solver

    cfg = c5_members([0], args.n)[0]
    g = cfg["grid"]
    s = Solver(g.nx, g.ny, g.lx, g.ly, cfg["depth"], device=dev, mode="iter", max_sweeps=args.max_sweeps,
               accel=None if args.accel == "none" else args.accel)
    if args.autotune:
        s.autotune()
    eta = torch.tensor(cfg["eta"][None], dtype=torch.float64, device=dev)
    phi = torch.tensor(cfg["phi"][None], dtype=torch.float64, device=dev)
    dt, tol, Tp = cfg["dt"], cfg["tol"], cfg["period"]
    _, w = s.step_adaptive(eta, phi, Tp, dt, rk_tol, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_end = w["t"] + args.adaptive_periods * Tp
    st, info = s.step_adaptive(eta, phi, t_end, w["dt_next"], rk_tol, tol=tol, t=w["t"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fixed = args.adaptive_periods * Tp / dt
    att = info["accepted"] + info["rejected"]
    return dict(value=g.nx * g.ny * fixed / el, ms_per_fixed_step=1e3 * el / fixed, status=st, rk_tol=rk_tol,
                periods=args.adaptive_periods, accepted=info["accepted"], rejected=info["rejected"],
                mean_dt_over_Tp=round(args.adaptive_periods / max(info["accepted"], 1), 4),
                ms_per_attempt=round(1e3 * el / max(att, 1), 3), err_max=info["err_max"],
                sweeps_mean=round(info["sweeps_total"] / max(info["solves"], 1), 2), sweeps_max=info["sweeps_max"])


def run_c2_tank(args, dev):
    """The 1D submerged-bar tank (N=4096, 160 h0, short-wave case), SA mode, FP64,
    the paper's low-pass filter, eager steps of T/64: waves made by the
    pneumatic wavemaker and absorbed by
    the damping pressure (the tank of Sec. 3.2), beside the same tank driven by
    relaxation zones."""
    import numpy as np
    import torch

    from paper_2310_19840_amd import Solver
    from sbi_inputs import config_c2

    cfg = config_c2(case=2)
    g = cfg["grid"]
    rz = cfg["relax"]
    out = {}
    for kind in ("tank", "relaxation"):
        s = Solver(g.nx, 1, g.lx, 1.0, cfg["depth"], h_ref=cfg["h_ref"], device=dev, mode="sa",
                   filter_beta=cfg["filter_beta"])
        plan = s.autotune() if args.autotune else s.plan()
        if kind == "tank":
            s.set_wavemaker([(rz["a"], rz["k"], rz["omega"], 0.0)], x0=7 * g.lx / 8, width=4 * math.pi)
        else:
            s.set_relaxation(rz["a"], rz["k"], rz["omega"], rz["gen_len"], rz["abs_len"], rz["ramp_periods"])
        eta = torch.zeros((1, 1, g.nx), dtype=torch.float64, device=dev)
        phi = torch.zeros((1, 1, g.nx), dtype=torch.float64, device=dev)
        s.step(eta, phi, cfg["dt"], args.c2_steps // 4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = s.step(eta, phi, cfg["dt"], args.c2_steps, t=cfg["dt"] * (args.c2_steps // 4))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[kind] = dict(value=g.nx * args.c2_steps / el, ms_per_step=1e3 * el / args.c2_steps, status=st,
                         max_eta=float(np.abs(eta.cpu().numpy()).max()), plan=plan)
    r = dict(out["tank"])
    r.update(points=g.nx, steps=args.c2_steps, relaxation_value=out["relaxation"]["value"],
             relaxation_ms_per_step=out["relaxation"]["ms_per_step"])
    return r


def run_full_1d(args, dev, bed=False):
    """The fully nonlinear W (the remaining integrals of App. A kept) stepping a
    steep one-dimensional random sea: N = 4096 over a flat bed (k_p h = 1, 32
    points per peak wavelength, k_p a up to ~0.25), FP64, W tol 1e-10, eager
    steps of T_p/64 after one warm-up step; every pair pass evaluates the
    single-layer kernel at N^2 point pairs.  bed: over two Gaussian bars
    (depth down to 0.5, the bed's remainder I^(B) kept as well): a sweep then
    evaluates 4 N^2 pairs (bed and surface passes, each over surface and bed
    sources), the first of a solve N^2."""
    import numpy as np
    import torch

    import sbi_inputs as si
    from paper_2310_19840_amd import Solver

    n = 4096
    lx = 2 * math.pi * n / 32
    gs = si.GridSpec(n, 1, lx, 1.0)
    eta0 = si.narrowband_random(gs, 4096, amp=0.12)
    phi0 = si.narrowband_random(gs, 4097, amp=0.24)
    depth = np.ones((1, n))
    if bed:
        x = np.arange(n) * lx / n
        depth = (1.0 - 0.5 * (np.exp(-((x - 0.3 * lx) / (0.08 * lx)) ** 2)
                              + 0.5 * np.exp(-((x - 0.7 * lx) / (0.12 * lx)) ** 2)))[None]
    dt = 2 * math.pi / math.sqrt(math.tanh(1.0)) / 64
    s = Solver(n, 1, lx, 1.0, depth, device=dev, mode="full", max_sweeps=100)
    eta = torch.tensor(eta0[None], dtype=torch.float64, device=dev)
    phi = torch.tensor(phi0[None], dtype=torch.float64, device=dev)
    s.step(eta, phi, dt, 1, tol=1e-10)
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    st, info = s.step(eta, phi, dt, args.full_steps, tol=1e-10, t=dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    pairs_ms, _ = prof.get("full_pairs", (0.0, 0))
    apply_ms, apply_n = prof.get("full_apply", (0.0, 0))
    # a solve of s sweeps runs s - 1 working pair passes (the launch that
    # decides returns at once): each evaluates the kernel at n^2 point pairs
    working = info["sweeps_total"] - info["solves"]
    pairs = (4 * working + info["solves"]) * n * n if bed else working * n * n
    return dict(value=n * args.full_steps / el, ms_per_step=1e3 * el / args.full_steps, status=st, points=n,
                steps=args.full_steps, sweeps_mean=info["sweeps_total"] / max(info["solves"], 1),
                pair_pass_us=round(1e3 * pairs_ms / max(working, 1), 2),
                apply_ms_per_step=round(apply_ms / args.full_steps, 3),
                pairs_per_s=float(f"{pairs / max(1e-3 * pairs_ms, 1e-12):.4g}"),
                max_eta=float(np.abs(eta.cpu().numpy()).max()), bed="two bars, depth 0.5-1" if bed else "flat")


def run_c4(args, dev):
    """The ragged ensemble (32 x 128^2 + 48 x 256^2 + 16 x 512^2), SA mode, FP32: its 64-step window as one
    captured graph per call, launch shapes chosen by the autotuner at set-up."""
    import torch

    from paper_2310_19840_amd import Batch
    from sbi_inputs import config_c4_member

    cfgs = [config_c4_member(m) for m in range(96)]
    mem = [dict(nx=c["grid"].nx, ny=c["grid"].ny, lx=c["grid"].lx, ly=c["grid"].ly, depth=c["depth"],
                precision="fp32", mode="sa") for c in cfgs]
    b = Batch(mem, device=dev, graph=True, autotune=args.autotune)
    etas = [torch.tensor(c["eta"], dtype=torch.float32, device=dev) for c in cfgs]
    phis = [torch.tensor(c["phi"], dtype=torch.float32, device=dev) for c in cfgs]
    dt = cfgs[0]["dt"]
    b.step(etas, phis, dt, args.c4_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, _ = b.step(etas, phis, dt, args.c4_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    npts = sum(c["grid"].nx * c["grid"].ny for c in cfgs)
    return dict(value=npts * args.c4_steps / el, ms_per_step=1e3 * el / args.c4_steps, status=st, members=96,
                points=npts, steps=args.c4_steps, groups=b.groups(), plans=b.plans())


def run_c3_precision(args, dev):
    """The 512^2 flat crossing sea (SA mode) in FP32 and FP64 side by side over one
    peak period (64 steps): throughput, relative energy drift and mass change
    (FP64 diagnostics), and the error of each against the FP64 oracle's state
    after the same 64 steps, stored at 4096 seeded sample points by
    tests/golden/make_config_goldens.py (max |eta - eta_oracle| over the samples
    relative to the oracle's max |eta| over the field)."""
    import numpy as np
    import torch

    from paper_2310_19840_amd import Solver
    from sbi_inputs import config_c3

    cfg = config_c3(seed=3, n=512)
    g = cfg["grid"]
    gold = np.load(os.path.join(ROOT, "tests", "golden", "c3_sa_640.npz"))
    idx, ref, scale = gold["idx"], gold["s64_eta"], float(gold["s64_eta_absmax"])
    out = {}
    for prec, dt_ in (("fp64", torch.float64), ("fp32", torch.float32)):
        s = Solver(g.nx, g.ny, g.lx, g.ly, cfg["depth"], h_ref=cfg["h_ref"], device=dev, mode="sa", precision=prec)
        plan = s.autotune() if args.autotune else s.plan()
        eta = torch.tensor(cfg["eta"][None], dtype=dt_, device=dev)
        phi = torch.tensor(cfg["phi"][None], dtype=dt_, device=dev)
        m0, e0 = s.diagnostics(eta, phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(eta, phi, cfg["dt"], 64)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        m1, e1 = s.diagnostics(eta, phi)
        e = eta.double().cpu().numpy().ravel()[idx]
        out[prec] = dict(value=g.nx * g.ny * 64 / el, ms_per_step=1e3 * el / 64, plan=plan,
                         energy_drift=float(abs(e1[0] - e0[0]) / abs(e0[0])),
                         mass_change=float(abs(m1[0] - m0[0])),
                         max_eta_rel_error_vs_oracle=float(np.abs(e - ref).max() / scale))
    return dict(steps=64, grid=[g.ny, g.nx], mode="sa", fp32=out["fp32"], fp64=out["fp64"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024, help="grid size (1024 = the benchmark workload)")
    ap.add_argument("--max-sweeps", type=int, default=400)
    ap.add_argument("--batch-sweeps", type=int, default=None,
                    help="sweep cap (max_sweeps) of the captured forms; default: that of the plain form.  Their "
                         "launches follow the speculative budget (largest recent sweep count + 3), not the cap")
    ap.add_argument("--members", type=int, default=2, help="realisations of the batched forms")
    ap.add_argument("--c4-steps", type=int, default=64)
    ap.add_argument("--c2-steps", type=int, default=256)
    ap.add_argument("--full-steps", type=int, default=8)
    ap.add_argument("--forms",
                    default="plain,plain-relaxed,batched+prev,batched+learned,plain-fp32,plain-mixed,adaptive,"
                            "c2-tank,c4,c3-precision,full-1d,full-1d-bed")
    ap.add_argument("--accel", default="anderson", choices=["anderson", "none"],
                    help="iteration of the W solves: Anderson-mixed (default) or plain relaxed sweeps")
    ap.add_argument("--adaptive-periods", type=float, default=4.0)
    ap.add_argument("--rk-tol", type=float, default=3e-7,
                    help="error bound of the adaptive form; at 3e-7 its global error over two periods of a "
                         "128^2 sample of the sea (1.9e-7) is below that of fixed RK4 at T_p/64 (4.9e-7)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default launch plans instead of the autotuner's")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver is built and measured on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    accel = None if args.accel == "none" else args.accel
    if args.batch_sweeps is None:
        args.batch_sweeps = args.max_sweeps
    plain = run_plain(args, dev, "fp64", 1e-8, accel=accel, keep_state="plain-mixed" in forms)
    plain_end = plain.pop("end", None)
    cfg = plain.pop("cfg")
    g = cfg["grid"]
    tkey = plain["dominant"] + ("_aa" if accel == "anderson" else "")
    traffic = measured_traffic(tkey) if (g.nx, g.ny) == (1024, 1024) else None
    roofline = dict(plain["roofline"])
    roofline["traffic"] = round(traffic) if traffic is not None else None
    out_forms = {"plain": {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in plain.items()
                           if k in ("value", "ms_per_step", "sweeps_mean", "sweeps_max", "max_residual", "status",
                                    "plan")}}
    if "batched+prev" in forms:
        out_forms["batched+prev"] = run_batched(args, dev, "prev", args.members, accel)
    if "batched+learned" in forms:
        out_forms["batched+learned"] = run_batched(args, dev, "net", args.members, accel)
    if "plain-fp32" in forms:
        f32 = run_plain(args, dev, "fp32", 1e-6, accel=accel)
        f32.pop("cfg")
        out_forms["plain-fp32"] = {k: v for k, v in f32.items() if k in ("value", "ms_per_step", "sweeps_mean",
                                                                          "sweeps_max", "max_residual", "status",
                                                                          "roofline", "plan")}
        out_forms["plain-fp32"]["tol"] = 1e-6
    if "plain-mixed" in forms:
        mx = run_plain(args, dev, "mixed", 1e-8, accel=accel, keep_state=True)
        mx.pop("cfg")
        eta_m, en_m = mx.pop("end")
        eta_p, en_p = plain_end
        out_forms["plain-mixed"] = {k: v for k, v in mx.items() if k in ("value", "ms_per_step", "sweeps_mean",
                                                                          "sweeps_fp32_mean", "sweeps_max",
                                                                          "max_residual", "status", "roofline",
                                                                          "kernel_ms")}
        # against the FP64 form after the same steps (warm-up included)
        out_forms["plain-mixed"]["vs_fp64"] = {
            "max_eta_rel_diff": float(f"{float(np.abs(eta_m - eta_p).max() / np.abs(eta_p).max()):.3g}"),
            "energy_rel_diff": float(f"{abs(en_m - en_p) / abs(en_p):.3g}"),
            "steps": args.warmup + args.steps}
    if "plain-relaxed" in forms:
        rx = run_plain(args, dev, "fp64", 1e-8, accel=None)
        rx.pop("cfg")
        out_forms["plain-relaxed"] = {k: v for k, v in rx.items() if k in ("value", "ms_per_step", "sweeps_mean",
                                                                            "sweeps_max", "max_residual", "status",
                                                                            "roofline", "kernel_ms")}
    if "adaptive" in forms:
        out_forms["adaptive"] = run_adaptive(args, dev, args.rk_tol)
    if "c2-tank" in forms:
        out_forms["c2-tank"] = run_c2_tank(args, dev)
    if "c4" in forms:
        out_forms["c4"] = run_c4(args, dev)
    if "full-1d" in forms:
        out_forms["full-1d"] = run_full_1d(args, dev)
    if "full-1d-bed" in forms:
        out_forms["full-1d-bed"] = run_full_1d(args, dev, bed=True)
    if "c3-precision" in forms:
        out_forms["c3-precision"] = run_c3_precision(args, dev)
    for f, d in out_forms.items():
        if isinstance(d.get("value"), float) and f != "plain":
            d["vs_plain"] = round(d["value"] / plain["value"], 3)

    out = {
        "metric": METRIC,
        "value": round(plain["value"], 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(plain["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"crossing JONSWAP seas {g.nx}x{g.ny}, 128 lambda_p, Gaussian-bump bathymetry, "
                               f"k_p h_ref={cfg['h_ref']:.3f}, IF-RK4 dt=T_p/64, W iteration tol 1e-08 FP64 "
                               f"with {'Anderson-mixed' if accel else 'relaxed'} sweeps "
                               f"(plain: linear-guess seed, single member; other forms under 'forms')",
                   "grid": [g.ny, g.nx], "form": "plain", "iteration": accel or "relaxed"},
        "sweeps_per_solve_mean": round(plain["sweeps_mean"], 2),
        "sweeps_per_solve_max": plain["sweeps_max"],
        "max_residual": plain["max_residual"],
        "status": plain["status"],
        "roofline": roofline,
        "kernel_ms": plain["kernel_ms"],
        "forms": out_forms,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
