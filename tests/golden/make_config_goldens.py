"""Write the oracle's end states of the benchmark configurations at their own
sizes and windows, for the GPU parity tests (tests/test_gpu_configs.py).

Test infrastructure: calls only the FP64 oracle (oracle/) and the seeded input
generators (sbi_inputs/); nothing here runs or reads the HIP library.

Usage:  python tests/golden/make_config_goldens.py [name ...] [--jobs N]

Each golden is an .npz next to this script:
  1D configurations (C1, C2): the whole end state (eta, phi) in FP64;
  2D configurations (C3, C4 members, C5): the end state at 4096 seeded sample
    points (flat indices `idx`), its max |eta|, max |phi|, sum eta and sum eta^2
    over the whole field;
  iteration runs also hold the sweep count of every W solve (`sweeps`).
Running it again reproduces the files bit for bit (no randomness beyond the
seeded generators).
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NSAMPLE = 4096

# name -> (config, window, solver options); windows are the configurations'
# own step counts where the oracle can run them (C1: 640 steps = 10 periods,
# C2: 20,000 steps, C4: its 64-step window), else stated here (C3: 10 of its
# 100 peak periods, with the first period also stored; C5: 2 of its 32 steps).
# C2 runs with the low-pass filter of its configuration; without it the
# 4096-point tank amplifies round-off at the dealiasing edge (a 1e-13
# perturbation grows past 1e-10 within ~3500 steps), so the unfiltered run is
# compared over 4000 steps only.
GOLDENS = {
    "c1_iter_640": dict(cfg="c1", steps=640, opts=dict(mode="iter", max_sweeps=200)),
    "c2_case1_20000": dict(cfg="c2", case=1, steps=20000, opts=dict(mode="sa"), filter=True),
    "c2_case2_20000": dict(cfg="c2", case=2, steps=20000, opts=dict(mode="sa"), filter=True),
    "c2_case1_nofilter_4000": dict(cfg="c2", case=1, steps=4000, opts=dict(mode="sa"), filter=False),
    "c2_case2_nofilter_4000": dict(cfg="c2", case=2, steps=4000, opts=dict(mode="sa"), filter=False),
    "c3_sa_640": dict(cfg="c3", steps=640, snap=(64,), opts=dict(mode="sa")),
    "c4_m5_sa_64": dict(cfg="c4", member=5, steps=64, opts=dict(mode="sa")),
    "c4_m40_sa_64": dict(cfg="c4", member=40, steps=64, opts=dict(mode="sa")),
    "c4_m90_sa_64": dict(cfg="c4", member=90, steps=64, opts=dict(mode="sa")),
    "c5_sa_2": dict(cfg="c5", steps=2, opts=dict(mode="sa")),
    "c5_iter_aa_2": dict(cfg="c5", steps=2, opts=dict(mode="iter", max_sweeps=400, accel="anderson")),
}


def config(spec):
    import sbi_inputs as si
    c = spec["cfg"]
    if c == "c1":
        return si.config_c1()
    if c == "c2":
        return si.config_c2(case=spec["case"])
    if c == "c3":
        return si.config_c3()
    if c == "c4":
        return si.config_c4_member(spec["member"])
    if c == "c5":
        return si.config_c5()
    raise ValueError(c)


def sample_idx(npt: int, name: str) -> np.ndarray:
    seed = sum(ord(ch) for ch in name)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(npt, size=min(NSAMPLE, npt), replace=False)).astype(np.int64)


def summary(prefix, eta, phi, idx, full):
    out = {}
    if full:
        out[prefix + "eta"] = eta
        out[prefix + "phi"] = phi
    else:
        out[prefix + "eta"] = eta.ravel()[idx]
        out[prefix + "phi"] = phi.ravel()[idx]
    out[prefix + "eta_absmax"] = np.abs(eta).max()
    out[prefix + "phi_absmax"] = np.abs(phi).max()
    out[prefix + "eta_sum"] = eta.sum()
    out[prefix + "eta_sumsq"] = (eta * eta).sum()
    return out


def make(name: str) -> str:
    from oracle import Grid, Solver
    spec = GOLDENS[name]
    cfg = config(spec)
    g = cfg["grid"]
    opts = dict(spec["opts"])
    kw = {}
    if spec["cfg"] == "c2":
        kw["relaxation_zone"] = cfg["relax"]
        if spec.get("filter"):
            kw["filter_beta"] = cfg["filter_beta"]
    o = Solver(Grid(g.nx, g.ny, g.lx, g.ly if g.ny > 1 else 1.0), cfg["depth"], h_ref=cfg["h_ref"], **opts, **kw)
    tol = cfg["tol"] if opts["mode"] == "iter" else 0.0
    full = g.ny == 1
    idx = sample_idx(g.nx * g.ny, name)
    out = dict(idx=idx, steps=spec["steps"], dt=cfg["dt"], tol=tol, nx=g.nx, ny=g.ny)
    t0 = time.time()
    eta, phi = cfg["eta"], cfg["phi"]
    sweeps = []
    done = 0
    t = 0.0
    for stop in sorted(set(spec.get("snap", ())) | {spec["steps"]}):
        eta, phi, st = o.step(eta, phi, cfg["dt"], stop - done, tol=tol, t0=t)
        t += (stop - done) * cfg["dt"]
        done = stop
        sweeps += [s.sweeps for s in st]
        if stop != spec["steps"]:
            out.update(summary(f"s{stop}_", eta, phi, idx, full))
    out.update(summary("", eta, phi, idx, full))
    if opts["mode"] == "iter":
        out["sweeps"] = np.array(sweeps, dtype=np.int32)
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **out)
    return f"{name}: {time.time() - t0:.0f} s, max|eta| {np.abs(eta).max():.4g}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    names = a.names or list(GOLDENS)
    with ProcessPoolExecutor(max_workers=a.jobs) as ex:
        for msg in ex.map(make, names):
            print(msg, flush=True)


if __name__ == "__main__":
    main()
