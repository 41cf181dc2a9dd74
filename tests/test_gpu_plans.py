"""Launch plans and the autotuner: every row variant and rows-per-workgroup
choice the library builds gives the oracle's W (a plan changes rounding order
only), the autotuner picks a built plan, records it in the plan cache and
takes it from there the next time, and tuned ensembles still match the
oracle.  FP64 within 1e-11 (W) / 1e-10 (steps), FP32 within 1e-5.
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


def _t(x, dtype, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _case(nx, ny, seed):
    lx = 2 * math.pi * nx / 16
    ly = 2 * math.pi * ny / 16
    gs = si.GridSpec(nx, ny, lx, ly)
    eta = si.narrowband_random(gs, seed, amp=0.06)
    phi = si.narrowband_random(gs, seed + 1, amp=0.3)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.5 - 0.3 * np.exp(-((X - lx / 3) ** 2 / (0.02 * lx * lx) + (Y - ly / 2) ** 2 / (0.02 * ly * ly)))
    return lx, ly, eta, phi, depth


def _rows_candidates(cap, ny):
    cap = min(cap, ny)
    return [r for r in (cap, cap // 2, cap // 4) if r >= 1]


# (nx, ny): 512-point rows have every variant in FP32 (radix 16 included),
# 1024-point rows the cached twiddle powers in the sweep and radix 16 in SA
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny", [(512, 64), (1024, 32)])
def test_every_plan_matches_oracle(gpu, nx, ny, precision):
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Solver
    lx, ly, eta, phi, depth = _case(nx, ny, nx + ny)
    g = Grid(nx, ny, lx, ly)
    fp32 = precision == "fp32"
    dt = torch.float32 if fp32 else torch.float64
    if fp32:
        eta = eta.astype(np.float32).astype(np.float64)
        phi = phi.astype(np.float32).astype(np.float64)
    tol_gpu = 1e-6 if fp32 else 1e-12
    bar = 1e-5 if fp32 else 1e-11
    for mode, accel in (("sa", None), ("iter", "anderson")):
        o = OSolver(g, depth, mode=mode, max_sweeps=200, accel=accel)
        Wo, oi = o.vertical_velocity(eta, phi, tol=1e-12)
        s = Solver(nx, ny, lx, ly, depth, device=gpu, mode=mode, max_sweeps=200, accel=accel, precision=precision)
        variants = s.plan_variants()
        assert 0 in variants
        elems = {0: 8, 1: 8, 2: 16, 3: 4}   # values per thread of each row variant
        caps = {v: max(1, 256 // (nx // 2 // e)) for v, e in elems.items()}
        plans = [(v, r, 0) for v in variants for r in _rows_candidates(caps[v], ny)] + [(0, 0, 2048)]
        for v, r, sp in plans:
            s.set_plan(v, r, sp)
            assert s.plan()["row_variant"] == v and s.plan()["row_rows"] == r and s.plan()["col_split"] == sp
            W, st, info = s.vertical_velocity(_t(eta, dt, gpu), _t(phi, dt, gpu), tol=tol_gpu)
            err = _rel(W.cpu().numpy()[0].astype(np.float64), Wo)
            _say(f"{precision} {nx}x{ny} {mode:4s} plan (variant {v}, rows {r}, split {sp}): W err {err:.2e}"
                 + (f" sweeps {info[0][0]}/{oi.sweeps}" if mode == "iter" else ""))
            assert err < bar
            if mode == "iter" and not fp32:
                assert info[0][0] == oi.sweeps
        # variants that are not built are refused and leave the plan alone
        for v in range(4):
            if v not in variants:
                from paper_2310_19840_amd import SBIError
                before = s.plan()
                with pytest.raises(SBIError):
                    s.set_plan(v, 0, 0)
                assert s.plan() == before
    # precision-specific availability: radix 16 only in FP32, cached powers in
    # the FP64 sweep never (it would spill); radix 4 in both
    s_it = Solver(nx, ny, lx, ly, depth, device=gpu, mode="iter", accel="anderson", precision=precision)
    s_sa = Solver(nx, ny, lx, ly, depth, device=gpu, mode="sa", precision=precision)
    if fp32:
        assert 1 in s_it.plan_variants() and 2 in s_sa.plan_variants()
    else:
        assert 1 not in s_it.plan_variants() and 2 not in s_sa.plan_variants()
    assert 3 in s_it.plan_variants() and 3 in s_sa.plan_variants()


def test_autotune_picks_a_built_plan_and_caches_it(gpu, tmp_path):
    import torch
    from oracle import Grid, Solver as OSolver
    import paper_2310_19840_amd as sbi
    nx, ny = 1024, 64
    lx, ly, eta, phi, depth = _case(nx, ny, 77)
    kw = dict(device=gpu, mode="iter", accel="anderson", precision="fp32", max_sweeps=200)
    s = sbi.Solver(nx, ny, lx, ly, depth, **kw)
    p = s.autotune(force=True)
    _say("tuned:", p)
    assert p["row_variant"] in s.plan_variants() and p["us"] > 0 and not p["cached"]
    assert s.plan()["row_variant"] == p["row_variant"] and s.plan()["row_rows"] == p["row_rows"]
    # the tuned context solves correctly
    e32 = eta.astype(np.float32)
    p32 = phi.astype(np.float32)
    Wo, _ = OSolver(Grid(nx, ny, lx, ly), depth, mode="iter", max_sweeps=200, accel="anderson").vertical_velocity(
        e32.astype(np.float64), p32.astype(np.float64), tol=1e-12)
    W, _, _ = s.vertical_velocity(_t(e32, torch.float32, gpu), _t(p32, torch.float32, gpu), tol=1e-6)
    assert _rel(W.cpu().numpy()[0].astype(np.float64), Wo) < 1e-5
    # a second context of the same kind takes the plan from the cache
    s2 = sbi.Solver(nx, ny, lx, ly, depth, **kw)
    p2 = s2.autotune()
    assert p2["cached"] and (p2["row_variant"], p2["row_rows"], p2["col_split"]) == \
        (p["row_variant"], p["row_rows"], p["col_split"])
    # another batch size is another key: searched again
    s3 = sbi.Solver(nx, ny, lx, ly, np.stack([depth, depth]), batch=2, **kw)
    assert not s3.autotune()["cached"]
    # the cache survives a save and a load
    path = str(tmp_path / "plans.txt")
    n = sbi.tune_cache_save(path)
    assert n >= 2
    assert sbi.tune_cache_load(path) == n


def test_tuned_ensemble_matches_oracle(gpu):
    """A ragged SA ensemble tuned at set-up: every group gets a built plan and
    its members' steps match the oracle."""
    import torch
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Batch
    cases = [(512, 32, 3), (256, 16, 4), (512, 32, 5)]
    mem, data = [], []
    for nx, ny, seed in cases:
        lx, ly, eta, phi, depth = _case(nx, ny, seed)
        mem.append(dict(nx=nx, ny=ny, lx=lx, ly=ly, depth=depth, precision="fp64", mode="sa"))
        data.append((lx, ly, eta, phi, depth))
    b = Batch(mem, device=gpu, graph=True, autotune=True)
    plans = b.plans()
    _say("plans:", plans)
    assert len(plans) == 2
    etas = [_t(d[2], torch.float64, gpu) for d in data]
    phis = [_t(d[3], torch.float64, gpu) for d in data]
    dt = 0.1
    b.step(etas, phis, dt, 2)
    for (nx, ny, _), (lx, ly, eta, phi, depth), e, p in zip(cases, data, etas, phis):
        o = OSolver(Grid(nx, ny, lx, ly), depth, mode="sa")
        eo, po, _ = o.step(eta, phi, dt, 2)
        assert _rel(e.cpu().numpy().reshape(eo.shape), eo) < 1e-10
        assert _rel(p.cpu().numpy().reshape(po.shape), po) < 1e-10
