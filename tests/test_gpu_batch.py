"""Ensembles of uneven grids (include/sbi_batch.h) on the GPU.

A member of a batch runs the same kernels as a context of its own, so its
states must equal the single-context run exactly; graph replays must equal
the same calls made without capture, replay after replay; and one member is
checked against the FP64 oracle (1e-10).
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


def _member(n_x, n_y, seed, precision="fp64", mode="iter", bump=0.15, wl=4.0, seed_mode="linear"):
    lx = wl * 2 * math.pi * n_x / 64
    ly = wl * 2 * math.pi * n_y / 64 if n_y > 1 else 1.0
    gs = si.GridSpec(n_x, n_y, lx, ly)
    eta, phi = si.jonswap_crossing_sea(gs, 1.2, seed=seed, hs_half=0.04)
    X, Y = np.meshgrid(gs.x(), gs.y())
    depth = 1.2 - bump * np.exp(-((X - lx / 2) ** 2 + (Y - ly / 3) ** 2) / (0.02 * lx * lx))
    return dict(nx=n_x, ny=n_y, lx=lx, ly=ly, depth=depth, precision=precision, mode=mode, max_sweeps=120,
                seed=seed_mode), eta, phi


def _ragged(precision="fp64", mode="iter", seed_mode="linear"):
    specs = [(64, 64, 1), (128, 64, 2), (64, 64, 3), (64, 32, 4), (128, 64, 5)]
    return [_member(a, b, s, precision, mode, seed_mode=seed_mode) for a, b, s in specs]


def _tensors(mems, gpu):
    import torch
    out_e, out_p = [], []
    for m, e, p in mems:
        dt = torch.float64 if m["precision"] == "fp64" else torch.float32
        out_e.append(torch.tensor(e, dtype=dt, device=gpu).contiguous())
        out_p.append(torch.tensor(p, dtype=dt, device=gpu).contiguous())
    return out_e, out_p


DT = 2 * math.pi / math.sqrt(math.tanh(1.2)) / 32


@pytest.mark.parametrize("mode", ["iter", "sa"])
def test_batch_members_equal_single_contexts(gpu, mode):
    from paper_2310_19840_amd import Batch, Solver
    mems = _ragged(mode=mode)
    _say("ragged batch vs single contexts", mode)
    b = Batch([m for m, _, _ in mems], device=gpu, graph=False)
    assert [g[0] for g in b.groups()] == [2, 2, 1]
    et, pt = _tensors(mems, gpu)
    st, info = b.step(et, pt, DT, 2, tol=1e-11)
    assert st == 0
    for i, (m, e, p) in enumerate(mems):
        s = Solver(m["nx"], m["ny"], m["lx"], m["ly"], m["depth"], device=gpu, mode=mode, max_sweeps=120)
        es, ps = _tensors([(m, e, p)], gpu)
        _, si_ = s.step(es[0], ps[0], DT, 2, tol=1e-11)
        assert np.array_equal(et[i].cpu().numpy(), es[0].cpu().numpy().reshape(et[i].shape)), i
        assert np.array_equal(pt[i].cpu().numpy(), ps[0].cpu().numpy().reshape(pt[i].shape)), i
        if mode == "iter":
            assert info[i]["solves"] == 8
            assert info[i]["sweeps_total"] == si_["sweeps_total"]
            assert info[i]["sweeps_max"] == si_["sweeps_max"]


def test_batch_member_matches_oracle(gpu):
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Batch
    mems = _ragged()
    _say("batch member vs oracle")
    b = Batch([m for m, _, _ in mems], device=gpu, graph=True)
    et, pt = _tensors(mems, gpu)
    b.step(et, pt, DT, 2, tol=1e-11)
    m, e, p = mems[1]
    o = OSolver(Grid(m["nx"], m["ny"], m["lx"], m["ly"]), m["depth"], mode="iter", max_sweeps=120)
    eo, po, _ = o.step(e, p, DT, 2, tol=1e-11)
    assert np.abs(et[1].cpu().numpy() - eo).max() < 1e-10 * np.abs(eo).max()
    assert np.abs(pt[1].cpu().numpy() - po).max() < 1e-10 * np.abs(po).max()


@pytest.mark.parametrize("seed_mode", ["linear", "prev"])
def test_graph_replays_equal_eager_calls(gpu, seed_mode):
    from paper_2310_19840_amd import Batch
    mems = _ragged(seed_mode=seed_mode)
    _say("graph replays vs eager", seed_mode)
    bg = Batch([m for m, _, _ in mems], device=gpu, graph=True)
    be = Batch([m for m, _, _ in mems], device=gpu, graph=False)
    eg, pg = _tensors(mems, gpu)
    ee, pe = _tensors(mems, gpu)
    for call in range(3):
        sg, ig = bg.step(eg, pg, DT, 1, tol=1e-11)
        se, ie = be.step(ee, pe, DT, 1, tol=1e-11)
        assert sg == se == 0
        for i in range(len(mems)):
            assert np.array_equal(eg[i].cpu().numpy(), ee[i].cpu().numpy()), (call, i)
            assert np.array_equal(pg[i].cpu().numpy(), pe[i].cpu().numpy()), (call, i)
            assert ig[i]["sweeps_total"] == ie[i]["sweeps_total"]


def test_fp32_sa_batch_matches_fp64(gpu):
    from paper_2310_19840_amd import Batch
    _say("fp32 SA batch vs fp64")
    m32 = _ragged(precision="fp32", mode="sa")
    m64 = _ragged(precision="fp64", mode="sa")
    b32 = Batch([m for m, _, _ in m32], device=gpu, graph=True)
    b64 = Batch([m for m, _, _ in m64], device=gpu, graph=True)
    e32, p32 = _tensors(m32, gpu)
    e64, p64 = _tensors(m64, gpu)
    b32.step(e32, p32, DT, 2)
    b64.step(e64, p64, DT, 2)
    for i in range(len(m32)):
        a, r = e32[i].cpu().numpy().astype(np.float64), e64[i].cpu().numpy()
        assert np.abs(a - r).max() < 1e-5 * np.abs(r).max(), i


def test_autotuned_batch_matches_oracle(gpu):
    from oracle import Grid, Solver as OSolver
    from paper_2310_19840_amd import Batch
    mems = _ragged()
    _say("autotuned batch")
    b = Batch([m for m, _, _ in mems], device=gpu, graph=True, autotune=True)
    _say("splits", b.groups())
    et, pt = _tensors(mems, gpu)
    b.step(et, pt, DT, 1, tol=1e-11)
    for i in (0, 1, 3):
        m, e, p = mems[i]
        o = OSolver(Grid(m["nx"], m["ny"], m["lx"], m["ly"]), m["depth"], mode="iter", max_sweeps=120)
        eo, po, _ = o.step(e, p, DT, 1, tol=1e-11)
        assert np.abs(et[i].cpu().numpy() - eo).max() < 1e-10 * np.abs(eo).max(), i


def test_speculative_budget_redo_is_exact(gpu):
    """Captured iterations run on a sweep budget taken from the previous call;
    a call whose solves outrun it (here: a tighter tolerance) is redone with a
    larger budget, and every call equals the eager single-context run bit for
    bit."""
    import torch
    from paper_2310_19840_amd import Batch, Solver
    mems = [_member(64, 64, 11, seed_mode="prev"), _member(128, 64, 12, seed_mode="prev")]
    for m, _, _ in mems:
        m["max_sweeps"] = 200
        m["accel"] = "anderson"
    _say("speculative sweep budget")
    b = Batch([m for m, _, _ in mems], device=gpu, graph=True)
    et, pt = _tensors(mems, gpu)
    singles = []
    for m, e, p in mems:
        s = Solver(m["nx"], m["ny"], m["lx"], m["ly"], m["depth"], device=gpu, mode="iter", seed="prev",
                   max_sweeps=200, accel="anderson")
        singles.append((s, torch.tensor(e, dtype=torch.float64, device=gpu), torch.tensor(p, dtype=torch.float64,
                                                                                          device=gpu)))
    budgets = []
    for call, tol in enumerate((1e-8, 1e-8, 1e-8, 1e-12, 1e-12)):
        b.step(et, pt, DT, 1, tol=tol)
        for s, e, p in singles:
            s.step(e, p, DT, 1, tol=tol)
        for (s, e, p), eb, pb in zip(singles, et, pt):
            assert torch.equal(e, eb) and torch.equal(p, pb), call
        budgets.append(b.budgets())
    _say("   budgets per call:", budgets)
    # after the first call the budget follows the sweeps needed, far below the cap
    assert all(x < 200 for x in budgets[1][0])
    # the tighter tolerance outran it at least once, and was redone
    assert budgets[-1][1] >= 1


@pytest.mark.parametrize("mode,seed_mode", [("iter", "prev"), ("sa", "linear")])
def test_long_graph_calls_split_into_parts_equal_single_contexts(gpu, mode, seed_mode):
    """A captured call of 9 steps runs as a prologue, parts of 4, 4 and 1
    steps and an epilogue; the spectral state stays on the device between the
    parts, so every member equals its single-context 9-step call bit for bit,
    on the first call (seeds change between the parts) and on a replay."""
    from paper_2310_19840_amd import Batch, Solver
    mems = _ragged(mode=mode, seed_mode=seed_mode)[:3]
    _say("9-step graph calls vs single contexts", mode, seed_mode)
    b = Batch([m for m, _, _ in mems], device=gpu, graph=True)
    et, pt = _tensors(mems, gpu)
    singles = []
    for m, e, p in mems:
        s = Solver(m["nx"], m["ny"], m["lx"], m["ly"], m["depth"], device=gpu, mode=mode, max_sweeps=120,
                   seed=seed_mode)
        es, ps = _tensors([(m, e, p)], gpu)
        singles.append((s, es[0], ps[0]))
    for call in range(2):
        st, info = b.step(et, pt, DT, 9, tol=1e-11)
        assert st == 0
        for i, (s, es, ps) in enumerate(singles):
            _, si_ = s.step(es, ps, DT, 9, tol=1e-11)
            assert np.array_equal(et[i].cpu().numpy(), es.cpu().numpy().reshape(et[i].shape)), (call, i)
            assert np.array_equal(pt[i].cpu().numpy(), ps.cpu().numpy().reshape(pt[i].shape)), (call, i)
            if mode == "iter":
                assert info[i]["solves"] == 36
                assert info[i]["sweeps_total"] == si_["sweeps_total"], (call, i)
