"""Pins of the oracle's Anderson-accelerated iteration (mixing of the relaxed
sweep over the last two differences): it reaches the fixed point of the same
summed operator as the relaxed sweeps, in fewer sweeps, and with depth 0 it
is the relaxed iteration itself."""
import numpy as np
import pytest

from oracle import Grid, Solver
import sbi_inputs as si


def _pair(cfg, **kw):
    gs = cfg["grid"]
    g = Grid(gs.nx, gs.ny, gs.lx, gs.ly)
    return (Solver(g, cfg["depth"], mode="iter", max_sweeps=200, **kw),
            Solver(g, cfg["depth"], mode="iter", max_sweeps=200, accel="anderson", **kw))


@pytest.mark.parametrize("cfg", [si.config_c5(seed=1, n=128), si.config_c3(n=128)], ids=["variable bed", "flat"])
def test_same_fixed_point_in_fewer_sweeps(cfg):
    a, b = _pair(cfg)
    tol = 1e-11
    Wa, ia = a.vertical_velocity(cfg["eta"], cfg["phi"], tol=tol)
    Wb, ib = b.vertical_velocity(cfg["eta"], cfg["phi"], tol=tol)
    assert ia.status == 0 and ib.status == 0
    assert ib.sweeps <= 0.7 * ia.sweeps, (ia.sweeps, ib.sweeps)
    # both stop within ~tol/(1 - contraction) of the common fixed point
    assert np.abs(Wa - Wb).max() <= 20 * tol * np.abs(Wa).max()


def test_depth_zero_is_the_relaxed_iteration():
    cfg = si.config_c5(seed=2, n=64)
    a, _ = _pair(cfg)
    gs = cfg["grid"]
    b = Solver(Grid(gs.nx, gs.ny, gs.lx, gs.ly), cfg["depth"], mode="iter", max_sweeps=200, accel="anderson",
               aa_depth=0)
    Wa, ia = a.vertical_velocity(cfg["eta"], cfg["phi"], tol=1e-10)
    Wb, ib = b.vertical_velocity(cfg["eta"], cfg["phi"], tol=1e-10)
    assert ia.sweeps == ib.sweeps and ia.history == ib.history
    assert np.array_equal(Wa, Wb)


def test_stepping_with_anderson_matches_relaxed_sweeps():
    cfg = si.config_c5(seed=3, n=64)
    a, b = _pair(cfg)
    ea, pa, sa = a.step(cfg["eta"], cfg["phi"], cfg["dt"], 2, tol=1e-11)
    eb, pb, sb = b.step(cfg["eta"], cfg["phi"], cfg["dt"], 2, tol=1e-11)
    assert sum(x.sweeps for x in sb) < 0.75 * sum(x.sweeps for x in sa)
    assert np.abs(ea - eb).max() <= 1e-9 * np.abs(ea).max()
