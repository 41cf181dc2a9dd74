"""The allocation-free W solve (sbi_vertical_velocity_noalloc) against the
same solve through a context (sbi_init + sbi_vertical_velocity): identical
sweep counts and bit-identical W, on two calls in a row, the second on a
smaller grid, so the second reads the scratch array the first left behind."""
import math
import sys

import numpy as np
import pytest

import sbi_inputs as si

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(nx, ny, batch, seed):
    lx = 2 * math.pi * nx / 16
    ly = 2 * math.pi * ny / 16 if ny > 1 else 1.0
    gs = si.GridSpec(nx, ny, lx, ly)
    etas, phis, deps = [], [], []
    X, Y = np.meshgrid(gs.x(), gs.y())
    for b in range(batch):
        etas.append(si.narrowband_random(gs, seed + 2 * b, amp=0.06))
        phis.append(si.narrowband_random(gs, seed + 2 * b + 1, amp=0.3))
        deps.append(1.5 - (0.2 + 0.05 * b) * np.exp(-((X - lx / 3) ** 2 + ((Y - ly / 2) ** 2 if ny > 1 else 0.0))
                                                     / (0.02 * lx * lx)))
    return lx, ly, np.stack(etas), np.stack(phis), np.stack(deps)


def _both(gpu, nx, ny, batch, seed, **opts):
    import torch
    from paper_2310_19840_amd import Solver, vertical_velocity_noalloc
    prec = opts.get("precision", "fp64")
    dt = torch.float64 if prec == "fp64" else torch.float32
    lx, ly, eta, phi, depth = _case(nx, ny, batch, seed)
    e = torch.tensor(eta, dtype=dt, device=gpu)
    p = torch.tensor(phi, dtype=dt, device=gpu)
    W0, st0, info0 = vertical_velocity_noalloc(e, p, depth, nx, ny, lx, ly, tol=1e-11, **opts)
    s = Solver(nx, ny, lx, ly, depth, batch=batch, device=gpu, **opts)
    W1, st1, info1 = s.vertical_velocity(e, p, tol=1e-11)
    s.close()
    _say(f"   {nx}x{ny} x{batch} {opts}: status {st0}/{st1} sweeps {[i[0] for i in info0]}/{[i[0] for i in info1]}")
    assert st0 == st1
    assert [i[:2] for i in info0] == [i[:2] for i in info1]
    assert torch.equal(W0, W1)
    return W0


def test_noalloc_matches_context_solve_twice(gpu):
    _say("no-alloc: 2D 256x128 FP64 mixed iteration, batch 2, then 1D 512 SA")
    _both(gpu, 256, 128, 2, 11, mode="iter", accel="anderson", max_sweeps=200)
    _both(gpu, 512, 1, 1, 23, mode="sa")
    # and back to a larger grid in FP32 after the smaller one
    _both(gpu, 128, 64, 1, 31, mode="iter", max_sweeps=200, precision="fp32")


def test_noalloc_rejects_grids_beyond_its_scratch(gpu):
    import torch
    from paper_2310_19840_amd import SBIError, _lib, vertical_velocity_noalloc
    nx = ny = 512  # 121 MiB in FP64 > 64 MiB
    e = torch.zeros((1, ny, nx), dtype=torch.float64, device=gpu)
    with pytest.raises(SBIError) as ex:
        vertical_velocity_noalloc(e, e, np.full((ny, nx), 1.0), nx, ny, 100.0, 100.0)
    assert ex.value.code == _lib.SBI_ERR_WORKSPACE
    with pytest.raises(SBIError) as ex:
        vertical_velocity_noalloc(e[:, :64, :64].contiguous(), e[:, :64, :64].contiguous(), np.full((64, 64), 1.0),
                                  64, 64, 10.0, 10.0, seed="net")
    assert ex.value.code == _lib.SBI_ERR_UNSUPPORTED
