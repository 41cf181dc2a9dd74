"""MI355X-native spectral boundary-integral (SBI) water-wave solver.

Python face of libsbi.so (include/sbi.h).  This module only marshals
arguments: device memory and streams come from PyTorch, and every step of the
computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import SBIError  # noqa: F401

_PREC = {"fp64": _lib.SBI_FP64, "fp32": _lib.SBI_FP32}
_MODE = {"iter": _lib.SBI_MODE_ITER, "sa": _lib.SBI_MODE_SA}
_SEED = {"linear": _lib.SBI_SEED_LINEAR, "prev": _lib.SBI_SEED_PREV, "net": _lib.SBI_SEED_NET,
         "user": _lib.SBI_SEED_USER}


def make_grid(nx, ny, lx, ly=1.0, order=7, dealias=0.5, precision="fp64", mode="iter", seed="linear",
              max_sweeps=64, relax=True, filter_beta=None) -> _lib.sbi_grid:
    lib = _lib.load()
    g = _lib.sbi_grid()
    lib.sbi_grid_defaults(C.byref(g))
    g.nx, g.ny, g.lx, g.ly = int(nx), int(ny), float(lx), float(ly)
    g.order, g.dealias = int(order), float(dealias)
    g.precision, g.mode, g.seed = _PREC[precision], _MODE[mode], _SEED[seed]
    g.max_sweeps, g.relax = int(max_sweeps), int(bool(relax))
    if filter_beta is not None:
        g.filter_beta1, g.filter_beta2 = float(filter_beta[0]), float(filter_beta[1])
    return g


def workspace_bytes(grid: _lib.sbi_grid, batch: int = 1) -> int:
    return int(_lib.load().sbi_workspace_bytes(C.byref(grid), int(batch)))


class Solver:
    """One context of the library: `batch` members of one grid on one stream."""

    def __init__(self, nx, ny, lx, ly, depth, h_ref=-1.0, batch=1, device=None, stream=None, **opts):
        import torch

        self.torch = torch
        self.lib = _lib.load()
        self.grid = make_grid(nx, ny, lx, ly, **opts)
        self.batch = int(batch)
        self.nx, self.ny = int(nx), int(ny)
        self.dtype = torch.float64 if self.grid.precision == _lib.SBI_FP64 else torch.float32
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = workspace_bytes(self.grid, self.batch)
        if nbytes == 0:
            raise SBIError(_lib.SBI_ERR_INVALID_ARG, "sbi_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        d = self._host_depth(depth)
        ctx = C.c_void_p()
        st = self.lib.sbi_init(C.byref(ctx), C.byref(self.grid), self.batch,
                               d.ctypes.data_as(C.POINTER(C.c_double)), float(h_ref),
                               C.c_void_p(self.workspace.data_ptr()), nbytes, C.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise SBIError(st, "sbi_init")
        self.init_status = st
        self.ctx = ctx

    # -- marshalling helpers ------------------------------------------------
    def _host_depth(self, depth):
        d = np.ascontiguousarray(np.asarray(depth, dtype=np.float64))
        d = np.broadcast_to(d.reshape((-1, self.ny, self.nx)), (self.batch, self.ny, self.nx))
        return np.ascontiguousarray(d)

    def _dev(self, x, name):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.device != self.device or x.dtype != self.dtype or not x.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {self.dtype} tensor on {self.device}")
        if x.numel() != self.batch * self.ny * self.nx:
            raise ValueError(f"{name} must hold batch*ny*nx = {self.batch * self.ny * self.nx} values")
        return C.c_void_p(x.data_ptr())

    def empty(self):
        return self.torch.empty((self.batch, self.ny, self.nx), dtype=self.dtype, device=self.device)

    # -- calls ---------------------------------------------------------------
    def vertical_velocity(self, eta, phi_s, tol=1e-10, h=None, w_seed=None, out=None):
        out = self.empty() if out is None else out
        infos = (_lib.sbi_solve_info * self.batch)()
        hp = None
        if h is not None:
            hd = self._host_depth(h)
            hp = hd.ctypes.data_as(C.POINTER(C.c_double))
        seed = self._dev(w_seed, "w_seed") if w_seed is not None else None
        st = self.lib.sbi_vertical_velocity(self.ctx, self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), hp,
                                            float(tol), seed, self._dev(out, "w_out"), infos)
        if st < 0:
            raise SBIError(st, "sbi_vertical_velocity")
        return out, st, [(i.sweeps, i.status, i.residual, i.omega) for i in infos]

    def step(self, eta, phi_s, dt, n, tol=1e-10, t=0.0):
        s = _lib.sbi_state(self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), float(t))
        info = _lib.sbi_step_info()
        st = self.lib.sbi_step(self.ctx, C.byref(s), float(dt), int(n), float(tol), C.byref(info))
        if st < 0:
            raise SBIError(st, "sbi_step")
        return st, dict(t=s.t, solves=info.solves, sweeps_total=info.sweeps_total, sweeps_max=info.sweeps_max,
                        fallbacks=info.fallbacks, max_residual=info.max_residual)

    def diagnostics(self, eta, phi_s, tol=1e-10):
        s = _lib.sbi_state(self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), 0.0)
        m = (C.c_double * self.batch)()
        e = (C.c_double * self.batch)()
        st = self.lib.sbi_diagnostics(self.ctx, C.byref(s), float(tol), m, e)
        if st < 0:
            raise SBIError(st, "sbi_diagnostics")
        return np.array(m[:]), np.array(e[:])

    def set_relaxation(self, a, k, omega, gen_len, abs_len, ramp_periods):
        arr = (C.c_double * 6)(a, k, omega, gen_len, abs_len, ramp_periods)
        st = self.lib.sbi_set_relaxation(self.ctx, arr, 6)
        if st < 0:
            raise SBIError(st, "sbi_set_relaxation")

    def last_stats(self):
        out = (C.c_double * 3)()
        n = self.lib.sbi_last_stats(self.ctx, out, 3)
        return dict(zip(("launches", "syncs", "sweeps"), out[:n]))

    def profile(self, enable=True):
        st = self.lib.sbi_profile_enable(self.ctx, int(bool(enable)))
        if st < 0:
            raise SBIError(st, "sbi_profile_enable")

    def profile_read(self):
        n = 32
        names = (C.c_char_p * n)()
        tot = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        k = self.lib.sbi_profile_read(self.ctx, names, tot, cnt, n)
        return {names[i].decode(): (tot[i], cnt[i]) for i in range(k)}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.sbi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
