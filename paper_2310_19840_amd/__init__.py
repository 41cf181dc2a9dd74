"""MI355X-native spectral boundary-integral (SBI) water-wave solver.

Python face of libsbi.so (include/sbi.h).  This module only marshals
arguments: device memory and streams come from PyTorch, and every step of the
computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib
from ._lib import SBIError  # noqa: F401

_PREC = {"fp64": _lib.SBI_FP64, "fp32": _lib.SBI_FP32, "mixed": _lib.SBI_MIXED}
_MODE = {"iter": _lib.SBI_MODE_ITER, "sa": _lib.SBI_MODE_SA, "full": _lib.SBI_MODE_FULL}
_SEED = {"linear": _lib.SBI_SEED_LINEAR, "prev": _lib.SBI_SEED_PREV, "net": _lib.SBI_SEED_NET,
         "user": _lib.SBI_SEED_USER}


_ACCEL = {None: _lib.SBI_ACCEL_NONE, "none": _lib.SBI_ACCEL_NONE, "anderson": _lib.SBI_ACCEL_ANDERSON}


def make_grid(nx, ny, lx, ly=1.0, order=7, dealias=0.5, precision="fp64", mode="iter", seed="linear",
              max_sweeps=64, relax=True, filter_beta=None, accel=None) -> _lib.sbi_grid:
    lib = _lib.load()
    g = _lib.sbi_grid()
    lib.sbi_grid_defaults(C.byref(g))
    g.nx, g.ny, g.lx, g.ly = int(nx), int(ny), float(lx), float(ly)
    g.order, g.dealias = int(order), float(dealias)
    g.precision, g.mode, g.seed = _PREC[precision], _MODE[mode], _SEED[seed]
    g.max_sweeps, g.relax = int(max_sweeps), int(bool(relax))
    if filter_beta is not None:
        g.filter_beta1, g.filter_beta2 = float(filter_beta[0]), float(filter_beta[1])
    g.accel = _ACCEL[accel]
    return g


def net_blob(theta, in_scale, out_scale) -> bytes:
    """Weight blob of the learned warm start: header + FP32 parameter vector.
    out_scale: the scales of the V and phi_b corrections (two values)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
    if th.size != _lib.SBI_NET_PARAMS:
        raise ValueError(f"expected {_lib.SBI_NET_PARAMS} parameters")
    h = _lib.sbi_net_header()
    h.magic = b"SBIW"
    h.version, h.cin, h.width, h.nparams = 1, 8, 32, _lib.SBI_NET_PARAMS
    for i, v in enumerate(np.asarray(in_scale, dtype=np.float32).ravel()[:8]):
        h.in_scale[i] = float(v)
    osc = np.broadcast_to(np.asarray(out_scale, dtype=np.float64).ravel(), (2,))
    h.out_scale[0], h.out_scale[1] = float(osc[0]), float(osc[1])
    return bytes(h) + th.tobytes()


def net_blob_parts(blob: bytes):
    """(theta, in_scale, out_scale) of a weight blob."""
    h = _lib.sbi_net_header.from_buffer_copy(blob[:C.sizeof(_lib.sbi_net_header)])
    th = np.frombuffer(blob[C.sizeof(_lib.sbi_net_header):], dtype=np.float32).copy()
    return th, np.array(h.in_scale[:], dtype=np.float32), np.array(h.out_scale[:], dtype=np.float32)


def vertical_velocity_noalloc(eta, phi_s, depth, nx, ny, lx, ly=1.0, h_ref=-1.0, tol=1e-10, w_seed=None, out=None,
                              stream=None, **opts):
    """One W solve through sbi_vertical_velocity_noalloc (no allocation in the
    library: its workspace is the library's static device scratch).  eta, phi_s
    (and w_seed, out): contiguous [batch, ny, nx] tensors on the current device
    of the grid's precision.  Returns (W, status, [(sweeps, status, residual,
    omega, FP32 sweeps)] per member)."""
    import torch

    lib = _lib.load()
    g = make_grid(nx, ny, lx, ly, **opts)
    batch = eta.shape[0] if eta.dim() == 3 else 1
    dt = torch.float32 if g.precision == _lib.SBI_FP32 else torch.float64
    for x, name in ((eta, "eta"), (phi_s, "phi_s"), (w_seed, "w_seed"), (out, "w_out")):
        if x is not None and (x.dtype != dt or not x.is_contiguous() or x.numel() != batch * ny * nx):
            raise TypeError(f"{name} must be a contiguous {dt} tensor of {batch * ny * nx} values")
    out = torch.empty((batch, ny, nx), dtype=dt, device=eta.device) if out is None else out
    d = np.ascontiguousarray(np.broadcast_to(np.asarray(depth, dtype=np.float64).reshape((-1, ny, nx)),
                                             (batch, ny, nx)))
    stream = stream if stream is not None else torch.cuda.current_stream(eta.device)
    infos = (_lib.sbi_solve_info * batch)()
    st = lib.sbi_vertical_velocity_noalloc(C.byref(g), batch, d.ctypes.data_as(C.POINTER(C.c_double)),
                                           float(h_ref), C.c_void_p(eta.data_ptr()), C.c_void_p(phi_s.data_ptr()),
                                           float(tol), C.c_void_p(w_seed.data_ptr()) if w_seed is not None else None,
                                           C.c_void_p(out.data_ptr()), infos, C.c_void_p(stream.cuda_stream))
    res = [(i.sweeps, i.status, i.residual, i.omega, i.sweeps_fp32) for i in infos]
    if st < 0:
        raise SBIError(st, "sbi_vertical_velocity_noalloc", res)
    return out, st, res


def _plan_dict(p):
    return dict(row_variant=p.row_variant, row_rows=p.row_rows, col_split=p.col_split, us=p.us, cached=bool(p.cached))


def tune_cache_load(path: str) -> int:
    """Merge a plan-cache file into the process's plan cache; returns the entries read."""
    n = C.c_int32(0)
    st = _lib.load().sbi_tune_cache_load(os.fsencode(path), C.byref(n))
    if st < 0:
        raise SBIError(st, "sbi_tune_cache_load")
    return n.value


def tune_cache_save(path: str) -> int:
    """Write the process's plan cache to a file; returns the entries written."""
    n = C.c_int32(0)
    st = _lib.load().sbi_tune_cache_save(os.fsencode(path), C.byref(n))
    if st < 0:
        raise SBIError(st, "sbi_tune_cache_save")
    return n.value


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
        self.dtype = torch.float32 if self.grid.precision == _lib.SBI_FP32 else torch.float64
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
        res = [(i.sweeps, i.status, i.residual, i.omega, i.sweeps_fp32) for i in infos]
        if st < 0:
            raise SBIError(st, "sbi_vertical_velocity", res)
        return out, st, res

    def step(self, eta, phi_s, dt, n, tol=1e-10, t=0.0):
        s = _lib.sbi_state(self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), float(t))
        info = _lib.sbi_step_info()
        st = self.lib.sbi_step(self.ctx, C.byref(s), float(dt), int(n), float(tol), C.byref(info))
        if st < 0:
            raise SBIError(st, "sbi_step")
        return st, dict(t=s.t, solves=info.solves, sweeps_total=info.sweeps_total, sweeps_max=info.sweeps_max,
                        fallbacks=info.fallbacks, max_residual=info.max_residual,
                        sweeps_fp32_total=info.sweeps_fp32_total)

    def step_adaptive(self, eta, phi_s, t_end, dt, rk_tol, tol=1e-10, t=0.0, max_steps=1000):
        s = _lib.sbi_state(self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), float(t))
        info = _lib.sbi_adapt_info()
        st = self.lib.sbi_step_adaptive(self.ctx, C.byref(s), float(t_end), float(dt), float(rk_tol), float(tol),
                                        int(max_steps), C.byref(info))
        if st < 0:
            raise SBIError(st, "sbi_step_adaptive")
        v = info.solve
        return st, dict(t=s.t, accepted=info.accepted, rejected=info.rejected, dt_next=info.dt_next,
                        err_last=info.err_last, err_max=info.err_max, solves=v.solves, sweeps_total=v.sweeps_total,
                        sweeps_max=v.sweeps_max, fallbacks=v.fallbacks, max_residual=v.max_residual,
                        sweeps_fp32_total=v.sweeps_fp32_total)

    def diagnostics(self, eta, phi_s, tol=1e-10):
        s = _lib.sbi_state(self._dev(eta, "eta"), self._dev(phi_s, "phi_s"), 0.0)
        m = (C.c_double * self.batch)()
        e = (C.c_double * self.batch)()
        st = self.lib.sbi_diagnostics(self.ctx, C.byref(s), float(tol), m, e)
        if st < 0:
            raise SBIError(st, "sbi_diagnostics")
        return np.array(m[:]), np.array(e[:])

    # -- launch plans -----------------------------------------------------------
    def plan_variants(self):
        """Row variants built for this context (list of variant numbers)."""
        m = self.lib.sbi_plan_variants(self.ctx)
        return [v for v in range(4) if (m >> v) & 1]

    def plan(self):
        p = _lib.sbi_plan()
        st = self.lib.sbi_plan_get(self.ctx, C.byref(p))
        if st < 0:
            raise SBIError(st, "sbi_plan_get")
        return _plan_dict(p)

    def set_plan(self, row_variant=0, row_rows=0, col_split=0):
        p = _lib.sbi_plan(int(row_variant), int(row_rows), int(col_split), 0.0, 0)
        st = self.lib.sbi_plan_set(self.ctx, C.byref(p))
        if st < 0:
            raise SBIError(st, "sbi_plan_set")

    def autotune(self, force=False):
        p = _lib.sbi_plan()
        st = self.lib.sbi_autotune(self.ctx, _lib.SBI_TUNE_FORCE if force else 0, C.byref(p))
        if st < 0:
            raise SBIError(st, "sbi_autotune")
        return _plan_dict(p)

    # -- learned warm start ----------------------------------------------------
    def net_load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        st = self.lib.sbi_net_load(self.ctx, C.cast(buf, C.c_void_p), len(blob))
        if st < 0:
            raise SBIError(st, "sbi_net_load")

    def net_features(self, eta, phi_s, feat=None, wlin=None):
        t = self.torch
        if feat is None:
            feat = t.empty((self.batch, self.ny, self.nx, 8), dtype=t.float32, device=self.device)
        if wlin is None:
            wlin = self.empty()
        st = self.lib.sbi_net_features(self.ctx, self._dev(eta, "eta"), self._dev(phi_s, "phi_s"),
                                       C.c_void_p(feat.data_ptr()), self._dev(wlin, "wlin"))
        if st < 0:
            raise SBIError(st, "sbi_net_features")
        return feat, wlin

    def net_infer(self, feat, wlin):
        """(V seed, phi_b correction) predicted by the loaded network."""
        out, outb = self.empty(), self.empty()
        if feat.dtype != self.torch.float32 or not feat.is_contiguous() or feat.numel() != 8 * self.batch * self.ny * self.nx:
            raise TypeError("feat must be a contiguous float32 [batch, ny, nx, 8] tensor")
        st = self.lib.sbi_net_infer(self.ctx, C.c_void_p(feat.data_ptr()), self._dev(wlin, "wlin"),
                                    self._dev(out, "seed_out"), self._dev(outb, "dphib_out"))
        if st < 0:
            raise SBIError(st, "sbi_net_infer")
        return out, outb

    # -- learned history layer ------------------------------------------------
    def hist_load(self, taps, bins, dk, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
        if w.size != self.lib.sbi_net_hist_param_count(int(taps), int(bins)):
            raise ValueError("wrong number of history-layer weights")
        st = self.lib.sbi_net_hist_load(self.ctx, int(taps), int(bins), float(dk),
                                        w.ctypes.data_as(C.POINTER(C.c_float)))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_load")
        self._hist_n = w.size
        self._hist_shape = (int(taps), int(bins))

    def hist_train(self, enable=True):
        st = self.lib.sbi_net_hist_train(self.ctx, int(bool(enable)))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_train")

    def hist_gradient(self):
        """(loss sum, solves, gradient sum, Gram sums) accumulated since the last optimiser step."""
        loss = C.c_double()
        n = C.c_int32()
        g = np.zeros(self._hist_n, dtype=np.float64)
        K, nb = self._hist_shape
        gm = np.zeros(2 * 4 * nb * K * K * 2, dtype=np.float64)
        st = self.lib.sbi_net_hist_gradient(self.ctx, C.byref(loss), C.byref(n),
                                            g.ctypes.data_as(C.POINTER(C.c_double)),
                                            gm.ctypes.data_as(C.POINTER(C.c_double)))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_gradient")
        return loss.value, n.value, g, gm

    def hist_newton(self, lam=1e-9):
        loss = C.c_double()
        n = C.c_int32()
        st = self.lib.sbi_net_hist_newton(self.ctx, float(lam), C.byref(loss), C.byref(n))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_newton")
        return loss.value, n.value

    def hist_adam(self, lr):
        loss = C.c_double()
        n = C.c_int32()
        st = self.lib.sbi_net_hist_adam(self.ctx, C.c_float(lr), C.byref(loss), C.byref(n))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_adam")
        return loss.value, n.value

    def hist_params(self):
        w = np.zeros(self._hist_n, dtype=np.float32)
        st = self.lib.sbi_net_hist_params(self.ctx, w.ctypes.data_as(C.POINTER(C.c_float)))
        if st < 0:
            raise SBIError(st, "sbi_net_hist_params")
        return w

    def last_correction(self):
        """(V* - W_lin, phi_b - phi_b,lin) left by the last solve (seed="prev" contexts)."""
        dv, db = self.empty(), self.empty()
        st = self.lib.sbi_last_correction(self.ctx, self._dev(dv, "dv_out"), self._dev(db, "dphib_out"))
        if st < 0:
            raise SBIError(st, "sbi_last_correction")
        return dv, db

    def set_depth(self, depth, h_ref=-1.0):
        d = self._host_depth(depth)
        st = self.lib.sbi_set_depth(self.ctx, d.ctypes.data_as(C.POINTER(C.c_double)), float(h_ref))
        if st < 0:
            raise SBIError(st, "sbi_set_depth")
        return st

    def set_relaxation(self, a, k, omega, gen_len, abs_len, ramp_periods):
        arr = (C.c_double * 6)(a, k, omega, gen_len, abs_len, ramp_periods)
        st = self.lib.sbi_set_relaxation(self.ctx, arr, 6)
        if st < 0:
            raise SBIError(st, "sbi_set_relaxation")

    def set_wavemaker(self, comps=(), x0=None, width=4 * np.pi, h=None):
        """Wave-tank pressures: comps = [(a_j, k_j, omega_j, theta_j), ...] of the
        pneumatic wavemaker; damping centred at x0 with the given width (x0 None:
        no damping); h: depth of the generator's factor (None: h_ref)."""
        flat = [float(v) for c in comps for v in c]
        arr = (C.c_double * max(len(flat), 1))(*flat)
        st = self.lib.sbi_set_wavemaker(self.ctx, arr, len(flat) // 4, float(h or 0.0),
                                        float(x0 if x0 is not None else 0.0),
                                        float(width) if x0 is not None else 0.0)
        if st < 0:
            raise SBIError(st, "sbi_set_wavemaker")

    def last_stats(self):
        out = (C.c_double * 3)()
        n = self.lib.sbi_last_stats(self.ctx, out, 3)
        return dict(zip(("launches", "syncs", "sweeps"), out[:n]))

    def profile(self, enable=True, sweeps_only=False):
        """Time kernel launches with HIP events (all classes, or the sweep passes only)."""
        mode = _lib.SBI_PROFILE_OFF if not enable else (_lib.SBI_PROFILE_SWEEPS if sweeps_only else _lib.SBI_PROFILE_ALL)
        st = self.lib.sbi_profile_enable(self.ctx, mode)
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


class NetTrainer:
    """The library's warm-start trainer (FP32 masters, Adam) on `batch` periodic ny x nx fields."""

    def __init__(self, batch, ny, nx, theta, device=None, stream=None):
        import torch

        self.torch = torch
        self.lib = _lib.load()
        self.batch, self.ny, self.nx = int(batch), int(ny), int(nx)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = int(self.lib.sbi_net_trainer_bytes(self.batch, self.ny, self.nx))
        if nbytes == 0:
            raise SBIError(_lib.SBI_ERR_INVALID_ARG, "sbi_net_trainer_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
        if th.size != _lib.SBI_NET_PARAMS:
            raise ValueError(f"expected {_lib.SBI_NET_PARAMS} parameters")
        tr = C.c_void_p()
        st = self.lib.sbi_net_trainer_init(C.byref(tr), self.batch, self.ny, self.nx,
                                           th.ctypes.data_as(C.POINTER(C.c_float)),
                                           C.c_void_p(self.workspace.data_ptr()), nbytes,
                                           C.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise SBIError(st, "sbi_net_trainer_init")
        self.tr = tr

    def _f32(self, x, shape, name):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.dtype != t.float32 or x.device != self.device or not x.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if x.numel() != int(np.prod(shape)):
            raise ValueError(f"{name} must hold {int(np.prod(shape))} values")
        return C.c_void_p(x.data_ptr())

    def forward(self, feat):
        y = self.torch.empty((self.batch, self.ny, self.nx, 2), dtype=self.torch.float32, device=self.device)
        st = self.lib.sbi_net_trainer_forward(self.tr, self._f32(feat, (self.batch, self.ny, self.nx, 8), "feat"),
                                              C.c_void_p(y.data_ptr()))
        if st < 0:
            raise SBIError(st, "sbi_net_trainer_forward")
        return y

    def gradient(self, feat, target, want_grad=False):
        loss = C.c_double()
        g = np.zeros(_lib.SBI_NET_PARAMS, dtype=np.float32) if want_grad else None
        st = self.lib.sbi_net_trainer_gradient(
            self.tr, self._f32(feat, (self.batch, self.ny, self.nx, 8), "feat"),
            self._f32(target, (self.batch, self.ny, self.nx, 2), "target"), C.byref(loss),
            g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None)
        if st < 0:
            raise SBIError(st, "sbi_net_trainer_gradient")
        return (loss.value, g) if want_grad else loss.value

    def adam(self, lr):
        st = self.lib.sbi_net_trainer_adam(self.tr, C.c_float(lr))
        if st < 0:
            raise SBIError(st, "sbi_net_trainer_adam")

    def params(self):
        th = np.zeros(_lib.SBI_NET_PARAMS, dtype=np.float32)
        st = self.lib.sbi_net_trainer_params(self.tr, th.ctypes.data_as(C.POINTER(C.c_float)))
        if st < 0:
            raise SBIError(st, "sbi_net_trainer_params")
        return th

    def close(self):
        if getattr(self, "tr", None):
            self.lib.sbi_net_trainer_destroy(self.tr)
            self.tr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Members of uneven grids stepped together (include/sbi_batch.h).

    members: list of dicts with keys nx, ny, lx, ly, depth and any make_grid
    option (precision, mode, seed, max_sweeps, ...)."""

    def __init__(self, members, h_ref=-1.0, device=None, stream=None, graph=True, autotune=False):
        import torch

        self.torch = torch
        self.lib = _lib.load()
        self.m = len(members)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        grids = (_lib.sbi_grid * self.m)()
        self.shapes, self.dtypes = [], []
        deps = []
        for i, mb in enumerate(members):
            opts = {k: v for k, v in mb.items() if k not in ("nx", "ny", "lx", "ly", "depth")}
            grids[i] = make_grid(mb["nx"], mb["ny"], mb["lx"], mb.get("ly", 1.0), **opts)
            self.shapes.append((int(mb["ny"]), int(mb["nx"])))
            self.dtypes.append(torch.float32 if grids[i].precision == _lib.SBI_FP32 else torch.float64)
            d = np.ascontiguousarray(np.asarray(mb["depth"], dtype=np.float64).reshape(self.shapes[-1]))
            deps.append(d)
        self._deps = deps
        dptr = (C.POINTER(C.c_double) * self.m)(*[d.ctypes.data_as(C.POINTER(C.c_double)) for d in deps])
        nbytes = int(self.lib.sbi_batch_workspace_bytes(self.m, grids))
        if nbytes == 0:
            raise SBIError(_lib.SBI_ERR_INVALID_ARG, "sbi_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        flags = (_lib.SBI_BATCH_GRAPH if graph else 0) | (_lib.SBI_BATCH_AUTOTUNE if autotune else 0)
        b = C.c_void_p()
        st = self.lib.sbi_batch_init(C.byref(b), self.m, grids, dptr, float(h_ref),
                                     C.c_void_p(self.workspace.data_ptr()), nbytes,
                                     C.c_void_p(self.stream.cuda_stream), flags)
        if st < 0:
            raise SBIError(st, "sbi_batch_init")
        self.init_status = st
        self.b = b

    def step(self, etas, phis, dt, n, tol=1e-10, t=None):
        states = (_lib.sbi_state * self.m)()
        for i in range(self.m):
            for x, name in ((etas[i], "eta"), (phis[i], "phi_s")):
                if (x.dtype != self.dtypes[i] or x.device != self.device or not x.is_contiguous()
                        or x.numel() != self.shapes[i][0] * self.shapes[i][1]):
                    raise TypeError(f"member {i}: {name} must be a contiguous {self.dtypes[i]} tensor of "
                                    f"{self.shapes[i]} on {self.device}")
            states[i] = _lib.sbi_state(C.c_void_p(etas[i].data_ptr()), C.c_void_p(phis[i].data_ptr()),
                                       0.0 if t is None else float(t[i]))
        info = (_lib.sbi_step_info * self.m)()
        st = self.lib.sbi_batch_step(self.b, states, float(dt), int(n), float(tol), info)
        if st < 0:
            raise SBIError(st, "sbi_batch_step")
        return st, [dict(t=states[i].t, solves=info[i].solves, sweeps_total=info[i].sweeps_total,
                         sweeps_max=info[i].sweeps_max, max_residual=info[i].max_residual) for i in range(self.m)]

    def net_load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        st = self.lib.sbi_batch_net_load(self.b, C.cast(buf, C.c_void_p), len(blob))
        if st < 0:
            raise SBIError(st, "sbi_batch_net_load")

    def hist_load(self, taps, bins, dk, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
        st = self.lib.sbi_batch_net_hist_load(self.b, int(taps), int(bins), float(dk),
                                              w.ctypes.data_as(C.POINTER(C.c_float)))
        if st < 0:
            raise SBIError(st, "sbi_batch_net_hist_load")

    def budgets(self):
        """(sweep budget of each group, step calls redone with a larger budget)."""
        bud = (C.c_int32 * 64)()
        redos = self.lib.sbi_batch_budgets(self.b, bud, 64)
        return list(bud[:len(self.groups())]), redos

    def groups(self):
        mem = (C.c_int32 * 64)()
        spl = (C.c_int32 * 64)()
        k = self.lib.sbi_batch_groups(self.b, mem, spl, 64)
        return [(mem[i], spl[i]) for i in range(min(k, 64))]

    def plans(self):
        """Launch plan of each group."""
        out = []
        for g in range(len(self.groups())):
            p = _lib.sbi_plan()
            st = self.lib.sbi_batch_plan(self.b, g, C.byref(p))
            if st < 0:
                raise SBIError(st, "sbi_batch_plan")
            out.append(_plan_dict(p))
        return out

    def close(self):
        if getattr(self, "b", None):
            self.lib.sbi_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
