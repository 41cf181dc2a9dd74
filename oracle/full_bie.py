"""FP64 oracle of the fully nonlinear W solve on one-dimensional grids over a
flat bed: the boundary-integral equation of Sec. 2.3 with the remaining
integrals I^(S) of App. A kept.  TEST INFRASTRUCTURE ONLY (like the rest of
``oracle/``).

The paper writes V = sum_{j<=7} V^(j) + I^(S) (Eq. con-V): the convolution
orders V^(j) expand the integrands of the surface equation (Eq. bi-s) in the
elevation, and I^(S) integrates what the expansion leaves out -- the exact
kernels minus their truncated expansions (Eqs. app:iphis and app:ivs; over a
flat bed the bottom term app:ivarphis is absent).  Their sum is the exact
equation.  This module solves that exact equation for a periodic surface
x -> (x, eta(x)), 0 <= x < L, and so gives V with I^(S) included; I^(S)
itself is V minus the successive approximation of order 7.

Reading for one horizontal dimension (a two-dimensional flow): the paper's
kernels 1/r are those of three-dimensional flow; in two dimensions the free-
space Green function is -ln r and the jump coefficient of a smooth boundary is
pi instead of 2 pi, so the surface equation reads

    S[V](x) = pi phi_s(x) + D[phi_s](x),
    S[V](x) = int V(x') G(x, x') dx',
    D[f](x) = int f(x') dG/dn'(x, x') sqrt(1 + eta_x(x')^2) dx',

with V = dphi/dn' sqrt(1 + eta_x'^2) (as in the paper) and G the periodic
Green function with the image of the source in the flat bed z = -h (the
method of images that the paper's r_B term expresses):

    G = -ln|2 sin(pi (z - z') / L)| - ln|2 sin(pi (z - conj(z') + 2 i h) / L)|,
    z = x + i eta(x).

Over the undisturbed surface (eta = 0) S has the Fourier multiplier
S0 = (pi / |k|) (1 + exp(-2 |k| h)), and D the multiplier
-pi exp(-2 |k| h), so that V = S0^-1 (pi + D0) phi_hat = k tanh(kh) phi_hat:
the first order V^(1).  The solve iterates

    V_(n+1) = S0^-1 [ pi phi_s + D[phi_s] - (S - S0)[V_n] ],   V_0 = 0,

where S - S0 and D have smooth periodic kernels (their limits on the
diagonal are written out below), so the trapezoidal rule on the grid is
spectrally accurate, and S0^-1 acts on the discrete Fourier modes (the mean
of V is zero: no net flux through the surface).  In deep water (k_1 h > 18
for the longest wave k_1 = 2 pi / L, where exp(-2 k_1 h) < 1e-15) the image
terms are dropped.  No dealiasing applies inside the solve (the exact
equation has no truncated products); a solver in this mode masks the
returned spectrum like every other W.

Stopping rules are those of the iteration mode: r_n = max|V_n - V_(n-1)| /
max|V_n| (r_1 = 1 from V_0 = 0); converged at r_n <= tol after n sweeps;
non-finite; diverged when r_n > 1e6 or (n - 1 >= 3 and r_n > 10 min r);
not converged after max_sweeps.
"""
from __future__ import annotations

import math

import numpy as np

DEEP_K1H = 18.0


def is_deep(lx: float, h: float | None) -> bool:
    return h is None or (2.0 * math.pi / lx) * h > DEEP_K1H


def spectral_derivatives(eta, lx):
    """eta_x and eta_xx of a periodic grid function by its discrete Fourier
    series (the Nyquist mode, real for real eta, drops out of eta_x)."""
    n = eta.size
    k = 2 * np.pi * np.fft.fftfreq(n, d=lx / n)
    E = np.fft.fft(eta)
    return np.real(np.fft.ifft(1j * k * E)), np.real(np.fft.ifft(-k * k * E))


def _cot(z):
    return np.cos(z) / np.sin(z)


def kernels(eta, lx, h=None):
    """Quadrature matrices (rows: evaluation point x_i, columns: source x_j),
    trapezoidal weight dx included: KS of S - S0 and KD of D."""
    n = eta.size
    dx = lx / n
    x = np.arange(n) * dx
    ex, exx = spectral_derivatives(eta, lx)
    dxm = x[:, None] - x[None, :]
    dem = eta[:, None] - eta[None, :]
    s2 = np.sin(np.pi * dxm / lx) ** 2
    off = ~np.eye(n, dtype=bool)
    KS = np.empty((n, n))
    # direct part minus the flat kernel: -1/2 ln(1 + sinh^2(pi de / L) / sin^2(pi dx / L))
    KS[off] = -0.5 * np.log1p(np.sinh(np.pi * dem[off] / lx) ** 2 / s2[off])
    KS[~off] = -0.5 * np.log1p(ex ** 2)              # its limit as x' -> x
    z = x + 1j * eta
    u = z[None, :] - z[:, None]                       # z_j - z_i
    KD = np.empty((n, n))
    KD[off] = np.imag((np.pi / lx) * _cot(np.pi * u[off] / lx) * (1 + 1j * np.broadcast_to(ex[None, :], (n, n))[off]))
    KD[~off] = exx / (2.0 * (1.0 + ex ** 2))          # curvature limit of the double layer
    if not is_deep(lx, h):
        sh = np.sinh(np.pi * (eta[:, None] + eta[None, :] + 2 * h) / lx) ** 2
        KS += -0.5 * np.log(s2 + sh) + 0.5 * np.log(s2 + math.sinh(2 * np.pi * h / lx) ** 2)
        w = np.conj(z)[:, None] - 2j * h                # the evaluation point's image partner
        KD += np.imag((np.pi / lx) * _cot(np.pi * (z[None, :] - w) / lx) * (1 + 1j * ex[None, :]))
    return KS * dx, KD * dx


def s0_inverse(f, lx, h=None):
    """S0^-1 f: multiplier |k| / (pi (1 + exp(-2 |k| h))), zero at k = 0."""
    n = f.size
    ak = np.abs(2 * np.pi * np.fft.fftfreq(n, d=lx / n))
    eh = np.zeros(n) if is_deep(lx, h) else np.exp(-2 * ak * h)
    mult = np.where(ak > 0, ak / (np.pi * (1 + eh)), 0.0)
    return np.real(np.fft.ifft(mult * np.fft.fft(f)))


def vertical_velocity(eta, phi_s, lx, h=None, tol=1e-12, max_sweeps=64):
    """Fully nonlinear V at the grid points; returns (V, sweeps, status, residual)."""
    eta = np.asarray(eta, dtype=np.float64).ravel()
    phi = np.asarray(phi_s, dtype=np.float64).ravel()
    KS, KD = kernels(eta, lx, h)
    rhs = np.pi * phi + KD @ phi
    V = np.zeros_like(phi)
    rmin = math.inf
    r = 0.0
    for n in range(1, max_sweeps + 1):
        Vn = s0_inverse(rhs - KS @ V, lx, h)
        num = float(np.abs(Vn - V).max())
        den = float(np.abs(Vn).max())
        V = Vn
        if not (math.isfinite(num) and math.isfinite(den)):
            return V, n, -5, math.nan
        r = 0.0 if num == 0.0 else (num / den if den > 0 else math.inf)
        if r <= tol:
            return V, n, 0, r
        rmin = min(rmin, r)
        if r > 1e6 or (n - 1 >= 3 and r > 10.0 * rmin):
            return V, n, -6, r
    return V, max_sweeps, 1, r
