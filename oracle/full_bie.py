"""FP64 oracle of the fully nonlinear W solve on one-dimensional grids: the
boundary-integral equations of Sec. 2.3 with the remaining integrals I^(S) of
App. A (and, over a variable bed, I^(B) of App. B) kept.  TEST
INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

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

Over a variable bed z = -h + delta(x) the image no longer applies:
vertical_velocity_bed keeps the bed as a second boundary, with the potential
phi_b on it as a second unknown (the paper's bed equation, whose remainder is
I^(B)); see there.

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


def bed_kernels(eta, b, lx):
    """Quadrature matrices of the two-boundary equations, surface z = eta(x),
    bed z = b(x) (rows: evaluation point x_i, columns: source x_j; trapezoidal
    weight dx included): the single layer of the surface seen from the bed
    (SBS), the double layers of the surface seen from the bed (DBS), of the bed
    seen from the surface (DSB) and of the bed on itself (DBB).  The outward
    normal is (-eta_x, 1) ds/dx at the surface and (b_x, -1) ds/dx at the bed;
    with c = (pi / L) cot(pi (z_q - z_p) / L) for a source q and evaluation
    point p, the normal derivative of G at the source times ds/dx is
    Im(c (1 + i eta_x)) on the surface and -Im(c (1 + i b_x)) on the bed.  Only
    DBB has coincident points; its diagonal is the curvature limit
    -b_xx / (2 (1 + b_x^2)).  The bed lies below the surface, so every other
    kernel is smooth."""
    n = eta.size
    dx = lx / n
    x = np.arange(n) * dx
    ex, _ = spectral_derivatives(eta, lx)
    bx, bxx = spectral_derivatives(b, lx)
    zs = x + 1j * eta
    zb = x + 1j * b
    dxm = x[:, None] - x[None, :]
    s2 = np.sin(np.pi * dxm / lx) ** 2
    # G(p on the bed, q on the surface) = -1/2 ln(4 (sin^2(pi dx / L) + sinh^2(pi dz / L)))
    SBS = -0.5 * np.log(4.0 * (s2 + np.sinh(np.pi * (b[:, None] - eta[None, :]) / lx) ** 2))
    pl = np.pi / lx
    DBS = np.imag(pl * _cot(pl * (zs[None, :] - zb[:, None])) * (1 + 1j * ex[None, :]))
    DSB = -np.imag(pl * _cot(pl * (zb[None, :] - zs[:, None])) * (1 + 1j * bx[None, :]))
    off = ~np.eye(n, dtype=bool)
    u = zb[None, :] - zb[:, None]
    DBB = np.empty((n, n))
    DBB[off] = -np.imag(pl * _cot(pl * u[off]) * (1 + 1j * np.broadcast_to(bx[None, :], (n, n))[off]))
    DBB[~off] = -bxx / (2.0 * (1.0 + bx ** 2))
    return SBS * dx, DBS * dx, DSB * dx, DBB * dx


def s_image(f, lx, h):
    """(S0 - S_flat) f: multiplier (pi / |k|) exp(-2 |k| h), zero at k = 0 --
    what the flat bed adds to the single layer of the flat surface."""
    n = f.size
    ak = np.abs(2 * np.pi * np.fft.fftfreq(n, d=lx / n))
    mult = np.where(ak > 0, np.pi / np.where(ak > 0, ak, 1.0) * np.exp(-2 * ak * h), 0.0)
    return np.real(np.fft.ifft(mult * np.fft.fft(f)))


def vertical_velocity_bed(eta, phi_s, lx, h, delta, tol=1e-12, max_sweeps=64):
    """Fully nonlinear V over a variable bed z = -h + delta(x) (the remaining
    integrals I^(S) and I^(B) of App. A and App. B kept), from the surface and
    bed equations of Green's identity in two dimensions (no image):

        S[V] = pi phi_s + D_SS[phi_s] + D_SB[phi_b]           (surface points)
        pi phi_b = S_BS[V] - D_BS[phi_s] - D_BB[phi_b]         (bed points)

    (dphi/dn = 0 on the bed; phi_b the potential there).  A sweep updates
    phi_b from the bed equation with the current V, then V with the flat
    preconditioner S0 of the image form (the single layer of the flat surface
    over the flat bed z = -h, which is S_flat minus the bed's response
    D_SB S_BS / pi at flat geometry):

        phi_b <- (S_BS[V] - D_BS[phi_s] - D_BB[phi_b]) / pi
        V <- S0^-1 [ pi phi_s + D_SS[phi_s] + D_SB[phi_b] - (S - S_flat)[V]
                     + (S0 - S_flat)[V] ]

    from V = phi_b = 0; over flat geometry the first sweep is exact.  Stopping
    rules as in vertical_velocity.  Returns (V, sweeps, status, residual)."""
    eta = np.asarray(eta, dtype=np.float64).ravel()
    phi = np.asarray(phi_s, dtype=np.float64).ravel()
    delta = np.asarray(delta, dtype=np.float64).ravel()
    b = -h + delta
    KS, KD = kernels(eta, lx, None)
    SBS, DBS, DSB, DBB = bed_kernels(eta, b, lx)
    rhs_s = np.pi * phi + KD @ phi
    rhs_b = -(DBS @ phi)
    V = np.zeros_like(phi)
    pb = np.zeros_like(phi)
    rmin = math.inf
    r = 0.0
    for n in range(1, max_sweeps + 1):
        pb = (SBS @ V + rhs_b - DBB @ pb) / np.pi
        Vn = s0_inverse(rhs_s + DSB @ pb - KS @ V + s_image(V, lx, h), lx, h)
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
