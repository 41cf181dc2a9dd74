"""Seeded input fields for the SBI wave solver (host side, numpy, FP64).

Every generator is deterministic given its arguments and seed
(``numpy.random.Generator(PCG64(seed))``).  Lengths are in units of 1/k_p and
times in units of 1/omega_p with g = 1, the non-dimensionalisation of Sec. 2.1.

Linear wave theory (dispersion omega^2 = k tanh(k h) and the linear surface
potential of a progressive wave) is used here only to *build* initial
conditions; the solver's own arithmetic lives elsewhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GridSpec:
    """Periodic collocation grid: ny == 1 means a 1D (x only) problem."""

    nx: int
    ny: int
    lx: float
    ly: float = 1.0
    dealias: float = 0.5

    @property
    def mx_max(self) -> int:
        """Largest kept |m_x|: strictly below dealias * nx / 2."""
        return int(math.ceil(self.dealias * self.nx / 2 - 1e-9)) - 1

    @property
    def my_max(self) -> int:
        return 0 if self.ny == 1 else int(math.ceil(self.dealias * self.ny / 2 - 1e-9)) - 1

    def x(self) -> np.ndarray:
        return np.arange(self.nx) * (self.lx / self.nx)

    def y(self) -> np.ndarray:
        if self.ny == 1:
            return np.zeros(1)
        return np.arange(self.ny) * (self.ly / self.ny)

    def kband(self) -> float:
        """Largest |k| of the retained (alias-free) rectangle."""
        kx = 2 * math.pi * self.mx_max / self.lx
        ky = 0.0 if self.ny == 1 else 2 * math.pi * self.my_max / self.ly
        return math.hypot(kx, ky)


def _dispersion_k(omega: float, h: float) -> float:
    """Solve omega^2 = k tanh(k h) for k (Newton, FP64)."""
    k = max(omega * omega, omega / math.sqrt(h))
    for _ in range(100):
        t = math.tanh(k * h)
        f = k * t - omega * omega
        df = t + k * h * (1 - t * t)
        dk = f / df
        k -= dk
        if abs(dk) < 1e-15 * k:
            break
    return k


def band_limited_random(grid: GridSpec, seed: int, amp: float = 1.0, slope: float = 2.0):
    """Smooth random real field inside the retained rectangle (for operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = grid.ny, grid.nx
    c = np.zeros((ny, nx), dtype=np.complex128)
    mx_max, my_max = grid.mx_max, grid.my_max
    for my in range(-my_max, my_max + 1):
        for mx in range(-mx_max, mx_max + 1):
            if mx == 0 and my == 0:
                continue
            r = math.hypot(mx, my)
            a = amp / (1.0 + r) ** slope
            ph = rng.uniform(0, 2 * math.pi)
            c[my % ny, mx % nx] += a * np.exp(1j * ph)
    f = np.real(np.fft.ifft2(c)) * (nx * ny)
    return f


def narrowband_random(grid: GridSpec, seed: int, amp: float = 1.0, k0: float = 1.0, width: float = 0.5):
    """Random real field inside the retained rectangle whose modal amplitudes
    fall off as exp(-((|k| - k0)/width)^2) around |k| = k0 (in 1/length units,
    so the content sits near k0 whatever the domain size), with uniform random
    phases; scaled so that max |f| = amp."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = grid.ny, grid.nx
    c = np.zeros((ny, nx), dtype=np.complex128)
    mx_max, my_max = grid.mx_max, grid.my_max
    for my in range(-my_max, my_max + 1):
        for mx in range(-mx_max, mx_max + 1):
            if mx == 0 and my == 0:
                continue
            kx = 2 * math.pi * mx / grid.lx
            ky = 0.0 if ny == 1 else 2 * math.pi * my / grid.ly
            a = math.exp(-((math.hypot(kx, ky) - k0) / width) ** 2)
            ph = rng.uniform(0, 2 * math.pi)
            c[my % ny, mx % nx] += a * np.exp(1j * ph)
    f = np.real(np.fft.ifft2(c))
    return f * (amp / np.abs(f).max())


def jonswap_crossing_sea(grid: GridSpec, h: float, seed: int, gamma: float = 3.3,
                         hs_half: float = 0.1, directions_deg=(20.0, -20.0), s: float = 10.0,
                         sigma_a: float = 0.07, sigma_b: float = 0.09):
    """Two JONSWAP wave systems crossing at the given mean directions.

    Each system has k_p H_s / 2 = ``hs_half`` (variance m0 = (H_s/4)^2), peak
    wavenumber k_p = 1, directional spreading D(theta) ~ cos^(2s)((theta-theta_m)/2),
    deterministic amplitudes sqrt(2 F dkx dky) and uniform random phases.
    Returns (eta, phi_s) with phi_s from linear theory; both band-limited to the
    retained rectangle of ``grid``.
    """
    if grid.ny == 1:
        raise ValueError("crossing seas need a 2D grid")
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny = grid.nx, grid.ny
    mx = np.arange(-grid.mx_max, grid.mx_max + 1)
    my = np.arange(-grid.my_max, grid.my_max + 1)
    MX, MY = np.meshgrid(mx, my)
    KX = 2 * math.pi * MX / grid.lx
    KY = 2 * math.pi * MY / grid.ly
    K = np.hypot(KX, KY)
    TH = np.arctan2(KY, KX)
    dkx = 2 * math.pi / grid.lx
    dky = 2 * math.pi / grid.ly
    valid = K > 0
    Ks = np.where(valid, K, 1.0)
    OM = np.sqrt(Ks * np.tanh(Ks * h))
    om_p = math.sqrt(math.tanh(h))
    # d omega / d k
    th = np.tanh(Ks * h)
    dOM = (th + Ks * h * (1 - th * th)) / (2 * OM)
    sig = np.where(OM <= om_p, sigma_a, sigma_b)
    r = np.exp(-((OM - om_p) ** 2) / (2 * sig * sig * om_p * om_p))
    S = OM ** -5.0 * np.exp(-1.25 * (om_p / OM) ** 4) * gamma ** r
    total_var = np.zeros_like(K)
    amps = np.zeros_like(K)
    m0 = (2 * hs_half / 4.0) ** 2
    for dth in directions_deg:
        thm = math.radians(dth)
        D = np.cos((TH - thm) / 2.0) ** (2 * s)
        # normalise D numerically over (-pi, pi]
        tt = np.linspace(-math.pi, math.pi, 20001)
        Dn = np.trapezoid(np.cos((tt - thm) / 2.0) ** (2 * s), tt)
        F = np.where(valid, S * dOM * D / Dn / Ks, 0.0)  # F(kx, ky)
        var = F * dkx * dky
        var *= m0 / var.sum()
        total_var += var
    amps = np.sqrt(2.0 * total_var)
    phases = rng.uniform(0.0, 2 * math.pi, size=K.shape)
    c_eta = np.zeros((ny, nx), dtype=np.complex128)
    c_phi = np.zeros((ny, nx), dtype=np.complex128)
    A = amps * np.exp(1j * phases)
    A = np.where(valid, A, 0.0)
    c_eta[MY % ny, MX % nx] = A
    c_phi[MY % ny, MX % nx] = np.where(valid, -1j * A / OM, 0.0)
    eta = np.real(np.fft.ifft2(c_eta)) * (nx * ny)
    phi = np.real(np.fft.ifft2(c_phi)) * (nx * ny)
    return eta, phi


def stokes2_finite_depth(grid: GridSpec, a: float, h: float, k0: float = 1.0, x0: float = 0.0):
    """Second-order finite-depth Stokes wave (textbook), evaluated at z = eta.

    Returns (eta, phi_s, omega).  phi_s is the second-order potential evaluated
    exactly at the surface elevation, used as given data.
    """
    x = grid.x() - x0
    th = k0 * x
    kh = k0 * h
    om = math.sqrt(k0 * math.tanh(kh))
    c2 = k0 * a * a / 4.0 * math.cosh(kh) * (2 + math.cosh(2 * kh)) / math.sinh(kh) ** 3
    eta = a * np.cos(th) + c2 * np.cos(2 * th)
    z = eta
    phi = (a * om / k0) * np.cosh(k0 * (z + h)) / math.sinh(kh) * np.sin(th) \
        + 3.0 / 8.0 * a * a * om * np.cosh(2 * k0 * (z + h)) / math.sinh(kh) ** 4 * np.sin(2 * th)
    return eta[None, :].copy(), phi[None, :].copy(), om


def stokes3_deep(grid: GridSpec, a: float, k0: float = 1.0, x0: float = 0.0):
    """Third-order deep-water Stokes wave: (eta, phi_s, omega, celerity)."""
    x = grid.x() - x0
    th = k0 * x
    eta = a * (np.cos(th) + 0.5 * k0 * a * np.cos(2 * th) + 3.0 / 8.0 * (k0 * a) ** 2 * np.cos(3 * th))
    om = math.sqrt(k0) * (1 + 0.5 * (k0 * a) ** 2)
    phi = (a * om / k0) * np.exp(k0 * eta) * np.sin(th)
    return eta[None, :].copy(), phi[None, :].copy(), om, om / k0


def gaussian_bump_depth(grid: GridSpec, h0: float, height: float, xc: float, fwhm: float):
    x = grid.x()
    d = h0 - height * np.exp(-4.0 * math.log(2.0) * (x - xc) ** 2 / fwhm ** 2)
    return np.repeat(d[None, :], grid.ny, axis=0)


def trapezoid_bar_depth(grid: GridSpec, h0: float, crest_depth: float, x_start: float,
                        up_slope: float = 1 / 20, down_slope: float = 1 / 10, crest_len: float | None = None):
    """Submerged trapezoidal bar: 1:20 rise to the crest, flat crest, 1:10 fall."""
    if crest_len is None:
        crest_len = 5.0 * h0
    rise = h0 - crest_depth
    x = grid.x()
    x1 = x_start + rise / up_slope
    x2 = x1 + crest_len
    x3 = x2 + rise / down_slope
    d = np.full_like(x, h0)
    m = (x >= x_start) & (x < x1)
    d[m] = h0 - up_slope * (x[m] - x_start)
    m = (x >= x1) & (x < x2)
    d[m] = crest_depth
    m = (x >= x2) & (x < x3)
    d[m] = crest_depth + down_slope * (x[m] - x2)
    return np.repeat(d[None, :], grid.ny, axis=0)


def undulating_bars_depth(grid: GridSpec, h0: float, n_bars: int, amp: float):
    x = grid.x()
    delta = amp * (1.0 - np.cos(2 * math.pi * n_bars * x / grid.lx)) / 2.0
    return np.repeat((h0 - delta)[None, :], grid.ny, axis=0)


def random_bumps_depth(grid: GridSpec, h_ref: float, seed: int, n_min: int = 3, n_max: int = 8,
                       max_rel_height: float = 0.25, kdelta_max: float = 2.4):
    """3-8 Gaussian bumps, heights <= 0.25 h_ref, shrunk so k_band * max(delta) <= 2.4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = int(rng.integers(n_min, n_max + 1))
    X, Y = np.meshgrid(grid.x(), grid.y())
    delta = np.zeros((grid.ny, grid.nx))
    for _ in range(nb):
        xc = rng.uniform(0, grid.lx)
        yc = rng.uniform(0, grid.ly)
        hb = rng.uniform(0.3, 1.0) * max_rel_height * h_ref
        w = rng.uniform(0.05, 0.2) * min(grid.lx, grid.ly)
        dx = (X - xc + grid.lx / 2) % grid.lx - grid.lx / 2
        dy = (Y - yc + grid.ly / 2) % grid.ly - grid.ly / 2
        delta += hb * np.exp(-(dx * dx + dy * dy) / (w * w))
    dmax = delta.max()
    lim = kdelta_max / grid.kband()
    if dmax > lim:
        delta *= lim / dmax
    dmax = delta.max()
    if dmax > max_rel_height * h_ref:
        delta *= max_rel_height * h_ref / dmax
    return h_ref - delta


# ---------------------------------------------------------------------------
# Workload configurations (shapes and distributions of the paper's cases)
# ---------------------------------------------------------------------------

def config_c1():
    """1D N=256, 8 wavelengths, k0 h0 = 1, Gaussian bump 0.3 h0 (FWHM one
    wavelength), 2nd-order Stokes k0 a = 0.05; dt = T/64 for 10 periods."""
    lam = 2 * math.pi
    g = GridSpec(nx=256, ny=1, lx=8 * lam)
    h0 = 1.0
    depth = gaussian_bump_depth(g, h0, 0.3 * h0, g.lx / 2, lam)
    eta, phi, om = stokes2_finite_depth(g, 0.05, h0)
    T = 2 * math.pi / om
    return dict(grid=g, depth=depth, eta=eta, phi=phi, dt=T / 64, steps=640, period=T,
                mode="iter", tol=1e-10, precision="fp64", h_ref=h0)


def c2_wave(case: int):
    """Incident regular waves of the submerged-bar case (0.4 Hz / 1.0 Hz at
    h0 = 0.4 m), non-dimensionalised by their own wavenumber."""
    g_dim = 9.81
    h0_dim = 0.4
    f = {1: 0.4, 2: 1.0}[case]
    om = 2 * math.pi * f
    k = _dispersion_k(om / math.sqrt(g_dim), h0_dim)  # solves (om^2/g) = k tanh(k h)
    kh = k * h0_dim
    ka = {1: 0.02, 2: 0.1}[case]
    return kh, ka


def config_c2(case: int = 1, nx: int = 4096, steps: int = 20000):
    """1D submerged trapezoidal bar, N=4096, domain 160 h0; relaxation-zone
    generation of a regular wave; paper's plain (successive) method."""
    kh, ka = c2_wave(case)
    h0 = kh  # k0 = 1
    L = 160.0 * h0
    g = GridSpec(nx=nx, ny=1, lx=L)
    depth = trapezoid_bar_depth(g, h0, 0.33 * h0, x_start=0.3 * L)
    om = math.sqrt(math.tanh(h0))
    T = 2 * math.pi / om
    eta = np.zeros((1, nx))
    phi = np.zeros((1, nx))
    lam = 2 * math.pi
    relax = dict(a=ka, k=1.0, omega=om, gen_len=2 * lam, abs_len=3 * lam, ramp_periods=3.0)
    # the low-pass filter the paper applies at every step of its tank runs
    # (beta1 = 8, beta2 = 30, wavenumbers in units of the incident one)
    return dict(grid=g, depth=depth, eta=eta, phi=phi, dt=T / 64, steps=steps, period=T,
                mode="sa", tol=0.0, precision="fp64", h_ref=h0, relax=relax, filter_beta=(8.0, 30.0))


def config_c3(seed: int = 3, n: int = 512):
    """2D crossing seas, 512^2, 32 peak wavelengths, flat k_p h = 3."""
    lam = 2 * math.pi
    g = GridSpec(nx=n, ny=n, lx=32 * lam * n / 512, ly=32 * lam * n / 512)
    h = 3.0
    eta, phi = jonswap_crossing_sea(g, h, seed)
    depth = np.full((n, n), h)
    Tp = 2 * math.pi / math.sqrt(math.tanh(h))
    return dict(grid=g, depth=depth, eta=eta, phi=phi, dt=Tp / 64, steps=6400, period=Tp,
                mode="sa", tol=0.0, precision="fp32", h_ref=h)


def config_c4_member(member: int):
    """Ragged ensemble member: seeds 0-31 at 128^2, 32-79 at 256^2, 80-95 at 512^2;
    dx = lambda_p/16; undulating bars (4-12 bars, amplitude 0.1-0.25 h0)."""
    if member < 32:
        n = 128
    elif member < 80:
        n = 256
    else:
        n = 512
    lam = 2 * math.pi
    L = n / 16 * lam
    g = GridSpec(nx=n, ny=n, lx=L, ly=L)
    h0 = 3.0
    rng = np.random.Generator(np.random.PCG64(10_000 + member))
    nb = int(rng.integers(4, 13))
    amp = rng.uniform(0.1, 0.25) * h0
    depth = undulating_bars_depth(g, h0, nb, amp)
    eta, phi = jonswap_crossing_sea(g, h0, member)
    Tp = 2 * math.pi / math.sqrt(math.tanh(h0))
    return dict(grid=g, depth=depth, eta=eta, phi=phi, dt=Tp / 64, steps=64, period=Tp,
                mode="sa", tol=0.0, precision="fp32", h_ref=h0, n_bars=nb, amp=amp)


def config_c5(seed: int = 0, n: int = 1024, wavelengths: float = 128.0):
    """2D 1024^2 crossing seas over random Gaussian bumps, k_p h_ref in 0.8-3."""
    lam = 2 * math.pi
    L = wavelengths * lam * n / 1024
    g = GridSpec(nx=n, ny=n, lx=L, ly=L)
    rng = np.random.Generator(np.random.PCG64(20_000 + seed))
    h_ref = float(rng.uniform(0.8, 3.0))
    depth = random_bumps_depth(g, h_ref, 30_000 + seed)
    eta, phi = jonswap_crossing_sea(g, h_ref, seed)
    Tp = 2 * math.pi / math.sqrt(math.tanh(1.0 * h_ref))
    return dict(grid=g, depth=depth, eta=eta, phi=phi, dt=Tp / 64, steps=32, period=Tp,
                mode="iter", tol=1e-8, precision="fp64", h_ref=h_ref)
