"""Steady periodic water waves by the stream-function method (after Fenton,
"The numerical solution of steady water wave problems", 1988), used as exact
solutions of the full potential-flow problem against which the surface
vertical velocity of the accuracy studies of Sec. 4 (deep water) and Sec. 5
(finite depth) is checked.  TEST INFRASTRUCTURE ONLY (like the rest of
``oracle/``).

Units g = 1, wavenumber k = 1 (wavelength 2 pi).  In the frame moving with the
wave the flow is steady, with stream function

    psi(x, z) = -c z + sum_{j=1}^{N} B_j Z_j(z) cos(j x),
    Z_j = exp(j z) (deep water),  sinh(j (z + d)) / cosh(j d) (depth d),

which is harmonic, tends to the uniform stream -c at depth, and in finite
depth makes the bed z = -d a streamline.  Unknowns: the
surface eta_m at x_m = m pi / N (m = 0..N, crest at x = 0, symmetric), B_j,
the speed c, the surface stream value Q and the Bernoulli constant R.
Equations: the surface is the streamline psi = Q, Bernoulli's condition
(u^2 + w^2)/2 + eta = R holds there, the mean level is zero and the crest-to-
trough height is H.  Newton's method with exact (complex-step) derivatives,
continued in H from the linear wave.

In the fixed frame the potential is phi = sum_j B_j C_j(z) sin(j (x - c t)),
C_j = exp(j z) or cosh(j (z + d)) / cosh(j d), so at t = 0 the surface
potential is phi_s(x) = sum_j B_j C_j(eta) sin(j x) and the surface vertical
velocity V = phi_z - eta_x phi_x equals -c eta_x (the wave translates rigidly).
"""
from __future__ import annotations

import math

import numpy as np


class SteadyWave:
    def __init__(self, H: float, N: int = 32, steps: int = 12, tol: float = 1e-12, max_newton: int = 40,
                 depth: float | None = None):
        self.N = int(N)
        self.H = float(H)
        self.d = None if depth is None else float(depth)
        self.x = np.arange(self.N + 1) * math.pi / self.N
        z = self._linear(self.H / steps)
        for s in range(1, steps + 1):
            z = self._newton(z, self.H * s / steps, tol, max_newton)
        self.z = z
        n = self.N
        self.eta = z[:n + 1].real.copy()
        self.B = z[n + 1:2 * n + 1].real.copy()
        self.c, self.Q, self.R = (float(v.real) for v in z[2 * n + 1:])

    # unknown vector [eta_0..eta_N, B_1..B_N, c, Q, R]
    def _linear(self, H):
        n = self.N
        t = 1.0 if self.d is None else math.tanh(self.d)
        c = math.sqrt(t)
        z = np.zeros(2 * n + 4, dtype=complex)
        z[:n + 1] = 0.5 * H * np.cos(self.x)
        z[n + 1] = 0.5 * H * c / t     # surface streamline of the linear wave: B_1 Z_1(0) = c H / 2
        z[2 * n + 1] = c
        z[2 * n + 3] = 0.5 * c * c     # R = c^2 / 2
        return z

    def _basis(self, eta, j):
        """Z_j(eta) and its z-derivative over j (so u, w take j B_j factors): (S, C) with
        Z_j = S, dZ_j/dz / j = C (deep: both exp(j eta))."""
        je = np.outer(eta, j)
        if self.d is None:
            e = np.exp(je)
            return e, e
        jd = j * self.d
        # sinh(j(eta+d))/cosh(jd), cosh(j(eta+d))/cosh(jd), written with exponentials that do not overflow
        ep = np.exp(je)                                   # e^{j eta}
        em = np.exp(-je - 2.0 * jd[None, :])              # e^{-j eta - 2 j d}
        den = 1.0 + np.exp(-2.0 * jd)[None, :]            # 2 cosh(jd) e^{-jd}
        return (ep - em) / den, (ep + em) / den

    def residual(self, z, H):
        n = self.N
        eta = z[:n + 1]
        B = z[n + 1:2 * n + 1]
        c, Q, R = z[2 * n + 1], z[2 * n + 2], z[2 * n + 3]
        j = np.arange(1, n + 1)
        Zs, Zc = self._basis(eta, j)                      # Z_j(eta_m), Z_j'(eta_m) / j
        C = np.cos(np.outer(self.x, j))
        S = np.sin(np.outer(self.x, j))
        psi = -c * eta + (Zs * C) @ B
        u = -c + (Zc * C) @ (j * B)
        w = (Zs * S) @ (j * B)
        f1 = psi - Q
        f2 = 0.5 * (u * u + w * w) + eta - R
        f3 = (0.5 * eta[0] + eta[1:n].sum() + 0.5 * eta[n]) / n   # mean level (trapezoid)
        f4 = eta[0] - eta[n] - H
        return np.concatenate([f1, f2, [f3, f4]])

    def _newton(self, z, H, tol, max_newton):
        m = z.size
        hstep = 1e-30
        for _ in range(max_newton):
            f = self.residual(z, H).real
            if np.abs(f).max() < tol:
                return z
            J = np.empty((m, m))
            for i in range(m):
                zp = z.copy()
                zp[i] += 1j * hstep
                J[:, i] = self.residual(zp, H).imag / hstep
            z = z - np.linalg.solve(J, f)
        r = np.abs(self.residual(z, H).real)
        if not np.all(np.isfinite(r)) or r.max() > 1e3 * tol:
            raise RuntimeError("steady-wave Newton iteration did not converge")
        return z

    # -- the solution anywhere on the surface ---------------------------------
    def _eta_coeffs(self):
        """Cosine-series coefficients of eta from its values at x_m (DCT-I)."""
        n = self.N
        w = np.ones(n + 1)
        w[0] = w[n] = 0.5
        jm = np.outer(np.arange(n + 1), np.arange(n + 1)) * math.pi / n
        E = (2.0 / n) * (np.cos(jm) @ (w * self.eta))
        E[0] *= 0.5
        E[n] *= 0.5
        return E

    def surface(self, x):
        """(eta, eta_x, phi_s, V) at points x (fixed frame, t = 0)."""
        x = np.asarray(x, dtype=np.float64)
        E = self._eta_coeffs()
        jj = np.arange(self.N + 1)
        eta = np.cos(np.outer(x, jj)) @ E
        eta_x = -(np.sin(np.outer(x, jj)) * jj) @ E
        j = np.arange(1, self.N + 1)
        Zs, Zc = self._basis(eta, j)
        # phi = sum B_j Zc_j sin(jx): phi_x = sum j B_j Zc_j cos(jx), phi_z = sum j B_j Zs_j sin(jx)
        phi = (Zc * np.sin(np.outer(x, j))) @ self.B
        phi_x = (Zc * np.cos(np.outer(x, j))) @ (j * self.B)
        phi_z = (Zs * np.sin(np.outer(x, j))) @ (j * self.B)
        V = phi_z - eta_x * phi_x
        return eta, eta_x, phi, V
