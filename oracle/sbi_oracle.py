"""Plain FP64 oracle of the SBI wave solver (numpy).  TEST INFRASTRUCTURE ONLY.

Notation follows the paper: eta (surface elevation), phi_s (surface potential,
"phi tilde"), phi_b (bottom potential, "varphi tilde"), V (surface vertical
velocity), h (reference depth), delta (seabed variation; seabed at z=-h+delta),
T = tanh(kh), S = sech(kh).  Fourier transform: forward exp(-i k.x)
unnormalised, inverse 1/N (Sec. 2.2); numpy's pocketfft serves as the FFT
primitive and is pinned against a brute-force DFT in the tests.

Readings of the paper that this oracle fixes (each also listed in the design
notes of the repository):

* dealiasing ("2/(l+1) rule", Sec. 2.4): keep |m_x| < alpha nx/2 and
  |m_y| < alpha ny/2 with alpha = 1/2 (the submerged-bar case of Sec. 3.2 calls
  waves longer than L/(N/4) alias-free; Sec. 4 keeps "the first 16 modes" of 64
  points); applied to the spectrum of every product and to the state;
* the explicit orders of Appendix C, Eqs. (v2)-(v7), are authoritative where
  the general recursion of Sec. 2.4 differs from them;
* the iteration mode solves the fixed point of the recursion summed over
  orders (same expansion, J = L-1 convolution orders in both equations);
* time stepping is Lawson integrating-factor RK4 on the integrating-factor
  form of Eq. (prognostic) with omega = sqrt(k tanh(kh));
* the adaptive step of Sec. 2.2 (a six-stage fifth-order pair with an
  embedded fourth-order solution, coefficients not printed) uses the
  Cash-Karp pair in the same Lawson form; the "difference between the fifth-
  and fourth-order solutions" is measured in the linear-energy norm relative
  to the new state, and the step size follows the standard controller
  h <- h min(5, max(0.2, 0.9 (tol/err)^(1/5))) (no growth right after a
  rejection; rejected when err > tol);
* the wave tank's surface pressure p = p_g + p_d enters the dynamic surface
  condition as phi_t = ... - eta - p (the sign under which the generator's
  prefactor yields waves of amplitude a_j); the bell of p_g is centred on
  x = 0 (split over both ends of the periodic domain), the damping weight
  exp(-((x - x0)/w)^2) uses the periodic distance, w = 4 pi by default, and
  p_d's k = 0 mode is zero;
* the Anderson-accelerated iteration (an option of the build, not the
  paper's) mixes the relaxed sweep over the last two residual differences,
  with the residual, stopping rules and fixed point of the relaxed sweeps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# status codes (same meaning as the C interface)
OK = 0
WARN_NOT_CONVERGED = 1
WARN_DEPTH_CRITERION = 2
WARN_STEP_LIMIT = 4
ERR_NONFINITE = -5
ERR_DIVERGED = -6


class Grid:
    """Periodic grid, rfft2 half-spectrum layout (ny, nx//2+1)."""

    def __init__(self, nx: int, ny: int, lx: float, ly: float = 1.0, dealias: float = 0.5):
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        mx = np.arange(self.nx // 2 + 1)
        my = np.fft.fftfreq(self.ny, 1.0 / self.ny) if self.ny > 1 else np.zeros(1)
        self.kx = (2 * np.pi * mx / self.lx)[None, :]
        self.ky = (2 * np.pi * my / self.ly)[:, None] if self.ny > 1 else np.zeros((1, 1))
        self.k = np.sqrt(self.kx ** 2 + self.ky ** 2)
        # kept modes: |m| strictly below alpha*n/2 (alpha = 1/2: waves longer than
        # 4 grid spacings, Sec. 3.2; "the first 16 modes" of 64 points, Sec. 4)
        self.Mx = int(math.ceil(dealias * self.nx / 2 - 1e-9)) - 1
        self.My = 0 if self.ny == 1 else int(math.ceil(dealias * self.ny / 2 - 1e-9)) - 1
        keep = (mx[None, :] <= self.Mx) & (np.abs(my)[:, None] <= self.My)
        self.mask = keep.astype(np.float64)
        self.dA = (self.lx / self.nx) * ((self.ly / self.ny) if self.ny > 1 else 1.0)
        self.kband = math.hypot(2 * np.pi * self.Mx / self.lx,
                                (2 * np.pi * self.My / self.ly) if self.ny > 1 else 0.0)

    # transforms -----------------------------------------------------------
    def fft(self, f):
        return np.fft.rfft2(np.asarray(f, dtype=np.float64))

    def ifft(self, F):
        return np.fft.irfft2(F, s=(self.ny, self.nx))

    def MF(self, f):
        """Masked forward transform of a (product) field."""
        return self.mask * self.fft(f)

    def grad(self, F):
        """Physical gradient of the field whose spectrum is F."""
        gx = self.ifft(1j * self.kx * F)
        gy = self.ifft(1j * self.ky * F) if self.ny > 1 else None
        return gx, gy

    def ikdot(self, Fx, Fy):
        """ik . (Fx, Fy) in spectral space."""
        out = 1j * self.kx * Fx
        if Fy is not None:
            out = out + 1j * self.ky * Fy
        return out


def _sech(x):
    e = np.exp(-np.abs(x))
    return 2.0 * e / (1.0 + e * e)


@dataclass
class SolveInfo:
    sweeps: int = 0
    residual: float = 0.0
    status: int = OK
    omega: float = 1.0
    history: list = field(default_factory=list)
    fallback: bool = False


class Solver:
    """W solve (successive approximation / iteration) and IF-RK4 time step."""

    def __init__(self, grid: Grid, depth, h_ref: float | None = None, order: int = 7,
                 mode: str = "iter", max_sweeps: int = 64, relax: bool = True,
                 filter_beta=None, relaxation_zone=None, seed: str = "linear", net=None, wavemaker=None,
                 accel: str | None = None, aa_depth: int = 2, hist=None):
        self.g = grid
        depth = np.asarray(depth, dtype=np.float64).reshape(grid.ny, grid.nx)
        if np.any(~np.isfinite(depth)) or np.any(depth <= 0):
            raise ValueError("depth must be finite and positive")
        self.h = float(depth.max()) if (h_ref is None or h_ref <= 0) else float(h_ref)
        # seabed at z = -h + delta  (Sec. 2.1)
        self.delta = self.h - depth
        self.flat = not np.any(self.delta != 0.0)
        self.L = int(order)
        if not 1 <= self.L <= 7:
            raise ValueError("order must be in 1..7")
        self.mode = mode
        if mode not in ("sa", "iter", "full"):
            raise ValueError("mode must be 'sa', 'iter' or 'full'")
        if mode == "full" and grid.ny != 1:
            # the exact boundary-integral solve (oracle.full_bie) covers one
            # horizontal dimension
            raise ValueError("mode 'full' needs a one-dimensional grid")
        self.max_sweeps = int(max_sweeps)
        self.relax = relax
        k = grid.k
        kh = k * self.h
        self.T = np.tanh(kh)
        self.S = _sech(kh)
        self.om2 = k * self.T              # omega^2 = k tanh(kh)
        self.om = np.sqrt(self.om2)
        self.filter_beta = filter_beta
        self.rz = relaxation_zone
        # numerical wave tank of Sec. 3.2: pneumatic wavemaker p_g and damping
        # pressure p_d (Eq. pd) acting on the surface.  wavemaker = dict(
        #   comps=[(a_j, k_j, omega_j, theta_j), ...]  (p_g components; may be empty),
        #   h=depth in the generator's factor (default h_ref),
        #   x0=centre of the damping weight (None: no damping), width=its length (default 4 pi))
        self.wm = wavemaker
        # acceleration of the iteration: None (relaxed sweeps) or "anderson"
        # (Anderson mixing of the relaxed sweep over the last aa_depth differences)
        if accel not in (None, "anderson"):
            raise ValueError("accel must be None or 'anderson'")
        self.accel = accel
        self.aa_depth = int(aa_depth)
        # seed of the iteration:
        #   "linear": the initiation of Sec. 2.4;
        #   "prev":   the linear guess plus the nonlinear part left by this
        #             solver's previous solve, (V* - kT phi_hat, phi_b - S phi_hat);
        #   "net":    the learned warm start (oracle.warmstart) with net =
        #             (theta, in_scale, out_scale): the linear guess plus the
        #             network's corrections (nV, nB) when there is no previous
        #             solve to start from, else the "prev" seed; a failed solve
        #             from the network's seed is redone from the linear guess.
        if seed not in ("linear", "prev", "net"):
            raise ValueError("seed must be 'linear', 'prev' or 'net'")
        #   with hist = (K, nb, dk, theta): the learned history seed of
        #             oracle.history_seed for fixed-step solves that have K
        #             earlier fixed-step solves behind them (seed "net" only).
        if seed == "net" and net is None and hist is None:
            raise ValueError("seed 'net' needs the network (theta, in_scale, out_scale) or the history layer")
        self.seed = seed
        self.net = net
        self._prev = None
        self.hist = None
        if hist is not None:
            from . import history_seed as hs
            K, nb, dk, theta = hist
            self.hist = dict(K=int(K), nb=int(nb), dk=float(dk), theta=np.asarray(theta, dtype=np.float32).copy(),
                             b=hs.bins(grid, float(dk), int(nb)), c=hs.mode_weights(grid))
        self._hist = []           # nonlinear parts (N_V, N_B) of the last fixed-step solves, newest first
        self.hist_train = False   # accumulate the history layer's loss gradient over fixed-step solves
        self._hist_acc = None     # sums over solves: grad (2, 4, nb, K), gram (2, 4, nb, K, K), loss, samples
        self._hist_adam = None    # [m, v, step]
        # depth-validity criterion of Sec. 5: k |delta| < 2.4 at the largest wavenumber
        self.depth_warning = grid.kband * float(np.abs(self.delta).max()) > 2.4

    # helpers ---------------------------------------------------------------
    def Tn(self, n):
        """tanh^<n/2>(kh): T for odd n, 1 for even n (Sec. 2.4)."""
        return self.T if (n % 2) else 1.0

    def kpow(self, p):
        """k^p with the k = 0 mode set to 0 for p < 0 (every such term carries ik)."""
        k = self.g.k
        if p >= 0:
            return k ** p
        with np.errstate(divide="ignore"):
            out = np.where(k > 0, k ** float(p), 0.0)
        return out

    # ------------------------------------------------------------------------
    # Successive approximation, paper-exact (Sec. 2.4, Appendix C)
    # ------------------------------------------------------------------------
    def w_sa_hat(self, eta, ph):
        """Spectrum of V = sum_{l=1}^{L} V_l for masked potential spectrum ph.

        Order recursion in the form of Appendix C: for 2 <= l <= L,
          F{V_l}   = sum_j [ -T_j k^j/j! MF{eta^j V_{l-j}}
                              + <j> S k^(j-1)/j! ik.MF{delta^j grad phi_b,l-j} ]
                     - T_l k^(l-2)/(l-1)! ik.MF{eta^(l-1) grad phi_s}
          F{phi_b,l} = sum_j [ -<j> S k^(j-1)/j! MF{eta^j V_{l-j}}
                              + (-1)^j T_j k^(j-2)/j! ik.MF{delta^j grad phi_b,l-j} ]
                     - <l> S k^(l-3)/(l-1)! ik.MF{eta^(l-1) grad phi_s}
        with V_1 = k T phi_hat and phi_b,1 = S phi_hat; phi_b only to order L-1.
        """
        g, k, S, L = self.g, self.g.k, self.S, self.L
        gpx, gpy = g.grad(ph)
        Vh = {1: k * self.T * ph}
        Bh = {1: S * ph}
        Vp = {1: g.ifft(Vh[1])}
        gB = {1: g.grad(Bh[1])}
        for l in range(2, L + 1):
            acc = np.zeros_like(ph)
            accB = np.zeros_like(ph)
            for j in range(1, l):
                fj = math.factorial(j)
                P = g.MF(eta ** j * Vp[l - j])
                acc = acc - self.Tn(j) * k ** j / fj * P
                accB = accB - (j % 2) * S * self.kpow(j - 1) / fj * P
                if not self.flat:
                    bx, by = gB[l - j]
                    D = g.ikdot(g.MF(self.delta ** j * bx),
                                g.MF(self.delta ** j * by) if by is not None else None)
                    acc = acc + (j % 2) * S * self.kpow(j - 1) / fj * D
                    accB = accB + (-1) ** j * self.Tn(j) * self.kpow(j - 2) / fj * D
            fl = math.factorial(l - 1)
            Fl = g.ikdot(g.MF(eta ** (l - 1) * gpx),
                         g.MF(eta ** (l - 1) * gpy) if gpy is not None else None)
            acc = acc - self.Tn(l) * self.kpow(l - 2) / fl * Fl
            accB = accB - (l % 2) * S * self.kpow(l - 3) / fl * Fl
            Vh[l] = acc
            Vp[l] = g.ifft(acc)
            if l <= L - 1:
                Bh[l] = accB
                gB[l] = g.grad(accB)
        return sum(Vh[l] for l in range(1, L + 1))

    # ------------------------------------------------------------------------
    # Iteration on the summed operator (fixed point of the same expansion)
    # ------------------------------------------------------------------------
    def forcing(self, eta, ph):
        """Constant parts (b_V, b_phi) of the summed operator."""
        g, k, S, L = self.g, self.g.k, self.S, self.L
        gpx, gpy = g.grad(ph)
        bV = k * self.T * ph
        bB = S * ph
        for l in range(2, L + 1):
            fl = math.factorial(l - 1)
            Fl = g.ikdot(g.MF(eta ** (l - 1) * gpx),
                         g.MF(eta ** (l - 1) * gpy) if gpy is not None else None)
            bV = bV - self.Tn(l) * self.kpow(l - 2) / fl * Fl
            bB = bB - (l % 2) * S * self.kpow(l - 3) / fl * Fl
        return bV, bB

    def apply_T(self, eta, bV, bB, Vh, Bh):
        """One sweep (V', phi_b') = T(V, phi_b) of the summed operator, J = L-1."""
        g, k, S = self.g, self.g.k, self.S
        J = self.L - 1
        V = g.ifft(Vh)
        bx, by = g.grad(Bh)
        Vn = bV.copy()
        Bn = bB.copy()
        for j in range(1, J + 1):
            fj = math.factorial(j)
            P = g.MF(eta ** j * V)
            Vn = Vn - self.Tn(j) * k ** j / fj * P
            Bn = Bn - (j % 2) * S * self.kpow(j - 1) / fj * P
            if not self.flat:
                D = g.ikdot(g.MF(self.delta ** j * bx),
                            g.MF(self.delta ** j * by) if by is not None else None)
                Vn = Vn + (j % 2) * S * self.kpow(j - 1) / fj * D
                Bn = Bn + (-1) ** j * self.Tn(j) * self.kpow(j - 2) / fj * D
        return Vn, Bn

    def relax_factor(self, eta):
        """Relaxation weight from the local symbol of the sweep (truncated exp).

        lambda(x) = sum_{j<=J} x^j/j!, x = k_band * eta at the highest crest and
        the deepest trough; omega_r = min(1, 2 / (lambda_min + lambda_max)).
        """
        if not self.relax or self.L < 2:
            return 1.0
        J = self.L - 1
        kb = self.g.kband

        def lam(x):
            return sum(x ** j / math.factorial(j) for j in range(J + 1))

        lmax = lam(kb * float(np.max(eta)))
        lmin = lam(kb * float(np.min(eta)))
        s = lmin + lmax
        if not np.isfinite(s) or s <= 0:
            return 1.0
        return min(1.0, 2.0 / s)

    def _net_corrections(self, eta, ph):
        """Physical corrections (nV, nB) of the learned warm start at a state."""
        from . import warmstart as ws
        theta, in_scale, out_scale = self.net
        f, _ = ws.features(self, eta, self.g.ifft(ph))
        x = (f * np.asarray(in_scale, dtype=np.float32).astype(np.float64))[None]
        y = ws.forward(theta, x, bf16_weights=True, bf16_acts=True)[0]
        osc = np.asarray(out_scale, dtype=np.float32).astype(np.float64)
        return osc[0] * y[..., 0], osc[1] * y[..., 1]

    def _sweeps(self, eta, bV, bB, Vh, Bh, w, tol):
        """Sweeps from (Vh, Bh) until the stopping rules end them: returns
        (T_V(V) of the last sweep, the phi_b iterate after the relaxed update
        of the last sweep, info)."""
        g = self.g
        info = SolveInfo()
        info.omega = w
        rmin = np.inf
        Vn = Vh
        for n in range(self.max_sweeps):
            Vn, Bn = self.apply_T(eta, bV, bB, Vh, Bh)
            Vnew = g.ifft(Vn)
            dif = g.ifft(Vn - Vh)
            num = float(np.max(np.abs(dif)))
            den = float(np.max(np.abs(Vnew)))
            if not (np.isfinite(num) and np.isfinite(den)):
                info.status = ERR_NONFINITE
                info.sweeps = n + 1
                info.residual = float("nan")
                return Vn, Bn, info
            r = 0.0 if num == 0.0 else (num / den if den > 0 else np.inf)
            info.history.append(r)
            info.sweeps = n + 1
            info.residual = r
            if r <= tol:
                return Vn, Bh + w * (Bn - Bh), info
            rmin = min(rmin, r)
            if r > 1e6 or (n >= 3 and r > 10.0 * rmin):
                info.status = ERR_DIVERGED
                return Vn, Bn, info
            Vh = Vh + w * (Vn - Vh)
            Bh = Bh + w * (Bn - Bh)
        info.status = WARN_NOT_CONVERGED
        return Vn, Bh, info

    def _wdot(self, a, b):
        """Real inner product of two masked half spectra, each mode weighted
        by the number of modes of the full spectrum it stands for (Parseval)."""
        g = self.g
        w = np.where(np.arange(a.shape[1])[None, :] == 0, 1.0, 2.0) * g.mask
        return float(np.sum(w * (a.real * b.real + a.imag * b.imag)))

    def _sweeps_anderson(self, eta, bV, bB, Vh, Bh, w, tol):
        """Sweeps with Anderson mixing (type II, depth m = aa_depth) of the
        relaxed sweep G(x) = x + w (T(x) - x), x = (V, phi_b) (phi_b only over
        a variable bed): with f_i = T(x_i) - x_i and g_i = G(x_i) over the last
        k <= m + 1 sweeps, gamma minimises |f_n - sum_i gamma_i (f_(i+1) - f_i)|
        in the inner product of _wdot (normal equations, regularised by
        1e-12 trace / k; gamma = 0 if they fail), and
        x_(n+1) = g_n - sum_i gamma_i (g_(i+1) - g_i).
        Same residual, stopping rules and returned values as _sweeps."""
        g = self.g
        info = SolveInfo()
        info.omega = w
        rmin = np.inf
        use_b = not self.flat
        F, G = [], []
        Vn = Vh
        for n in range(self.max_sweeps):
            Vn, Bn = self.apply_T(eta, bV, bB, Vh, Bh)
            Vnew = g.ifft(Vn)
            dif = g.ifft(Vn - Vh)
            num = float(np.max(np.abs(dif)))
            den = float(np.max(np.abs(Vnew)))
            if not (np.isfinite(num) and np.isfinite(den)):
                info.status = ERR_NONFINITE
                info.sweeps = n + 1
                info.residual = float("nan")
                return Vn, Bn, info
            r = 0.0 if num == 0.0 else (num / den if den > 0 else np.inf)
            info.history.append(r)
            info.sweeps = n + 1
            info.residual = r
            # the next iterate (formed before the decision, as the device does)
            f = (Vn - Vh, Bn - Bh)
            F.append(f)
            G.append((Vh + w * f[0], Bh + w * f[1]))
            if len(F) > self.aa_depth + 1:
                F.pop(0)
                G.pop(0)
            k = len(F) - 1
            gam = np.zeros(k)
            if k > 0:
                dF = [(F[i + 1][0] - F[i][0], F[i + 1][1] - F[i][1]) for i in range(k)]

                def dot(a, b):
                    return self._wdot(a[0], b[0]) + (self._wdot(a[1], b[1]) if use_b else 0.0)

                A = np.array([[dot(dF[i], dF[j]) for j in range(k)] for i in range(k)])
                y = np.array([dot(dF[i], f) for i in range(k)])
                tr = np.trace(A)
                try:
                    gam = np.linalg.solve(A + (1e-12 * tr / k) * np.eye(k), y)
                    if not np.all(np.isfinite(gam)) or not tr > 0:
                        gam = np.zeros(k)
                except np.linalg.LinAlgError:
                    gam = np.zeros(k)
            Vx, Bx = G[-1]
            for i in range(k):
                Vx = Vx - gam[i] * (G[i + 1][0] - G[i][0])
                Bx = Bx - gam[i] * (G[i + 1][1] - G[i][1])
            if r <= tol:
                return Vn, Bx, info
            rmin = min(rmin, r)
            if r > 1e6 or (n >= 3 and r > 10.0 * rmin):
                info.status = ERR_DIVERGED
                return Vn, Bn, info
            Vh, Bh = Vx, Bx
        info.status = WARN_NOT_CONVERGED
        return Vn, Bh, info

    def w_iter_hat(self, eta, ph, tol, seed_hat=None, seed_b_hat=None, stage=None):
        """Iteration on the summed operator from the solver's seed (see the
        constructor), or from the seed spectrum seed_hat of V (and the
        bottom-potential correction seed_b_hat added to its linear guess).
        stage: the RK4 stage (0..3) of a fixed-step solve, None otherwise."""
        from . import history_seed as hs
        g = self.g
        bV, bB = self.forcing(eta, ph)
        Vlin = g.k * self.T * ph
        Blin = self.S * ph
        w = self.relax_factor(eta)
        net = False
        H = self.hist
        use_hist = (seed_hat is None and self.seed == "net" and H is not None and stage is not None
                    and len(self._hist) >= H["K"])
        if use_hist:
            net = True
            W = hs.to_complex(H["theta"], H["K"], H["nb"])
            pV, pB = hs.predict(W, self._hist[:H["K"]], stage, H["b"])
            Vh = Vlin + g.mask * pV
            Bh = Blin if pB is None else Blin + g.mask * pB
        elif seed_hat is not None:
            Vh = g.mask * seed_hat
            Bh = Blin if seed_b_hat is None else Blin + g.mask * seed_b_hat
        elif self.seed == "net" and self._prev is None and self.net is not None:
            net = True
            nV, nB = self._net_corrections(eta, ph)
            Vh = Vlin + g.MF(nV)
            Bh = Blin + g.MF(nB)
        elif self.seed in ("prev", "net") and self._prev is not None:
            Vh = Vlin + self._prev[0]
            Bh = Blin + self._prev[1]
        else:
            Vh, Bh = Vlin, Blin
        sweeps = self._sweeps_anderson if self.accel == "anderson" else self._sweeps
        Vn, Bl, info = sweeps(eta, bV, bB, Vh, Bh, w, tol)
        if net and info.status < 0:
            # the linear guess is the fallback of the learned seed
            Vn, Bl, info = sweeps(eta, bV, bB, Vlin, Blin, w, tol)
            info.fallback = True
        # nonlinear part of this solve: the seed of the next one
        self._prev = (Vn - Vlin, Bl - Blin) if info.status >= 0 else None
        if self._prev is None or stage is None:
            # only successful fixed-step solves form the history layer's input
            self._hist = []
        else:
            part = (self._prev[0], None if self.flat else self._prev[1])
            if H is not None and self.hist_train and len(self._hist) >= H["K"]:
                W = hs.to_complex(H["theta"], H["K"], H["nb"])
                loss, grad, gram = hs.loss_grad(W, self._hist[:H["K"]], part, stage, H["b"], H["c"], H["nb"])
                if self._hist_acc is None:
                    K_, nb_ = H["K"], H["nb"]
                    self._hist_acc = dict(grad=np.zeros((2, hs.STAGES, nb_, K_), complex),
                                          gram=np.zeros((2, hs.STAGES, nb_, K_, K_), complex), loss=0.0, n=0)
                self._hist_acc["grad"][:, stage] += grad
                self._hist_acc["gram"][:, stage] += gram
                self._hist_acc["loss"] += loss
                self._hist_acc["n"] += 1
            self._hist.insert(0, part)
            del self._hist[max(H["K"], 1) if H is not None else 1:]
        return Vn, info

    def hist_adam(self, lr):
        """One Adam step of the history layer with the mean gradient of the
        solves accumulated since the last step; returns (mean loss, samples)."""
        from . import history_seed as hs
        H = self.hist
        acc = self._hist_acc
        if acc is None or acc["n"] == 0:
            return 0.0, 0
        g = acc["grad"] / acc["n"]
        gflat = np.stack([g.real, g.imag], axis=-1).ravel()
        if self._hist_adam is None:
            self._hist_adam = [np.zeros_like(gflat), np.zeros_like(gflat), 0]
        m, v, step = self._hist_adam
        step += 1
        th, m, v = hs.adam_step(H["theta"].astype(np.float64), m, v, gflat, step, lr)
        H["theta"] = th.astype(np.float32)
        self._hist_adam = [m, v, step]
        out = (acc["loss"] / acc["n"], acc["n"])
        self._hist_acc = None
        return out

    def hist_newton(self, lam=1e-9):
        """Gauss-Newton step of the history layer on the solves accumulated
        since the last step (oracle.history_seed.newton); returns (mean loss,
        samples)."""
        from . import history_seed as hs
        H = self.hist
        acc = self._hist_acc
        if acc is None or acc["n"] == 0:
            return 0.0, 0
        W = hs.to_complex(H["theta"], H["K"], H["nb"])
        W = hs.newton(W, acc["grad"], acc["gram"], lam)
        H["theta"] = hs.to_flat(W).astype(np.float32)
        out = (acc["loss"] / acc["n"], acc["n"])
        self._hist_acc = None
        return out

    # ------------------------------------------------------------------------
    def w_full_hat(self, eta, ph, tol):
        """W with the remaining integrals of App. A and App. B kept
        (oracle.full_bie), masked: the image form over a flat bed, or a bed so
        deep that it is invisible (k_1 times the smallest depth beyond 18); the
        two-boundary form over any other bed."""
        from . import full_bie
        g = self.g
        e = np.asarray(eta).ravel()
        p = g.ifft(ph).ravel()
        dmin = self.h - float(self.delta.max())
        if self.flat or full_bie.is_deep(g.lx, dmin):
            V, sweeps, status, r = full_bie.vertical_velocity(e, p, g.lx, self.h, tol, self.max_sweeps)
        else:
            V, sweeps, status, r = full_bie.vertical_velocity_bed(e, p, g.lx, self.h, self.delta.ravel(), tol,
                                                                  self.max_sweeps)
        return g.MF(V.reshape(1, g.nx)), SolveInfo(sweeps=sweeps, residual=r, status=status)

    def solve_hat(self, eta, ph, tol=1e-10, seed_hat=None, seed_b_hat=None, stage=None):
        if self.mode == "sa":
            return self.w_sa_hat(eta, ph), SolveInfo(sweeps=0)
        if self.mode == "full":
            return self.w_full_hat(eta, ph, tol)
        return self.w_iter_hat(eta, ph, tol, seed_hat, seed_b_hat, stage)

    def vertical_velocity(self, eta, phi_s, tol=1e-10, seed=None, seed_b=None):
        """W = V at z = eta for physical (eta, phi_s); phi_s is band-limited by the mask.
        seed / seed_b: optional physical seed of V and correction of phi_b."""
        g = self.g
        eta = np.asarray(eta, dtype=np.float64).reshape(g.ny, g.nx)
        ph = g.MF(phi_s)
        seed_hat = None if seed is None else g.fft(seed)
        seed_b_hat = None if seed_b is None else g.fft(seed_b)
        Vh, info = self.solve_hat(eta, ph, tol, seed_hat, seed_b_hat)
        return g.ifft(Vh), info

    # ------------------------------------------------------------------------
    # Prognostic step: Eq. (prognostic) in integrating-factor form
    # ------------------------------------------------------------------------
    # ------------------------------------------------------------------------
    # Surface pressures of the numerical wave tank (Sec. 3.2)
    # ------------------------------------------------------------------------
    def _x_periodic(self, x0):
        """x - x0 of every grid column, wrapped to [-lx/2, lx/2)."""
        g = self.g
        x = np.arange(g.nx) * (g.lx / g.nx)
        return (x - x0 + g.lx / 2) % g.lx - g.lx / 2

    def wavemaker_pressure(self, t):
        """p_g(x, t) of the pneumatic wavemaker: bell-shaped components centred
        on x = 0, i.e. split in halves over both ends of the periodic domain,
        uniform in y."""
        wm = self.wm
        h = wm.get("h") or self.h
        xs = self._x_periodic(0.0)
        p = np.zeros(self.g.nx)
        for a, k, om, th in wm.get("comps", ()):
            kh2 = 2.0 * k * h
            G = kh2 / math.sinh(kh2) if kh2 < 700.0 else 0.0
            p += a * math.sqrt(math.e / (2 * math.pi)) * (1.0 + G) * np.exp(-0.5 * (k * xs) ** 2) * math.sin(om * t + th)
        return np.broadcast_to(p[None, :], (self.g.ny, self.g.nx))

    def damping_weight(self):
        wm = self.wm
        w = wm.get("width") or 4 * math.pi
        mu = np.exp(-(self._x_periodic(wm["x0"]) / w) ** 2)
        return np.broadcast_to(mu[None, :], (self.g.ny, self.g.nx))

    def damping_pressure_hat(self, ph, mu):
        """Spectrum of p_d = F^-1{ ik/(-k^2) . MF{mu grad phi} } (Eq. pd), with the
        weighted gradient dealiased like every product and the k = 0 mode 0."""
        g = self.g
        px, py = g.grad(ph)
        num = g.ikdot(g.MF(mu * px), None if py is None else g.MF(mu * py))
        k2 = g.k ** 2
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(k2 > 0, num / np.where(k2 > 0, -k2, 1.0), 0.0)

    def rhs(self, eh, ph, tol, t=0.0, stage=None):
        """N = (V_hat - omega^2 phi_hat, MF{ (V + grad eta.grad phi)^2/(2(1+|grad eta|^2))
        - |grad phi|^2/2 - p_g } - p_d_hat)  for masked state spectra (eh, ph) at time t;
        the surface pressure p = p_g + p_d of the wave tank (zero without it)
        enters the dynamic condition beside the elevation."""
        g = self.g
        eta = g.ifft(eh)
        Vh, info = self.solve_hat(eta, ph, tol, stage=stage)
        if info.status < 0:
            raise FloatingPointError(f"W solve failed with status {info.status}")
        V = g.ifft(Vh)
        ex, ey = g.grad(eh)
        px, py = g.grad(ph)
        if ey is None:
            gg = ex * ex
            q = V + ex * px
            pp = px * px
        else:
            gg = ex * ex + ey * ey
            q = V + ex * px + ey * py
            pp = px * px + py * py
        nphi = 0.5 * (q * q / (1.0 + gg) - pp)
        Nphi = None
        if self.wm is not None:
            nphi = nphi - self.wavemaker_pressure(t)
            if self.wm.get("x0") is not None:
                Nphi = g.MF(nphi) - self.damping_pressure_hat(ph, self.damping_weight())
        if Nphi is None:
            Nphi = g.MF(nphi)
        return Vh - self.om2 * ph, Nphi, Vh, info

    def propagate(self, a, b, tau):
        """E(tau) applied to the pair (a, b): exact linear propagator."""
        om = self.om
        c = np.cos(om * tau)
        s = np.sin(om * tau)
        with np.errstate(divide="ignore", invalid="ignore"):
            sw = np.where(om > 0, s / np.where(om > 0, om, 1.0), tau)
        return c * a + om * s * b, -sw * a + c * b

    def step_hat(self, eh, ph, dt, tol, stats=None, t=0.0):
        """One Lawson IF-RK4 step on masked spectra from time t."""
        h = dt
        a = self.rhs(eh, ph, tol, t, stage=0)
        if stats is not None:
            stats.append(a[3])
        u2 = self.propagate(eh + h / 2 * a[0], ph + h / 2 * a[1], h / 2)
        b = self.rhs(*u2, tol, t + h / 2, stage=1)
        eh_h, ph_h = self.propagate(eh, ph, h / 2)
        u3 = (eh_h + h / 2 * b[0], ph_h + h / 2 * b[1])
        c = self.rhs(*u3, tol, t + h / 2, stage=2)
        ec, pc = self.propagate(c[0], c[1], h / 2)
        eh_f, ph_f = self.propagate(eh, ph, h)
        u4 = (eh_f + h * ec, ph_f + h * pc)
        d = self.rhs(*u4, tol, t + h, stage=3)
        if stats is not None:
            stats.extend([b[3], c[3], d[3]])
        ea, pa = self.propagate(a[0], a[1], h)
        ebc, pbc = self.propagate(b[0] + c[0], b[1] + c[1], h / 2)
        en = eh_f + h / 6 * (ea + 2 * ebc + d[0])
        pn = ph_f + h / 6 * (pa + 2 * pbc + d[1])
        en = self.g.mask * en
        pn = self.g.mask * pn
        if self.filter_beta is not None:
            b1, b2 = self.filter_beta
            lam = np.exp(-np.abs(self.g.k / b1) ** b2)  # Eq. (filter)
            en = lam * en
            pn = lam * pn
        return en, pn

    def relaxation_target(self, t):
        rz = self.rz
        T = 2 * np.pi / rz["omega"]
        tr = rz["ramp_periods"] * T
        r = 0.5 * (1 - np.cos(np.pi * t / tr)) if t < tr else 1.0
        x = np.arange(self.g.nx) * (self.g.lx / self.g.nx)
        th = rz["k"] * x - rz["omega"] * t
        eta_t = rz["a"] * r * np.cos(th)
        phi_t = rz["a"] * r / rz["omega"] * np.sin(th)
        return eta_t[None, :], phi_t[None, :]

    def relaxation_weights(self):
        rz = self.rz
        x = np.arange(self.g.nx) * (self.g.lx / self.g.nx)
        L = self.g.lx
        wg = np.zeros_like(x)
        m = x < rz["gen_len"]
        s = x[m] / rz["gen_len"]
        wg[m] = 1.0 - (3 * s * s - 2 * s ** 3)
        wa = np.zeros_like(x)
        m = x > L - rz["abs_len"]
        s = (L - x[m]) / rz["abs_len"]
        wa[m] = 1.0 - (3 * s * s - 2 * s ** 3)
        return wg[None, :], wa[None, :]

    def apply_relaxation(self, eh, ph, t):
        g = self.g
        eta = g.ifft(eh)
        phi = g.ifft(ph)
        wg, wa = self.relaxation_weights()
        et, pt = self.relaxation_target(t)
        eta = (1 - wg) * eta + wg * et
        phi = (1 - wg) * phi + wg * pt
        eta = (1 - wa) * eta
        phi = (1 - wa) * phi
        return g.MF(eta), g.MF(phi)

    def step(self, eta, phi_s, dt, n, tol=1e-10, t0=0.0):
        """Advance physical (eta, phi_s) by n steps of dt; returns (eta, phi_s, solve_infos)."""
        g = self.g
        eh = g.MF(np.asarray(eta, dtype=np.float64).reshape(g.ny, g.nx))
        ph = g.MF(np.asarray(phi_s, dtype=np.float64).reshape(g.ny, g.nx))
        stats = []
        t = t0
        for _ in range(n):
            eh, ph = self.step_hat(eh, ph, dt, tol, stats, t)
            t += dt
            if self.rz is not None:
                eh, ph = self.apply_relaxation(eh, ph, t)
        return g.ifft(eh), g.ifft(ph), stats

    # ------------------------------------------------------------------------
    # Adaptive step (Sec. 2.2): embedded fifth/fourth-order pair, Lawson form
    # ------------------------------------------------------------------------
    def linear_energy(self, eh, ph):
        """sum over the grid of eta^2 + phi D(phi), D the linear Dirichlet-to-
        Neumann operator F^-1{k tanh(kh) F{.}}: twice the linear part of the
        energy of Eq. (energy) per unit cell area."""
        g = self.g
        e = g.ifft(eh)
        p = g.ifft(ph)
        dp = g.ifft(self.om2 * ph)
        return float(np.sum(e * e) + np.sum(p * dp))

    def step_rk54_hat(self, eh, ph, dt, tol, stats=None, t=0.0):
        """One step of the embedded pair on masked spectra.  Returns the
        fifth-order state (masked, then filtered when the filter is on) and
        the relative difference sqrt(E(u5 - u4) / E(u5)) of the unfiltered
        solutions in the linear-energy norm (0 when both vanish)."""
        def f(u, tau):
            r = self.rhs(u[0], u[1], tol, t + tau)
            if stats is not None:
                stats.append(r[3])
            return (r[0], r[1])

        u5, u4 = lawson_rk54((eh, ph), dt, f, lambda u, tau: self.propagate(u[0], u[1], tau))
        num = self.linear_energy(u5[0] - u4[0], u5[1] - u4[1])
        den = self.linear_energy(u5[0], u5[1])
        err = 0.0 if num == 0.0 else math.sqrt(num / den) if den > 0.0 else math.inf
        en = self.g.mask * u5[0]
        pn = self.g.mask * u5[1]
        if self.filter_beta is not None:
            b1, b2 = self.filter_beta
            lam = np.exp(-np.abs(self.g.k / b1) ** b2)  # Eq. (filter)
            en = lam * en
            pn = lam * pn
        return en, pn, err

    def step_adaptive(self, eta, phi_s, t0, t_end, dt, rk_tol, tol=1e-10, max_steps=1000):
        """Advance physical (eta, phi_s) from t0 to t_end with the adaptive pair.
        dt is the first trial step.  Returns (eta, phi_s, info) with info keys
        t, dt_next, accepted, rejected, status, history = [(h, err, accepted)].
        A step whose trial size reaches t_end (within a relative 1e-9) is cut
        to land on t_end exactly; dt_next after such a cut step is the larger
        of the controller's proposal and the trial size before the cut."""
        SAFETY, FAC_MIN, FAC_MAX = 0.9, 0.2, 5.0
        g = self.g
        eh = g.MF(np.asarray(eta, dtype=np.float64).reshape(g.ny, g.nx))
        ph = g.MF(np.asarray(phi_s, dtype=np.float64).reshape(g.ny, g.nx))
        t, h = float(t0), float(dt)
        acc = rej = 0
        last_rejected = False
        status = OK
        hist = []
        while t < t_end:
            if acc + rej >= max_steps:
                status = WARN_STEP_LIMIT
                break
            final = t_end - t <= h * (1.0 + 1e-9)
            hs = t_end - t if final else h
            en, pn, err = self.step_rk54_hat(eh, ph, hs, tol, t=t)
            fmax = 1.0 if last_rejected else FAC_MAX
            if not math.isfinite(err):
                fac = FAC_MIN
            elif err == 0.0:
                fac = fmax
            else:
                fac = min(fmax, max(FAC_MIN, SAFETY * (rk_tol / err) ** 0.2))
            ok = err <= rk_tol
            hist.append((hs, err, ok))
            if ok:
                eh, ph = en, pn
                t = t_end if final else t + hs
                acc += 1
                last_rejected = False
                if self.rz is not None:
                    eh, ph = self.apply_relaxation(eh, ph, t)
                h = max(hs * fac, h) if final else hs * fac
            else:
                rej += 1
                last_rejected = True
                h = hs * fac
                if h < 1e-12 * max(abs(t_end - t0), abs(t)):
                    raise FloatingPointError("step size underflow")
        info = dict(t=t, dt_next=h, accepted=acc, rejected=rej, status=status, history=hist)
        return g.ifft(eh), g.ifft(ph), info

    # ------------------------------------------------------------------------
    # Diagnostics, Eq. (energy)
    # ------------------------------------------------------------------------
    def diagnostics(self, eta, phi_s, tol=1e-10):
        """(mass, energy) = (dA sum eta, dA/2 sum (V phi_s + eta^2)) at the masked state."""
        g = self.g
        eh = g.MF(eta)
        ph = g.MF(phi_s)
        e = g.ifft(eh)
        p = g.ifft(ph)
        Vh, _ = self.solve_hat(e, ph, tol)
        V = g.ifft(Vh)
        mass = g.dA * float(np.sum(e))
        energy = 0.5 * g.dA * float(np.sum(V * p + e * e))
        return mass, energy


# ---------------------------------------------------------------------------
# Six-stage fifth-order Runge-Kutta pair with an embedded fourth-order
# solution (the integrator class of Sec. 2.2): the coefficients of Cash & Karp
# (ACM TOMS 16, 1990), nodes CK_C, stage matrix CK_A (row i: a_i0 .. a_i,i-1),
# weights CK_B5 (order 5) and CK_B4 (order 4).
# ---------------------------------------------------------------------------
CK_C = (0.0, 1 / 5, 3 / 10, 3 / 5, 1.0, 7 / 8)
CK_A = (
    (),
    (1 / 5,),
    (3 / 40, 9 / 40),
    (3 / 10, -9 / 10, 6 / 5),
    (-11 / 54, 5 / 2, -70 / 27, 35 / 27),
    (1631 / 55296, 175 / 512, 575 / 13824, 44275 / 110592, 253 / 4096),
)
CK_B5 = (37 / 378, 0.0, 250 / 621, 125 / 594, 0.0, 512 / 1771)
CK_B4 = (2825 / 27648, 0.0, 18575 / 48384, 13525 / 55296, 277 / 14336, 1 / 4)


def lawson_rk54(u, h, f, E):
    """One step of the pair in integrating-factor (Lawson) form for
    u' = L u + f(u, t - t_n), with E(x, tau) = exp(L tau) x (Sec. 2.2's
    integrating factor): in v = E(u, -(t - t_n)) the pair is applied to
    v' = E(f(E(v, t - t_n)), -(t - t_n)), which written back in u reads
        U_i = E(u, c_i h) + h sum_j a_ij E(N_j, (c_i - c_j) h),  N_i = f(U_i, c_i h)
        u_q = E(u, h)     + h sum_j b_j  E(N_j, (1 - c_j) h)     (q = 5, 4).
    u and the values of f and E are tuples of arrays.  Returns (u5, u4)."""
    def axpy(acc, a, x):
        return tuple(ai + a * xi for ai, xi in zip(acc, x))

    N = []
    for i in range(6):
        U = E(u, CK_C[i] * h)
        for j, a in enumerate(CK_A[i]):
            if a != 0.0:
                U = axpy(U, h * a, E(N[j], (CK_C[i] - CK_C[j]) * h))
        N.append(f(U, CK_C[i] * h))
    out = []
    for b in (CK_B5, CK_B4):
        v = E(u, h)
        for j in range(6):
            if b[j] != 0.0:
                v = axpy(v, h * b[j], E(N[j], (1.0 - CK_C[j]) * h))
        out.append(v)
    return out[0], out[1]


# ---------------------------------------------------------------------------
# Second, independent coding: the explicit orders of Appendix C written out
# term by term (Eqs. v2-v7).  Used only to cross-check Solver.w_sa_hat.
# ---------------------------------------------------------------------------
def w_sa_appc(solver: Solver, eta, phi_s, L: int = 7):
    g = solver.g
    k, T, S = g.k, solver.T, solver.S
    d = solver.delta
    ph = g.MF(phi_s)
    with np.errstate(divide="ignore"):
        kinv = np.where(k > 0, 1.0 / np.where(k > 0, k, 1.0), 0.0)

    def F(f):
        return g.MF(f)

    def ik(fx, fy):
        return g.ikdot(fx, fy)

    gx, gy = g.grad(ph)

    def eg(p):  # F{eta^p grad phi_s} as a pair
        return F(eta ** p * gx), (F(eta ** p * gy) if gy is not None else None)

    def dgB(p, B):  # F{delta^p grad phi_b} as a pair
        bx, by = g.grad(B)
        return F(d ** p * bx), (F(d ** p * by) if by is not None else None)

    def eV(p, V):  # F{eta^p V}
        return F(eta ** p * g.ifft(V))

    def lin(a, pa, b, pb):  # a*pa + b*pb for pairs
        x = a * pa[0] + b * pb[0]
        y = None if pa[1] is None else a * pa[1] + b * pb[1]
        return x, y

    V1 = k * T * ph
    B1 = S * ph
    # Eq. (v2)
    V2 = -k * T * eV(1, V1) - ik(*lin(1.0, eg(1), -S, dgB(1, B1)))
    B2 = -S * eV(1, V1) - kinv * T * ik(*dgB(1, B1))
    # third order
    V3 = -k * T * eV(1, V2) - 0.5 * k ** 2 * eV(2, V1) \
        - ik(*lin(0.5 * k * T, eg(2), -S, dgB(1, B2)))
    t1 = lin(-0.5 * S, eg(2), -kinv * T, dgB(1, B2))
    t2 = dgB(2, B1)
    B3 = -S * eV(1, V2) + ik(*lin(1.0, t1, 0.5, t2))
    # fourth order
    V4 = -T * (k * eV(1, V3) + k ** 3 / 6 * eV(3, V1)) - 0.5 * k ** 2 * eV(2, V2) \
        - ik(*lin(k ** 2 / 6, eg(3), -S, lin(1.0, dgB(1, B3), k ** 2 / 6, dgB(3, B1))))
    B4 = -S * (eV(1, V3) + k ** 2 / 6 * eV(3, V1)) \
        + ik(*lin(0.5, dgB(2, B2), -T, lin(kinv, dgB(1, B3), k / 6, dgB(3, B1))))
    # fifth order
    V5 = -T * (k * eV(1, V4) + k ** 3 / 6 * eV(3, V2)) - 0.5 * k ** 2 * eV(2, V3) \
        - k ** 4 / 24 * eV(4, V1) \
        + ik(*lin(-k ** 3 / 24 * T, eg(4), S, lin(1.0, dgB(1, B4), k ** 2 / 6, dgB(3, B2))))
    B5 = -S * (eV(1, V4) + k ** 2 / 6 * eV(3, V2)) \
        + ik(*lin(1.0, lin(-k ** 2 / 24 * S, eg(4), -T, lin(kinv, dgB(1, B4), k / 6, dgB(3, B2))),
                  1.0, lin(0.5, dgB(2, B3), k ** 2 / 24, dgB(4, B1))))
    # sixth order
    V6 = -T * (k * eV(1, V5) + k ** 3 / 6 * eV(3, V3) + k ** 5 / 120 * eV(5, V1)) \
        - 0.5 * k ** 2 * eV(2, V4) - k ** 4 / 24 * eV(4, V2) \
        + ik(*lin(-k ** 4 / 120, eg(5), S,
                  lin(1.0, lin(1.0, dgB(1, B5), k ** 2 / 6, dgB(3, B3)), k ** 4 / 120, dgB(5, B1))))
    B6 = -S * (eV(1, V5) + k ** 2 / 6 * eV(3, V3) + k ** 4 / 120 * eV(5, V1)) \
        + ik(*lin(-T, lin(1.0, lin(kinv, dgB(1, B5), k / 6, dgB(3, B3)), k ** 3 / 120, dgB(5, B1)),
                  1.0, lin(0.5, dgB(2, B4), k ** 2 / 24, dgB(4, B2))))
    # Eq. (v7)
    V7 = -T * (k * eV(1, V6) + k ** 3 / 6 * eV(3, V4) + k ** 5 / 120 * eV(5, V2)) \
        - 0.5 * k ** 2 * eV(2, V5) - k ** 4 / 24 * eV(4, V3) - k ** 6 / 720 * eV(6, V1) \
        + ik(*lin(-k ** 5 / 720 * T, eg(6), S,
                  lin(1.0, lin(1.0, dgB(1, B6), k ** 2 / 6, dgB(3, B4)), k ** 4 / 120, dgB(5, B2))))
    Vs = [V1, V2, V3, V4, V5, V6, V7][:L]
    return g.ifft(sum(Vs))
