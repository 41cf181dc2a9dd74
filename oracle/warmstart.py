"""FP64 oracle of the learned warm start of the W iteration.  TEST INFRASTRUCTURE ONLY.

The paper's solver starts the successive approximation from the linear
initiation of Sec. 2.4, V0 = F^-1{k tanh(kh) phi_hat}.  The learned warm start
adds a correction predicted by a small periodic convolution network from local
surface quantities, so that the iteration (which still decides convergence by
its own residual) starts closer to its fixed point.

Network (channel-last fields x[b, y, x, c], periodic in y and x):

    features  f = (eta, W_lin, d_x eta, d_y eta, d_x phi, d_y phi, delta, eta * W_lin)
              x_c = s_c * f_c                     (s: per-channel input scales)
    layer 1   z1 = b1 + conv3x3(x; W1)   8 -> 32,  a1 = silu(z1)
    layer 2   z2 = b2 + conv3x3(a1; W2) 32 -> 32,  a2 = silu(z2)
    layer 3   z3 = b3 + conv1x1(a2; W3) 32 -> 32,  a3 = silu(z3)
    layer 4   y  = b4 + conv1x1(a3; W4) 32 -> 2
    seed      V0 = W_lin + out_scale[0] * y[0]                      (surface)
              phi_b0 = F^-1{sech(kh) phi_hat} + out_scale[1] * y[1]   (bottom)

conv3x3 is a periodic cross-correlation:
    z[o](p) = b[o] + sum_{t=0..8} sum_c W[o, t, c] * a[c](p + off(t)),
    off(t) = (t // 3 - 1, t % 3 - 1)  as (dy, dx);
silu(z) = z / (1 + exp(-z)).

The iteration is seeded in both of its unknowns: with a variable bed the bottom
potential's error slows convergence as much as the surface one.  Training
minimises the mean over points and both outputs of (y - t)^2 with the targets
t = ((W* - W_lin) / out_scale[0], (phi_b* - phi_b,lin) / out_scale[1]), the
nonlinear parts left by a converged iteration from the linear guess.  The
optimiser is Adam (Kingma & Ba 2015) with bias correction; the forward pass
uses the BF16 rounding of the FP32 master weights.

Parameter vector (FP32 masters, this order): W1[32,9,8], b1[32], W2[32,9,32],
b2[32], W3[32,32], b3[32], W4[2,32], b4[2].
"""
from __future__ import annotations

import math

import numpy as np

CIN = 8
WIDTH = 32
SHAPES = [("W1", (WIDTH, 9, CIN)), ("b1", (WIDTH,)),
          ("W2", (WIDTH, 9, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)),
          ("W4", (2, WIDTH)), ("b4", (2,))]
PARAM_COUNT = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Split the flat parameter vector into named arrays (views)."""
    out, i = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[i:i + n]).reshape(shp)
        i += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


# ---------------------------------------------------------------------------
# BF16 rounding (round to nearest, ties to even), taken as float64 -> float32
# (nearest) -> bfloat16 (nearest even on the top 16 bits of the float32)
# ---------------------------------------------------------------------------
def bf16(x):
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


# ---------------------------------------------------------------------------
# periodic convolutions on channel-last fields a[b, y, x, c]
# ---------------------------------------------------------------------------
def _shift(a, dy, dx):
    """a(p + (dy, dx)) with periodic wrap."""
    return np.roll(np.roll(a, -dy, axis=1), -dx, axis=2)


def conv3x3(a, W, b):
    out = np.zeros(a.shape[:3] + (W.shape[0],)) + b
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        out += _shift(a, dy, dx) @ W[:, t, :].T
    return out


def conv3x3_grad_input(g, W):
    """d/da of sum(g * conv3x3(a, W, b)):  sum_t sum_o g[o](p - off(t)) W[o, t, c]."""
    out = np.zeros(g.shape[:3] + (W.shape[2],))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        out += _shift(g, -dy, -dx) @ W[:, t, :]
    return out


def conv3x3_grad_weight(g, a):
    """d/dW[o, t, c] of sum(g * conv3x3(a, W, b)) = sum_p g[o](p) a[c](p + off(t))."""
    cout, cin = g.shape[-1], a.shape[-1]
    dW = np.zeros((cout, 9, cin))
    G = g.reshape(-1, cout)
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        dW[:, t, :] = G.T @ _shift(a, dy, dx).reshape(-1, cin)
    return dW


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def forward(theta, x, bf16_weights=True, bf16_acts=False, keep=False):
    """Network output y[b, y, x, 2] for features x[b, y, x, 8] (already scaled).

    bf16_weights: use the BF16 rounding of the weights and the FP32 rounding
    of the biases, as the device does.
    bf16_acts: also round the inputs of the first three layers to BF16, as the
    matrix-core inference does (layer 3's output and layer 4 stay unrounded).
    """
    p = unpack(np.asarray(theta, dtype=np.float64))
    rw = bf16 if bf16_weights else (lambda v: v)
    ra = bf16 if bf16_acts else (lambda v: v)
    rb = (lambda v: v.astype(np.float32).astype(np.float64)) if bf16_weights else (lambda v: v)
    b1, b2, b3, b4 = rb(p["b1"]), rb(p["b2"]), rb(p["b3"]), rb(p["b4"])
    x0 = ra(x)
    z1 = conv3x3(x0, rw(p["W1"]), b1)
    a1 = ra(silu(z1))
    z2 = conv3x3(a1, rw(p["W2"]), b2)
    a2 = ra(silu(z2))
    z3 = a2 @ rw(p["W3"]).T + b3
    a3 = silu(z3)
    y = a3 @ rw(p["W4"]).T + b4
    if keep:
        return y, dict(x=x0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3)
    return y


def loss_and_grad(theta, x, target, bf16_weights=True):
    """Mean-square loss and its gradient with respect to the parameters.

    With bf16_weights the forward pass uses the rounded weights and the
    gradient is taken with respect to those rounded values (applied to the
    FP32 masters by the optimiser).
    """
    p = unpack(np.asarray(theta, dtype=np.float64))
    rw = bf16 if bf16_weights else (lambda v: v)
    W1, W2, W3, W4 = rw(p["W1"]), rw(p["W2"]), rw(p["W3"]), rw(p["W4"])
    y, c = forward(theta, x, bf16_weights=bf16_weights, keep=True)
    n = y.size
    r = y - target
    loss = float(np.sum(r * r) / n)
    gy = 2.0 * r / n                                   # dL/dy
    g = {}
    g["W4"] = np.einsum("byxk,byxc->kc", gy, c["a3"])
    g["b4"] = gy.reshape(-1, 2).sum(axis=0)
    g3 = (gy @ W4) * dsilu(c["z3"])                    # dL/dz3
    g["W3"] = g3.reshape(-1, WIDTH).T @ c["a2"].reshape(-1, WIDTH)
    g["b3"] = g3.reshape(-1, WIDTH).sum(axis=0)
    g2 = (g3 @ W3) * dsilu(c["z2"])                    # dL/dz2
    g["W2"] = conv3x3_grad_weight(g2, c["a1"])
    g["b2"] = g2.reshape(-1, WIDTH).sum(axis=0)
    g1 = conv3x3_grad_input(g2, W2) * dsilu(c["z1"])    # dL/dz1
    g["W1"] = conv3x3_grad_weight(g1, c["x"])
    g["b1"] = g1.reshape(-1, WIDTH).sum(axis=0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction (step counts from 1)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


# ---------------------------------------------------------------------------
# features of a state (uses the SBI oracle's spectral machinery)
# ---------------------------------------------------------------------------
def features(solver, eta, phi_s):
    """Unscaled features [ny, nx, 8] and W_lin of one state.

    eta is used as given (it is the elevation the solve sees); its gradient is
    taken from its masked spectrum; phi_s enters through its masked spectrum.
    """
    g = solver.g
    eta = np.asarray(eta, dtype=np.float64).reshape(g.ny, g.nx)
    eh = g.MF(eta)
    ph = g.MF(phi_s)
    wlin = g.ifft(g.k * solver.T * ph)
    ex, ey = g.grad(eh)
    px, py = g.grad(ph)
    if ey is None:
        raise ValueError("the learned warm start is defined on 2D grids")
    f = np.stack([eta, wlin, ex, ey, px, py, solver.delta, eta * wlin], axis=-1)
    return f, wlin


def seed(theta, in_scale, out_scale, solver, eta, phi_s, bf16_acts=True):
    """Physical seeds of the iteration for one state: V0 = W_lin + out_scale[0] y[0]
    and the bottom-potential correction out_scale[1] y[1]."""
    f, wlin = features(solver, eta, phi_s)
    x = (f * np.asarray(in_scale, dtype=np.float32).astype(np.float64))[None]
    y = forward(theta, x, bf16_weights=True, bf16_acts=bf16_acts)[0]
    os_ = np.asarray(out_scale, dtype=np.float32).astype(np.float64)
    return wlin + os_[0] * y[..., 0], os_[1] * y[..., 1]


def labels(solver, eta, phi_s, tol=1e-10):
    """Targets of one state: the nonlinear parts (W* - W_lin, phi_b - phi_b,lin)
    left by the iteration from the linear guess, in physical space."""
    g = solver.g
    ph = g.MF(phi_s)
    saved = (solver.seed, solver._prev)
    solver.seed, solver._prev = "prev", None
    try:
        _, info = solver.w_iter_hat(np.asarray(eta, dtype=np.float64).reshape(g.ny, g.nx), ph, tol)
        dV, dB = solver._prev
    finally:
        solver.seed, solver._prev = saved
    return g.ifft(dV), g.ifft(dB), info


def init_params(seed_value=0):
    """He-style initial weights; the last layer starts at zero so that the
    untrained network reproduces the linear seed exactly."""
    rng = np.random.Generator(np.random.PCG64(seed_value))
    p = {}
    p["W1"] = rng.standard_normal((WIDTH, 9, CIN)) * math.sqrt(2.0 / (9 * CIN))
    p["b1"] = np.zeros(WIDTH)
    p["W2"] = rng.standard_normal((WIDTH, 9, WIDTH)) * math.sqrt(2.0 / (9 * WIDTH))
    p["b2"] = np.zeros(WIDTH)
    p["W3"] = rng.standard_normal((WIDTH, WIDTH)) * math.sqrt(2.0 / WIDTH)
    p["b3"] = np.zeros(WIDTH)
    p["W4"] = np.zeros((2, WIDTH))
    p["b4"] = np.zeros(2)
    return pack(p).astype(np.float32).astype(np.float64)
