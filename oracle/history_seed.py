"""FP64 oracle of the learned history seed of the W iteration.  TEST
INFRASTRUCTURE ONLY.

The second layer of the learned warm start (the first is the convolution
network of ``warmstart``, which starts solves that have no history).  In
fixed-step time stepping (integrating-factor RK4, Sec. 2.2) every step makes
four W solves, at stages s = 0, 1, 2, 3 (states at t, t + h/2, t + h/2, t + h).
The nonlinear part of a converged solve is the pair of masked half spectra

    N_V = V* - k tanh(kh) phi_hat,      N_B = phi_b - sech(kh) phi_hat

(the second only over a variable bed).  The history layer predicts the
nonlinear part of the solve at stage s from those of the K solves before it,
h_0 (the most recent) .. h_(K-1), through their backward differences

    d_q = sum_{j <= q} (-1)^j C(q, j) h_j      (d_0 = h_0, d_1 = h_0 - h_1, ...),

mode by mode with complex weights that depend on the stage and on |k|
through nb radial bins of width dk:

    pred_P(k) = sum_{q < K} w[P, s, b(k), q] d_q,P(k),   P in {V, B},
    b(k) = min(floor(|k| / dk), nb - 1),

a spectral layer (per-mode weights mixing K history channels).  The iteration
starts from V0 = k tanh(kh) phi_hat + pred_V and phi_b0 = sech(kh) phi_hat +
pred_B; its residual test is unchanged, so the seed affects only the number of
sweeps.  With w[., ., ., 0] = 1 and the other weights 0 it is the
previous-solve seed; w = 1 for every q is Newton's backward-difference
extrapolation one (uniform) step ahead.

Training minimises, over fixed-step solves with a full history, the sum of

    L = sum_P  sum_k c_k |pred_P - N_P|^2 / D_P,   D_P = sum_k c_k |N_P|^2

(c_k = 1 at m_x = 0, else 2: the real-field weight of a half-spectrum mode;
the sums run over the kept modes; a part with D_P = 0 contributes nothing).
Per (P, s, b) the loss is a complex least-squares problem in w: with
G = sum c conj(d) d^T / D (K x K, Hermitian) and z = sum c conj(d) N / D,
gamma = G w - z is the derivative with respect to conj(w), and the gradient
with respect to the real and imaginary parts of w is (2 Re gamma, 2 Im gamma).
Two optimisers: Adam with bias correction on that gradient, and the
Gauss-Newton (here exact Newton) step w <- w - (G + lam tr(G)/K I)^-1 gamma,
which lands on the ridge-regularised least-squares weights in one step.

Parameter vector (FP32): w[P][s][b][q][re, im], P = 2, s = 4, b = nb, q = K.
"""
from __future__ import annotations

from math import comb

import numpy as np

STAGES = 4


def param_count(K: int, nb: int) -> int:
    return 2 * STAGES * nb * K * 2


def to_complex(theta, K, nb):
    """(2, 4, nb, K) complex view of the flat FP32 parameter vector."""
    t = np.asarray(theta, dtype=np.float64).reshape(2, STAGES, nb, K, 2)
    return t[..., 0] + 1j * t[..., 1]


def to_flat(W):
    W = np.asarray(W)
    return np.stack([W.real, W.imag], axis=-1).ravel()


def identity(K, nb):
    """Weights of the previous-solve seed: w_0 = 1, the rest 0."""
    W = np.zeros((2, STAGES, nb, K), complex)
    W[..., 0] = 1.0
    return to_flat(W).astype(np.float32)


def bins(grid, dk, nb):
    """Radial bin of every half-spectrum mode of the oracle's grid."""
    return np.minimum(np.floor(grid.k / dk).astype(np.int64), nb - 1)


def mode_weights(grid):
    """c_k: 1 at m_x = 0, 2 elsewhere, on kept modes only."""
    c = np.where(np.arange(grid.k.shape[1])[None, :] == 0, 1.0, 2.0)
    return c * grid.mask


def differences(hist, P):
    """Backward differences d_q of part P of the history [(N_V, N_B) newest first]."""
    K = len(hist)
    return [sum((-1) ** j * comb(q, j) * hist[j][P] for j in range(q + 1)) for q in range(K)]


def predict(W, hist, stage, b):
    """Predicted (N_V, N_B) from the history (None for a part it lacks)."""
    out = []
    for P in range(2):
        if any(h[P] is None for h in hist):
            out.append(None)
            continue
        d = differences(hist, P)
        out.append(sum(W[P, stage, b, q] * d[q] for q in range(len(hist))))
    return out[0], out[1]


def loss_grad(W, hist, target, stage, b, c, nb):
    """Loss of one solve, its gradient as (2, nb, K) complex (real part:
    d/d re w, imaginary part: d/d im w), and its Gram matrices G (2, nb, K, K)."""
    K = len(hist)
    grad = np.zeros((2, nb, K), complex)
    gram = np.zeros((2, nb, K, K), complex)
    loss = 0.0
    for P in range(2):
        y = target[P]
        if y is None:
            continue
        D = float(np.sum(c * np.abs(y) ** 2))
        if not D > 0.0:
            continue
        d = differences(hist, P)
        pred = sum(W[P, stage, b, q] * d[q] for q in range(K))
        r = pred - y
        loss += float(np.sum(c * np.abs(r) ** 2)) / D

        def binsum(f):
            return (np.bincount(b.ravel(), weights=f.real.ravel(), minlength=nb) +
                    1j * np.bincount(b.ravel(), weights=f.imag.ravel(), minlength=nb))

        for q in range(K):
            grad[P, :, q] = 2.0 * binsum(c * np.conj(d[q]) * r / D)
            for s in range(K):
                gram[P, :, q, s] = binsum(c * np.conj(d[q]) * d[s] / D)
    return loss, grad, gram


def newton(W, grad_sum, gram_sum, lam):
    """Gauss-Newton step on the summed gradient and Gram matrices of each
    (part, stage, bin): w - (G + lam tr(G)/K I)^-1 gamma with gamma the
    complex derivative (grad / 2); systems with tr(G) = 0 are left alone."""
    W = np.array(W, dtype=complex)
    P_, S_, B_, K = W.shape
    for P in range(P_):
        for s in range(S_):
            for bb in range(B_):
                G = gram_sum[P, s, bb]
                tr = float(np.trace(G).real)
                if not tr > 0.0:
                    continue
                A = G + lam * tr / K * np.eye(K)
                W[P, s, bb] = W[P, s, bb] - np.linalg.solve(A, grad_sum[P, s, bb] / 2.0)
    return W


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step on FP32 masters (all arrays flat)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
