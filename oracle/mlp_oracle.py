"""FP64 NumPy reference of the warm-start network (test infrastructure only;
only tests/ may use it).  Shares no code with the HIP kernels.

Network: input z = ((x - x_mean)/x_std, t/t_max)  (n + 1 values), three
hidden layers of width H with the exact GELU, gelu(v) = v Phi(v), and a
linear output of n + 2 values:
    out[:n]   lam_hat        terminal costate at horizon t, divided by lam_scale
    out[n]    log T_hat      predicted minimum time
    out[n+1]  r              bracket half-width delta = softplus(r) + DELTA_MIN
so that [T_hat e^{-delta}, T_hat e^{delta}] is the proposed bracket.

Loss per sample (target lam, log T*, reach mask mk):
    (1/n) sum_i (lam_hat_i - lam_i)^2
  + mk [ (e)^2 + max(0, |e| - delta) + ETA delta ],   e = log T_hat - log T*
averaged over the batch.  Parameters are the flat float vector
[W1 (n+1,H), b1, W2 (H,H), b2, W3 (H,H), b3, W4 (H,n+2), b4].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

DELTA_MIN = 1e-3
ETA = 0.05


def shapes(n, H=256):
    d_in, d_out = n + 1, n + 2
    return [(d_in, H), (H,), (H, H), (H,), (H, H), (H,), (H, d_out), (d_out,)]


def unflatten(theta, n, H=256):
    out, o = [], 0
    for s in shapes(n, H):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def gelu(v):
    return 0.5 * v * (1.0 + erf(v / math.sqrt(2.0)))


def gelu_grad(v):
    return 0.5 * (1.0 + erf(v / math.sqrt(2.0))) + v * np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)


def softplus(r):
    return np.logaddexp(0.0, r)


def sigmoid(r):
    return 0.5 * (1.0 + np.tanh(0.5 * r))


def forward(theta, Z, n, H=256):
    """Returns the output and the cache of pre-activations/activations."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(theta, n, H)
    a1 = Z @ W1 + b1
    h1 = gelu(a1)
    a2 = h1 @ W2 + b2
    h2 = gelu(a2)
    a3 = h2 @ W3 + b3
    h3 = gelu(a3)
    out = h3 @ W4 + b4
    return out, (Z, a1, h1, a2, h2, a3, h3)


def loss_and_grad(theta, Z, Y, n, H=256):
    """Y columns: lam (n), log T* (1), reach mask (1).  Returns (loss, grad)."""
    out, (Z, a1, h1, a2, h2, a3, h3) = forward(theta, Z, n, H)
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(theta, n, H)
    Bn = Z.shape[0]
    lam_hat, lt, r = out[:, :n], out[:, n], out[:, n + 1]
    lam, ltt, mk = Y[:, :n], Y[:, n], Y[:, n + 1]
    delta = softplus(r) + DELTA_MIN
    e = lt - ltt
    miss = np.abs(e) > delta
    per = (np.sum((lam_hat - lam) ** 2, axis=1) / n
           + mk * (e * e + np.maximum(0.0, np.abs(e) - delta) + ETA * delta))
    loss = float(np.mean(per))
    g_out = np.zeros_like(out)
    g_out[:, :n] = 2.0 * (lam_hat - lam) / (n * Bn)
    g_out[:, n] = mk * (2.0 * e + miss * np.sign(e)) / Bn
    g_out[:, n + 1] = mk * (-miss.astype(np.float64) + ETA) * sigmoid(r) / Bn
    gW4 = h3.T @ g_out
    gb4 = g_out.sum(0)
    g3 = (g_out @ W4.T) * gelu_grad(a3)
    gW3 = h2.T @ g3
    gb3 = g3.sum(0)
    g2 = (g3 @ W3.T) * gelu_grad(a2)
    gW2 = h1.T @ g2
    gb2 = g2.sum(0)
    g1 = (g2 @ W2.T) * gelu_grad(a1)
    gW1 = Z.T @ g1
    gb1 = g1.sum(0)
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns new (theta, m, v); t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
