"""Pins for the FP64 warm-start network reference: closed-form activation
values, central finite differences of the loss, and a hand-checked Adam step."""
import math

import numpy as np
from scipy.stats import norm

from oracle import mlp_oracle as M


def test_gelu_closed_form_and_derivative():
    v = np.linspace(-4, 4, 41)
    np.testing.assert_allclose(M.gelu(v), v * norm.cdf(v), atol=1e-15)
    h = 1e-6
    fd = (M.gelu(v + h) - M.gelu(v - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(v), fd, atol=1e-8)


def _problem(n=5, H=16, B=12, seed=0):
    rng = np.random.default_rng(seed)
    shp = M.shapes(n, H)
    theta = np.concatenate([rng.normal(0, 0.4, int(np.prod(s))) for s in shp])
    Z = rng.normal(size=(B, n + 1))
    Y = np.zeros((B, n + 2))
    Y[:, :n] = rng.normal(size=(B, n))
    Y[:, n] = rng.normal(0, 0.5, B)
    Y[:, n + 1] = (rng.uniform(size=B) < 0.7).astype(float)
    return theta, Z, Y, n, H


def test_loss_gradient_matches_finite_differences():
    theta, Z, Y, n, H = _problem()
    loss, g = M.loss_and_grad(theta, Z, Y, n, H)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(theta), 60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (M.loss_and_grad(tp, Z, Y, n, H)[0] - M.loss_and_grad(tm, Z, Y, n, H)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_terms_closed_form():
    """With zero weights the output is the output bias: check the loss value."""
    n, H = 3, 4
    theta = np.zeros(sum(int(np.prod(s)) for s in M.shapes(n, H)))
    b4 = np.array([0.5, -1.0, 2.0, math.log(2.0), 0.3])
    theta[-(n + 2):] = b4
    Z = np.zeros((1, n + 1))
    Y = np.array([[0.0, 0.0, 0.0, 0.0, 1.0]])
    loss, _ = M.loss_and_grad(theta, Z, Y, n, H)
    delta = math.log1p(math.exp(0.3)) + M.DELTA_MIN
    e = math.log(2.0)
    exact = (0.25 + 1.0 + 4.0) / 3 + e * e + max(0.0, e - delta) + M.ETA * delta
    assert abs(loss - exact) <= 1e-14


def test_adam_first_step_is_signed_lr():
    """After one Adam step from zero moments every parameter moves by lr*sign(g)
    (up to eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-4)
