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


def test_adam_bias_correction_over_several_steps():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each step
    moves a parameter by lr g / (|g| + eps): after t steps theta = -t lr g/(|g|+eps).
    A correction with the wrong power of b1 or b2 breaks this from t = 2 on."""
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    lr, eps = 0.01, 1e-8
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        th, m, v = M.adam_step(th, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(th, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)


def test_adam_second_step_by_hand():
    """Gradients 1 then -1 (b1 = 0.9, b2 = 0.999, lr = 1): after step 2
    m = 0.9*0.1 - 0.1 = -0.01, v = 0.999*0.001 + 0.001 = 0.001999, mh = -0.01/0.19,
    vh = 0.001999/0.001999 = 1, so theta moves by +0.01/0.19 (+ the first step's -1)."""
    th, m, v = M.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, 1.0, eps=0.0)
    th, m, v = M.adam_step(th, -np.ones(1), m, v, 2, 1.0, eps=0.0)
    np.testing.assert_allclose(m, [-0.01], rtol=1e-12)
    np.testing.assert_allclose(v, [0.001999], rtol=1e-12)
    np.testing.assert_allclose(th, [-1.0 + 0.01 / 0.19], rtol=1e-12)
