"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.

This module only draws random systems and query points.  It contains none of
the solver's arithmetic (no node table, quadrature, Hopf objective or
primal-dual step); the one library matrix exponential here moves a start
point under free motion (zero control) to plant it, so the oracle and the
HIP path can both read its output without sharing any of the method.

Workload shapes follow the paper's examples and the configurations the
library is benchmarked on:
  * the double integrator of Sec. VI-A (n=2, m=1, |u| <= 1, ball target);
  * its tychastic (sampled initial state) extension of Sec. VI-B/C: k copies
    sharing one control, d = 2k, a mean-squared-error target, with either
    random samples (equal weights) or the 5 sigma points of the unscented
    transform (d = 10, weighted target);
  * random stable-ish linear systems: A = S diag(eig) S^{-1} with
    eig ~ U[-1, 0.2] and S_ij ~ N(0, 1/n), B_ij ~ N(0,1)/sqrt(n), an
    axis-aligned ellipsoid target W = diag(q), q ~ U[0.05, 0.2], and either
    the unit l2 ball or the unit box as control set;
  * query points either literal (uniform box / isotropic Gaussian) or a
    "calibrated" isotropic Gaussian whose scale puts most points inside the
    reachable band.
All randomness comes from numpy.random.default_rng(seed).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SystemSpec:
    """Plain description of one system (all float64, row-major)."""
    A: np.ndarray
    B: np.ndarray
    W: np.ndarray
    c: np.ndarray
    uset: str            # "l2" or "box"
    N: int
    t_max: float
    quad: str            # "trap" or "left"
    name: str = ""
    c_tau: float = 0.0   # the system's primal step ratio for the solver (0: the call's)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def m(self):
        return self.B.shape[1]


def double_integrator(r=0.1, N=100, t_max=10.0, quad="trap"):
    """Sec. VI-A: position/velocity, scalar control in [-1, 1], ball target of
    radius r at the origin (W = r^2 I)."""
    A = np.array([[0.0, 1.0], [0.0, 0.0]])
    B = np.array([[0.0], [1.0]])
    W = (r * r) * np.eye(2)
    return SystemSpec(A, B, W, np.zeros(2), "box", N, t_max, quad, f"double_integrator_r{r}")


def tychastic_double_integrator(k, ell=0.04, N=100, t_max=2.0, quad="left"):
    """Sec. VI-B/C: k copies of the double integrator that share one scalar
    control in [-1, 1] (state dimension d = 2k, A~ = I_k (x) A, B~ = 1_k (x) B),
    with the terminal cost that bounds the mean squared distance of the k
    terminal states from the origin by ell.  In the ellipsoid form used here,
    {z : z^T W^-1 z <= 1}, that target is W = ell k I_d (the paper's shape
    k I_d, scaled by the threshold).  With ell = r^2 and k equal copies the
    problem is the single double integrator with a ball target of radius r."""
    A2 = np.array([[0.0, 1.0], [0.0, 0.0]])
    B2 = np.array([[0.0], [1.0]])
    A = np.kron(np.eye(k), A2)
    B = np.kron(np.ones((k, 1)), B2)
    d = 2 * k
    return SystemSpec(A, B, (ell * k) * np.eye(d), np.zeros(d), "box", N, t_max, quad,
                      f"tychastic_double_integrator_k{k}")


def tychastic_points(k, npts, mu, std, seed):
    """Each query point stacks k independent samples chi_i ~ N(mu, std^2 I_2)
    of the uncertain initial state (the randomly sampled variant of the
    unscented construction)."""
    rng = np.random.default_rng(seed)
    return (np.asarray(mu, dtype=np.float64)[None, None, :]
            + std * rng.normal(size=(npts, k, 2))).reshape(npts, 2 * k)


def unscented_weights(n, alpha=1.0, kappa=None):
    """Mean weights of the 2n+1 sigma points of the scaled unscented transform
    (Julier 2002; Thrun et al. 2005, Sec. 3.4): lam = alpha^2 (n + kappa) - n,
    w_0 = lam / (n + lam), w_i = 1 / (2 (n + lam)).  kappa defaults to 3 - n,
    which with alpha = 1 keeps every weight positive for n = 2 (1/3 and 1/6)."""
    if kappa is None:
        kappa = 3.0 - n
    lam = alpha * alpha * (n + kappa) - n
    w = np.full(2 * n + 1, 1.0 / (2.0 * (n + lam)))
    w[0] = lam / (n + lam)
    return w, lam


def unscented_double_integrator(ell=0.04, N=100, t_max=2.0, quad="left"):
    """Sec. VI-B: the double integrator augmented by its 2n+1 = 5 sigma points
    (d = 10), one shared scalar control in [-1, 1], and the target that bounds
    the weighted mean squared distance sum_i w_i |chi_i(T)|^2 of the terminal
    sigma points from the origin by ell.  In the ellipsoid form {z : z^T W^-1 z
    <= 1} that is W = blockdiag((ell / w_i) I_2), the paper's blocks
    w_i^-1 I_2 scaled by the threshold."""
    A2 = np.array([[0.0, 1.0], [0.0, 0.0]])
    B2 = np.array([[0.0], [1.0]])
    w, _ = unscented_weights(2)
    k = len(w)
    W = np.kron(np.diag(ell / w), np.eye(2))
    return SystemSpec(np.kron(np.eye(k), A2), np.kron(np.ones((k, 1)), B2), W, np.zeros(2 * k), "box", N,
                      t_max, quad, "unscented_double_integrator")


def unscented_points(npts, mu_lo, mu_hi, std, seed):
    """Each query point stacks the 2n+1 sigma points (mu; mu + s e_i; mu - s e_i,
    s = std sqrt(n + lam)) of x0 ~ N(mu, std^2 I_2), mu uniform in the box
    [mu_lo, mu_hi]; the weighted sigma points reproduce mu and std^2 I_2."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(np.asarray(mu_lo, dtype=np.float64), np.asarray(mu_hi, dtype=np.float64), size=(npts, 2))
    _, lam = unscented_weights(2)
    s = std * np.sqrt(2.0 + lam)
    off = np.concatenate([np.zeros((1, 2)), s * np.eye(2), -s * np.eye(2)])
    return (mu[:, None, :] + off[None, :, :]).reshape(npts, 10)


def random_system(n, m, N, uset, seed, t_max=10.0, quad="trap",
                  eig_lo=-1.0, eig_hi=0.2, q_lo=0.05, q_hi=0.2):
    """Random linear system by a seeded similarity transform (see module doc)."""
    rng = np.random.default_rng(seed)
    eig = rng.uniform(eig_lo, eig_hi, size=n)
    S = rng.normal(0.0, 1.0 / np.sqrt(n), size=(n, n))
    A = S @ np.diag(eig) @ np.linalg.inv(S)
    B = rng.normal(0.0, 1.0, size=(n, m)) / np.sqrt(n)
    q = rng.uniform(q_lo, q_hi, size=n)
    return SystemSpec(A, B, np.diag(q), np.zeros(n), uset, N, t_max, quad,
                      f"random_n{n}_m{m}_N{N}_{uset}_s{seed}")


def uniform_box_points(npts, n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(npts, n))


def gaussian_points(npts, n, std, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=(npts, n))


def planted_drift_points(spec, npts, T0_lo, T0_hi, seed, levels=64):
    """Points that reach the target's boundary at time T0 under zero control:
    x0 = e^{-T0 A} xi with xi uniform on the ellipsoid's boundary and T0 on a
    grid of `levels` values in [T0_lo, T0_hi] (free motion only, no control
    and no part of the solver).  Their minimum time is at most T0 whenever
    the sign of the value is monotone; the spread of T0 spreads the
    minimum times of the batch.  Returns (x0, T0)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(seed)
    n = spec.n
    grid = np.linspace(T0_lo, T0_hi, levels)
    E = np.stack([expm(-t * spec.A) for t in grid])
    idx = rng.integers(0, levels, size=npts)
    g = rng.normal(size=(npts, n))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    semi = np.sqrt(np.diag(spec.W))
    xi = spec.c + g * semi
    x0 = np.einsum("pij,pj->pi", E[idx], xi)
    return x0, grid[idx]
