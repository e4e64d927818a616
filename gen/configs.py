"""The five benchmark configurations (shapes, generators, seeds, solver
settings) and the paper's dimensional-scaling workload.  Settings the
configurations leave open are fixed here: t_max = 10 for every system,
trapezoid quadrature, c_tau chosen per system class on the oracle (the
n=100 headline workload's step ratio and certificate interval then measured
on the solver itself: c_tau 2, certificates every 75 iterations, where fewer
FP64 passes outweigh the iterations a probe runs past its certifiable
point), and, where the start points are
unspecified or almost all unreachable, a drift-planted companion
distribution.  The scaling workload keeps the paper's own setting instead
(left rule, N = 100 nodes over the solve's horizon)."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .workloads import (double_integrator, random_system, uniform_box_points, gaussian_points,
                        planted_drift_points, tychastic_double_integrator, tychastic_points,
                        unscented_double_integrator, unscented_points)


@dataclass
class Workload:
    name: str
    systems: list
    x: np.ndarray
    sys_id: np.ndarray | None
    opts: dict = field(default_factory=dict)
    meta: dict = field(default_factory=dict)


def config1(npts=256, seed=1):
    """Double integrator n=2, m=1, |u| <= 1, ball r = 0.1, N = 100 trapezoid,
    t in [0, 10], points uniform in [-2, 2]^2; FP64 iterations."""
    spec = double_integrator(0.1, 100)
    x = uniform_box_points(npts, 2, -2.0, 2.0, seed)
    return Workload("c1_double_integrator", [spec], x, None, dict(prec="fp64", c_tau=30.0))


def config2(npts=65536, seed=2, literal=False):
    """n=50, m=5, N=200, unit l2 ball; literal x ~ N(0, 4I) or the
    drift-planted companion."""
    spec = random_system(50, 5, 200, "l2", seed=1002)
    if literal:
        x = gaussian_points(npts, 50, 2.0, seed)
        meta = dict(points="literal N(0,4I)")
    else:
        x, T0 = planted_drift_points(spec, npts, 0.2, 3.0, seed)
        meta = dict(points="drift-planted T0~U[0.2,3]")
    return Workload("c2_n50_m5_N200", [spec], x, None, dict(prec="fp32", c_tau=5.0), meta)


def config5(npts=65536, seed=5, literal=False):
    """n=100, m=10, N=300, unit l2 ball, ellipsoid target (the metric's
    workload); start points unspecified: drift-planted companion by default."""
    spec = random_system(100, 10, 300, "l2", seed=1005)
    if literal:
        x = gaussian_points(npts, 100, 2.0, seed)
        meta = dict(points="literal N(0,4I)")
    else:
        x, T0 = planted_drift_points(spec, npts, 0.2, 3.0, seed)
        meta = dict(points="drift-planted T0~U[0.2,3]")
    return Workload("c5_n100_m10_N300", [spec], x, None, dict(prec="fp32", c_tau=2.0, check_every=75), meta)


def config3(npts=16384, seed=3, N=400):
    """Precision workload: n=200, m=20, N=400, unit box control, same A/B/W
    generators; x ~ N(0, 4I) (the literal distribution; almost all of these
    points cannot reach the target by t_max, so a min-time query is one
    certified unreachable probe at t_max) and horizons t ~ U[0.5, 10] for the
    value solves that carry the error statement."""
    spec = random_system(200, 20, N, "box", seed=1003)
    x = gaussian_points(npts, 200, 2.0, seed)
    t = np.random.default_rng(seed + 1).uniform(0.5, 10.0, npts)
    return Workload("c3_n200_m20_N400_box", [spec], x, None, dict(prec="bf16x3", c_tau=5.0, wide_min=4096),
                    dict(points="literal N(0,4I)", t=t))


def config4_systems(nsys=64, seed=4):
    """64 systems: n log-uniform in [4, 256], m = max(1, n // 4), N uniform in
    {100..500}, l2 and box control sets 32/32 in random order."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(4.0), np.log(256.0), nsys))).astype(int)
    Ns = rng.integers(100, 501, nsys)
    usets = np.array(["l2"] * (nsys // 2) + ["box"] * (nsys - nsys // 2))
    rng.shuffle(usets)
    specs = [random_system(int(n), max(1, int(n) // 4), int(N), str(u), seed=4000 + k)
             for k, (n, N, u) in enumerate(zip(ns, Ns, usets))]
    for s in specs:       # step ratios chosen on the oracle for the two control sets
        s.c_tau = 5.0 if s.uset == "l2" else 0.3
    return specs


def config4(seed=4, nsys=64, pts_lo=256, pts_hi=4096, scale=1.0):
    """Batched uneven systems: config4_systems, 256-4096 drift-planted points
    per system (T0 ~ U[0.2, 3]), all systems' points mixed in one call in
    random order; x rows padded to the largest n.  `scale` shrinks the point
    counts (for tests)."""
    specs = config4_systems(nsys, seed)
    rng = np.random.default_rng(seed + 100)
    counts = np.maximum(1, (rng.integers(pts_lo, pts_hi + 1, nsys) * scale).astype(int))
    nmax = max(s.A.shape[0] for s in specs)
    xs, ids = [], []
    for k, (s, c) in enumerate(zip(specs, counts)):
        xk, _ = planted_drift_points(s, int(c), 0.2, 3.0, seed=7000 + k)
        pad = np.zeros((int(c), nmax))
        pad[:, :xk.shape[1]] = xk
        xs.append(pad)
        ids.append(np.full(int(c), k, dtype=np.int32))
    x = np.concatenate(xs)
    sid = np.concatenate(ids)
    perm = rng.permutation(len(sid))
    return Workload("c4_batched_uneven", specs, x[perm], sid[perm], dict(prec="fp32", c_tau=1.0),
                    dict(points="drift-planted T0~U[0.2,3] per system", counts=counts.tolist()))


def config_tychastic(d=30, npts=65536, seed=6):
    """The dimensional-scaling experiment (Sec. VI-C): k = d/2 sampled copies
    of the double integrator sharing one control in [-1, 1], each copy's
    start drawn from N((1, 0), 0.0667^2 I) (the spread of Sec. VI-B around
    the start point of Sec. VI-A), target: mean squared terminal distance
    from the origin <= 0.04 (the squared radius 0.2 of Sec. VI-A).  Value
    solves at t = t_max = 2 with the left rule and N = 100 nodes, so every
    solve uses the paper's per-horizon nodes exactly."""
    if d % 2:
        raise ValueError("d must be even")
    k = d // 2
    spec = tychastic_double_integrator(k, ell=0.04, N=100, t_max=2.0, quad="left")
    x = tychastic_points(k, npts, (1.0, 0.0), 0.0667, seed + d)
    return Workload(f"tychastic_d{d}", [spec], x, None, dict(prec="fp32", c_tau=0.5, t=2.0),
                    dict(points="k samples of N((1,0), 0.0667^2 I) per point"))


def config_unscented(npts=65536, seed=7):
    """The unscented control problem of Sec. VI-B: the double integrator's
    five sigma points of N(mu, 0.0667^2 I) (d = 10) sharing one control in
    [-1, 1], target: the weighted mean squared terminal distance from the
    origin <= 0.04; mu uniform in [0.8, 1.2] x [-0.2, 0.2] around the start
    point of Sec. VI-A.  Value solves at t = t_max = 2, left rule, N = 100."""
    spec = unscented_double_integrator(ell=0.04, N=100, t_max=2.0, quad="left")
    x = unscented_points(npts, (0.8, -0.2), (1.2, 0.2), 0.0667, seed)
    return Workload("unscented_d10", [spec], x, None, dict(prec="fp32", c_tau=0.5, t=2.0),
                    dict(points="the 5 sigma points of N(mu, 0.0667^2 I), mu ~ U([0.8,1.2] x [-0.2,0.2])"))


def config_grid(per_axis=50):
    """The level-set experiment of Sec. VI-A: the double integrator with
    |u| <= 1 and the disk of radius 0.2 at the origin, value solves on a
    per_axis x per_axis grid over [-1, 1]^2 (the paper's is 50 x 50) at
    horizons spread over [0, T*], T* the minimum time from (1, 0); the
    paper's own discretisation, left rule with N = 100 nodes per horizon.
    The table's t_max (10) is only used to find T*; each horizon's solves
    use a table built over [0, t]."""
    spec = double_integrator(0.2, 100, t_max=10.0, quad="left")
    g = np.linspace(-1.0, 1.0, per_axis)
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel()], axis=1)
    return Workload(f"double_integrator_grid_{per_axis}", [spec], x, None, dict(prec="fp64", c_tau=10.0),
                    dict(points=f"{per_axis}x{per_axis} grid on [-1,1]^2"))
