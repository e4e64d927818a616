"""The five benchmark configurations (shapes, generators, seeds, solver
settings).  Settings the configurations leave open are fixed here: t_max = 10
for every system, trapezoid quadrature, c_tau chosen per system class on the
oracle, and, where the start points are unspecified or almost all
unreachable, a drift-planted companion distribution."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .workloads import (double_integrator, random_system, uniform_box_points, gaussian_points,
                        planted_drift_points)


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
    return Workload("c5_n100_m10_N300", [spec], x, None, dict(prec="fp32", c_tau=5.0), meta)
