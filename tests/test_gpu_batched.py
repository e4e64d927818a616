"""Batched uneven systems: points of several systems (different n, m, N,
control sets and quadrature rules) mixed in one call.  Each system's points
must come out exactly as in a call with that system alone (same kernels, same
tiles, same arithmetic), and sampled points must match the FP64 oracle."""
import sys

import numpy as np
import pytest

from gen import random_system
from gen.workloads import planted_drift_points
from oracle import hopf_oracle as O

pytestmark = pytest.mark.gpu

SHAPES = [(6, 1, 60, "l2", "trap"), (20, 5, 80, "box", "trap"), (40, 10, 50, "l2", "trap"),
          (70, 17, 40, "box", "trap"), (12, 3, 100, "l2", "left")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_1712_08226_amd import Solver
    s = Solver(0)
    yield s
    s.close()


def batch(npts_each=30, seed=0):
    specs = [random_system(n, m, N, u, seed=600 + k, t_max=4.0, quad=q) for k, (n, m, N, u, q) in enumerate(SHAPES)]
    nmax = max(n for n, *_ in SHAPES)
    xs, ids = [], []
    for k, s in enumerate(specs):
        xk, _ = planted_drift_points(s, npts_each + 3 * k, 0.2, 2.5, seed=80 + k)
        pad = np.zeros((len(xk), nmax))
        pad[:, :xk.shape[1]] = xk
        xs.append(pad)
        ids.append(np.full(len(xk), k, dtype=np.int32))
    x, sid = np.concatenate(xs), np.concatenate(ids)
    perm = np.random.default_rng(seed).permutation(len(sid))
    return specs, x[perm], sid[perm]


@pytest.mark.parametrize("mode,tail", [("min_time", 0), ("value", 0), ("min_time", 512), ("value", 512)])
def test_batched_equals_single_system_calls(solver, mode, tail):
    """tail=0: every job runs its own rounds on a pool of streams; tail=512:
    every job is parked and one combined tail launch finishes all systems."""
    say("case: batched", mode, "tail", tail)
    specs, x, sid = batch()
    solver.set_systems(specs)
    solver.set_opts(prec="fp32", c_tau=1.0, warm="cont", tail_max=tail)
    t = np.linspace(0.3, 3.9, len(sid))
    if mode == "min_time":
        rb = solver.min_time(x, sys_id=sid)
    else:
        rb = solver.value(x, t, sys_id=sid)
    tm = solver.last_timing()
    assert tm["alg_flops"] > 0
    assert (tm["tail_points"] > 0) == (tail > 0)
    for k, s in enumerate(specs):
        sel = np.flatnonzero(sid == k)
        n = s.A.shape[0]
        solver.set_systems([s])
        if mode == "min_time":
            r1 = solver.min_time(x[sel, :n])
            keys = ["T", "gap", "status", "probes", "iters"]
        else:
            r1 = solver.value(x[sel, :n], t[sel])
            keys = ["phi_lo", "phi_hi", "status", "iters"]
        for key in keys:
            assert np.array_equal(rb[key][sel], r1[key], equal_nan=True), (k, key)
        assert np.array_equal(rb["lam"][sel, :n], r1["lam"]), k
        solver.set_systems(specs)
    say("statuses", np.bincount(rb["status"], minlength=5))


def test_batched_min_time_vs_oracle(solver):
    say("case: batched vs oracle")
    specs, x, sid = batch(npts_each=20, seed=1)
    solver.set_systems(specs)
    solver.set_opts(prec="fp32", c_tau=1.0, warm="cont")
    r = solver.min_time(x, sys_id=sid)
    for k, s in enumerate(specs):
        S = O.System(s.A, s.B, s.W, s.c, uset=s.uset, N=s.N, t_max=s.t_max, quad=s.quad)
        n = s.A.shape[0]
        for i in np.flatnonzero(sid == k)[:2]:
            # the oracle keeps fixed steps, so it gets a larger iteration budget
            o = O.min_time(S, x[i, :n], O.Options(c_tau=1.0, warm="cont", max_iter=2000000))
            assert r["status"][i] == o.status, (k, i, r["status"][i], o.status)
            if o.status == O.PT_OK:
                assert abs(r["T"][i] - o.T) <= 1e-4 * o.T, (k, i, r["T"][i], o.T)
                assert r["gap"][i] <= 1e-6


def test_batched_rejects_bad_stride_and_ids(solver):
    specs, x, sid = batch(npts_each=4)
    solver.set_systems(specs)
    with pytest.raises(ValueError):
        solver.min_time(x[:, :10], sys_id=sid)
    bad = sid.copy()
    bad[0] = 99
    with pytest.raises(Exception):
        solver.min_time(x, sys_id=bad)
