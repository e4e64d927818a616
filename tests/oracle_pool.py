"""Run independent oracle solves in worker processes (test infrastructure).

The GPU tests compare sampled device results with the FP64 oracle; at the
shapes of the benchmark workloads one oracle query takes seconds, so the
samples are spread over a few spawned processes (spawned, not forked, so
that no worker inherits the parent's GPU runtime; the workers never touch
the GPU).  Each task carries plain arrays only."""
from __future__ import annotations

import math
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor


def _system(d):
    from oracle import hopf_oracle as O
    return O.System(d["A"], d["B"], d["W"], d.get("c"), d.get("Qu"), uset=d["uset"], N=d["N"],
                    t_max=d["t_max"], quad=d["quad"])


def _min_time_task(args):
    sysd, x, opts, lam0, tb = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import hopf_oracle as O
    r = O.min_time(_system(sysd), x, O.Options(**opts), lam0=lam0, t_bracket=tb)
    return dict(T=r.T, status=r.status, gap=r.gap_n, lo=r.lo, hi=r.hi, probes=r.probes, iters=r.iters)


def _value_task(args):
    sysd, x, t, opts = args
    from oracle import hopf_oracle as O
    pr = O.solve_value(_system(sysd), x, t, O.Options(**opts))
    return dict(phi_lo=pr.phi_lo, phi_hi=pr.phi_hi, gap=pr.gap_n(), iters=pr.iters)


def sysdict(spec, **over):
    d = dict(A=spec.A, B=spec.B, W=spec.W, c=spec.c, Qu=getattr(spec, "Qu", None), uset=spec.uset, N=spec.N,
             t_max=spec.t_max, quad=spec.quad)
    d.update(over)
    return d


def _workers():
    return max(1, min(8, (os.cpu_count() or 2) - 1))


def oracle_min_times(sysd, xs, opts, lam0=None, tbr=None):
    """Oracle min_time of every row of xs (lam0 / tbr rows when given)."""
    tasks = [(sysd, xs[i], opts, None if lam0 is None else lam0[i], None if tbr is None else tbr[i])
             for i in range(len(xs))]
    with ProcessPoolExecutor(max_workers=_workers(), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_min_time_task, tasks))


def oracle_values(sysd, xs, ts, opts):
    tasks = [(sysd, xs[i], float(ts[i]), opts) for i in range(len(xs))]
    with ProcessPoolExecutor(max_workers=_workers(), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_value_task, tasks))


def same_min_time(dev_T, dev_status, dev_gap, o, gap_tol=1e-6):
    """The parity bar for one minimum-time query: identical status; for a
    reached point |dT| <= 1e-4 T and the device's final gap <= gap_tol; an
    unreachable point has T = +inf on both sides."""
    if int(dev_status) != int(o["status"]):
        return False, f"status {int(dev_status)} vs oracle {o['status']}"
    if o["status"] == 0:
        if not (abs(dev_T - o["T"]) <= 1e-4 * o["T"]):
            return False, f"T {dev_T} vs oracle {o['T']}"
        if not (dev_gap <= gap_tol):
            return False, f"gap {dev_gap}"
    if o["status"] == 2 and not math.isinf(dev_T):
        return False, f"unreachable but T = {dev_T}"
    return True, ""
