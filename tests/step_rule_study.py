"""Iterations of the oracle's step rules (fixed, accelerated, diagonally
preconditioned; Sec. III and III-A) to a certified normalised gap of 1e-6:
value solves at the planted horizon T0 of drift-planted points, cold start,
on the n=100, m=10, N=300 l2 system of the headline workload and on an
n=64, m=16, N=300 box system.  Run: python -m tests.step_rule_study
(CPU only; the oracle in a process pool)."""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CAP = 200_000


def _solve(args):
    name, spec, x, T, steps, c_tau = args
    from oracle import hopf_oracle as O
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    t0 = time.perf_counter()
    pr = O.solve_value(S, x, T, O.Options(c_tau=c_tau, steps=steps, max_iter=CAP))
    return name, steps, c_tau, pr.iters, pr.gap_n() <= 1e-6, time.perf_counter() - t0


def main(npts=8):
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    from gen import random_system
    from gen.configs import config5
    from gen.workloads import planted_drift_points
    systems = {"l2 n100 m10 N300": (config5(npts=8).systems[0], [("fixed", 2.0), ("accel", 2.0),
                                                                  ("precond", 0.5), ("precond", 1.0),
                                                                  ("precond", 2.0), ("precond", 4.0),
                                                                  ("precond", 8.0)]),
               "box n64 m16 N300": (random_system(64, 16, 300, "box", seed=77), [("fixed", 0.3), ("accel", 0.3),
                                                                               ("precond", 0.1), ("precond", 0.3),
                                                                               ("precond", 1.0)])}
    jobs = []
    for name, (spec, rules) in systems.items():
        x, T0 = planted_drift_points(spec, npts, 0.2, 3.0, 21)
        for steps, c_tau in rules:
            jobs += [(name, spec, x[i], float(T0[i]), steps, c_tau) for i in range(npts)]
    res = {}
    with mp.get_context("spawn").Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        for name, steps, c_tau, it, ok, sec in pool.imap_unordered(_solve, jobs):
            r = res.setdefault((name, steps, c_tau), [0, 0, 0.0])
            r[0] += it
            r[1] += 0 if ok else 1
            r[2] += sec
            print(f"{name} {steps} c_tau={c_tau}: {it} iterations{'' if ok else ' (cap)'}", flush=True)
    print("\n| system | step rule | c_tau | iterations, sum over the points | points at the cap |")
    print("|---|---|---|---|---|")
    for (name, steps, c_tau), (it, cap, sec) in sorted(res.items()):
        print(f"| {name} | {steps} | {c_tau} | {it} | {cap} |")


if __name__ == "__main__":
    main()
