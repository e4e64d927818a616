"""Benchmark: minimum-time queries per second at certified gap <= 1e-6 on
the n=100, m=10, N=300 workload (one MI355X).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--npts 65536]

A step is one hopf_min_time_dev call over the whole batch (every query runs
its bisection and PDHG solves to a certified result) with the inputs already
resident in device memory.  Prints one JSON line.  The oracle's CPU rate on a
bounded sample of the same workload is reported as cpu_baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
METRIC = "min-time queries/sec at dual gap≤1e-6 (n=100,N=300): plain vs warm-start"


def _oracle_query(args):
    """One oracle min-time query (run in a worker process)."""
    spec, x, opts = args
    from oracle import hopf_oracle as O
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    r = O.min_time(S, x, O.Options(c_tau=opts.get("c_tau", 1.0)))
    return r.status, r.T, r.iters


def cpu_baseline(w, nsample, workers):
    """The FP64 oracle, as it stands, on the first `nsample` queries of the
    batch, one query per worker process (one thread each)."""
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    os.environ.setdefault("MKL_NUM_THREADS", "1")
    jobs = [(w.systems[0], w.x[i], w.opts) for i in range(nsample)]
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_query, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    return nsample / dt, dt, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--npts", type=int, default=65536)
    ap.add_argument("--warm", default="cold", choices=["cold", "cont"])
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle queries, first ones of the batch (0 = one per worker, 8 workers)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the queries are independent, "
              "so a multi-GPU run is the single-GPU run on a shard of the points.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from gen.configs import config5
    from paper_1712_08226_amd import Solver

    w = config5(npts=args.npts)
    spec = w.systems[0]
    dev = torch.device("cuda:0")
    solver = Solver(0)
    solver.set_systems([spec])
    solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], warm=args.warm)
    npts = w.x.shape[0]
    x = torch.tensor(w.x, dtype=torch.float64, device=dev)
    T = torch.empty(npts, dtype=torch.float64, device=dev)
    gap = torch.empty(npts, dtype=torch.float64, device=dev)
    status = torch.empty(npts, dtype=torch.int32, device=dev)
    probes = torch.empty(npts, dtype=torch.int32, device=dev)
    iters = torch.empty(npts, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        solver.min_time_dev(x, T, gap, status, probes=probes, iters=iters, stream=stream)

    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for i in range(args.warmup):
        step()
        print(f"warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tk, launches, rows = 0.0, 0, 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        tm = solver.last_timing()
        tk += tm["iter_kernel_s"]
        launches += tm["iter_launches"]
        rows += tm["point_rows"]
        print(f"step {i + 1}/{args.steps}: device {tm['total_s']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    qps = npts * args.steps / dt

    st = status.cpu().numpy()
    Tn = T.cpu().numpy()
    gn = gap.cpu().numpy()
    itn = iters.cpu().numpy()
    ok = st == 0
    flops = 4.0 * spec.m * spec.n * rows           # algorithmic: K lam and K^T y per point-row
    achieved = flops / tk / 1e12 if tk > 0 else 0.0
    per_launch_ms = 1e3 * tk / max(1, launches)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                "kernel": "k_pdhg (fused FP32 PDHG iterations)", "avg_launch_ms": round(per_launch_ms, 4),
                "launches": launches}
    out = {"metric": METRIC, "value": round(qps, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"min-time, n={spec.n} m={spec.m} N={spec.N} l2 control, ellipsoid target, "
                                  f"t_max={spec.t_max}, trapezoid, {npts} {w.meta.get('points')} points",
                      "npts": npts, "n": spec.n, "m": spec.m, "N": spec.N, "warm": args.warm,
                      "c_tau": w.opts["c_tau"], "gap_tol": 1e-6, "certificate": "fp64"},
           "results": {"ok": int(ok.sum()), "inside": int((st == 1).sum()), "unreachable": int((st == 2).sum()),
                       "noconv": int((st == 3).sum()), "nonfinite": int((st == 4).sum()),
                       "median_T": float(np.median(Tn[ok])) if ok.any() else None,
                       "max_gap_ok": float(gn[ok].max()) if ok.any() else None,
                       "mean_iters": float(itn.mean()),
                       "iters_p50_p90_p99_max": [float(v) for v in np.percentile(itn, [50, 90, 99, 100])],
                       "mean_probes": float(probes.cpu().numpy().mean())},
           "roofline": roofline}
    if not args.no_cpu:
        workers = min(8, os.cpu_count() or 1)
        ns = args.cpu_sample or workers
        cq, cdt, res = cpu_baseline(w, ns, workers)
        out["cpu_baseline"] = {"value": round(cq, 4), "unit": "queries/s", "cores": workers, "kind": "oracle",
                               "sample": f"first {ns} queries of the batch, one per process, {cdt:.1f} s wall"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
