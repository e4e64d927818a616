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
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
METRIC = "min-time queries/sec at dual gap≤1e-6 (n=100,N=300): plain vs warm-start"


KERNEL_SRC = os.path.join(ROOT, "paper_1712_08226_amd", "csrc", "hopf_device.h")
COUNTERS = os.path.join(ROOT, "profiles", "pdhg_n100_m10_N300_65536q_hbm_counters.md")


def counter_traffic(variant, check_every, c_tau, kernel):
    """HBM bytes per launch of an iteration kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs of this workload ('traffic:' JSON
    lines in the summary, one per profiled kernel and warm-start variant), or
    None when no record matches the kernel, variant, iterations per launch and
    step ratio of this run, or the kernel source has changed since the
    counters were taken."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            recs = [json.loads(l[len("traffic:"):]) for l in f if l.startswith("traffic:")]
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    for rec in recs:
        if (rec.get("kernel_source_sha256") == sha and rec.get("kernel") == kernel and rec.get("variant") == variant
                and rec.get("check_every") == check_every and rec.get("c_tau") == c_tau):
            return rec
    return None


def single_thread_workers():
    """One BLAS/OpenMP thread in every oracle worker started after this call
    (spawned workers read these at start-up).  Assigned, not defaulted: the
    environment may already ask for one thread per core, and as many workers
    as cores each spinning that many threads would measure contention, not
    the oracle."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[k] = "1"


def _oracle_query(args):
    """One oracle min-time query (run in a worker process); returns its
    status, T and wall seconds."""
    spec, x, opts = args
    from oracle import hopf_oracle as O
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    t0 = time.perf_counter()
    r = O.min_time(S, x, O.Options(**opts))
    return r.status, r.T, time.perf_counter() - t0


def _oracle_value_full(args):
    """One oracle value solve phi(x, t) (run in a worker process); returns
    the job's index, the certified interval, lambda, iterations and wall
    seconds."""
    k, spec, x, t, opts = args
    from oracle import hopf_oracle as O
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    t0 = time.perf_counter()
    pr = O.solve_value(S, x, t, O.Options(**opts))
    return k, -pr.P, -pr.D, pr.lam, pr.iters, time.perf_counter() - t0


def host_info():
    """CPU model, logical CPUs, and the NumPy / BLAS build of this host."""
    import platform
    import numpy as np
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg.get("Build Dependencies", {}).get("blas", {}).get("name")
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "numpy": np.__version__, "blas": blas}


def cpu_baseline(spec, xs, opts, workers):
    """The FP64 oracle, as it stands, on a fixed sample of queries run to
    completion, one query per worker process (one thread each).  The rate is
    the sample's queries over the wall time of the pool; the per-query times
    and statuses are returned as well."""
    import multiprocessing as mp
    import numpy as np
    single_thread_workers()
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_query, [(spec, x, opts) for x in xs], chunksize=1)
    wall = time.perf_counter() - t0
    per = np.array([r[2] for r in res])
    st = np.bincount([r[0] for r in res], minlength=5).tolist()
    return len(xs) / wall, wall, per, st


def stratified_sample(T0, k):
    """k query indices spread evenly over the planted times T0 (sorted), so
    that short and long queries are represented in proportion."""
    import numpy as np
    order = np.argsort(T0, kind="stable")
    return order[np.linspace(0, len(order) - 1, k).astype(int)]


DECLARED_WARM = "cont"     # the warm-start form timed for `value` (declared, not chosen by the run)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--npts", type=int, default=65536)
    ap.add_argument("--warm", default=DECLARED_WARM,
                    help="warm start of the timed form (cont: the previous probe's iterate; mlp_first / mlp_lam / "
                         "mlp: the learned start, trained first on separate queries), optionally +newton for the "
                         "Sec. IV hybrid search")
    ap.add_argument("--plain-budget", type=float, default=60.0,
                    help="seconds of timed steps for the plain form (cold start at every probe); at least one step")
    ap.add_argument("--literal-budget", type=float, default=40.0,
                    help="seconds of timed steps for the literal start points x ~ N(0, 4I); at least one step")
    ap.add_argument("--train-npts", type=int, default=65536, help="training queries for the learned warm start")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--cpu-sample", type=int, default=96, help="oracle queries in the CPU baseline sample")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle worker processes (one thread each)")
    ap.add_argument("--cpu-budget", type=float, default=30.0, help="seconds of oracle wall time (value workloads)")
    ap.add_argument("--c3-sample", type=int, default=8,
                    help="c3: points (evenly spaced) solved by the oracle for the CPU rate and the error line")
    ap.add_argument("--workload", default="c5", choices=["c5", "c2", "c1", "c3", "c4", "tychastic", "grid", "tune"],
                    help="c5: the headline min-time workload (default); c2 (n=50, m=5, N=200) and c1 (the "
                         "double integrator, FP64, points uniform in [-2,2]^2): the same legs on those "
                         "systems; c3: BF16 hi+lo precision "
                         "workload with its BF16 / FP32 difference; c4: 64 uneven systems in one call; "
                         "tychastic: the paper's dimensional-scaling value solves, d = 2k sampled copies; "
                         "grid: the paper's double-integrator level-set grid at ten horizons")
    ap.add_argument("--dims", default="30,60,90,120", help="tychastic: state dimensions d to sweep")
    ap.add_argument("--c4-scale", type=float, default=0.05, help="c4: fraction of each system's points")
    ap.add_argument("--c4-max-iter", type=int, default=20000, help="c4: iteration cap per solve")
    ap.add_argument("--c4-mode", default="min_time", choices=["min_time", "value"],
                    help="c4: minimum-time queries, or value solves at t ~ U[0.5, t_max]")
    ap.add_argument("--c-tau", type=float, default=None,
                    help="primal step ratio c_tau (default: the workload's)")
    ap.add_argument("--check-every", type=int, default=None,
                    help="iterations between certificates (default: the library's)")
    ap.add_argument("--tail-max", type=int, default=None,
                    help="points per system at which the per-point tail solver takes over (0: never)")
    ap.add_argument("--wide-min", type=int, default=None,
                    help="active points from which the 64-point LDS-staged kernel runs the iterations (0: never)")
    ap.add_argument("--deep-max", type=int, default=None,
                    help="active points up to which 16-point tiles run on 8 waves (-1: 16 per compute unit, 0: never)")
    ap.add_argument("--prec", default=None, choices=["fp32", "bf16x3"],
                    help="iteration precision (default: the workload's, fp32)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-literal", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the queries are independent, "
              "so a multi-GPU run is the single-GPU run on a shard of the points.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "tychastic":
        return bench_tychastic(args)
    if args.workload == "grid":
        return bench_grid(args)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "tune":
        return bench_tune(args)
    return bench_c5(args)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_c5(args):
    """The metric's workload: min-time queries on n=100, m=10, N=300 with
    the drift-planted start points, inputs resident in device memory.  Times
    the declared warm-start form (value) for K steps after W warmup steps,
    then the plain form (cold start at every probe) and the literal start
    points within wall budgets, then the oracle on a stratified sample.
    --workload c2 / c1 run the same legs on C2 (n=50, m=5, N=200, drift-
    planted and literal points) and C1 (the double integrator in FP64 on
    points uniform in [-2, 2]^2, --npts of them; no literal leg, and the
    oracle sample spread evenly over the batch)."""
    import numpy as np
    import torch
    from gen.configs import config1, config2, config5
    from gen.workloads import planted_drift_points
    from paper_1712_08226_amd import Solver
    from paper_1712_08226_amd.hopfpd import default_opts

    t_start = time.perf_counter()
    make, seed = {"c5": (config5, 5), "c2": (config2, 2), "c1": (config1, 1)}[args.workload]
    w = make(npts=args.npts)
    planted = args.workload != "c1"
    if args.prec:
        w.opts["prec"] = args.prec
    if args.c_tau is not None:
        w.opts["c_tau"] = args.c_tau
    ce_run = args.check_every if args.check_every is not None else w.opts.get("check_every",
                                                                              default_opts().check_every)
    spec = w.systems[0]
    # the planted times of the batch's points (C1's points are not planted)
    T0 = planted_drift_points(spec, args.npts, 0.2, 3.0, seed)[1] if planted else None
    dev = torch.device("cuda:0")
    solver = Solver(0)
    solver.set_systems([spec])
    npts = w.x.shape[0]
    stream = torch.cuda.current_stream(dev)

    def buffers(xh):
        k = xh.shape[0]
        return dict(x=torch.tensor(xh, dtype=torch.float64, device=dev),
                    T=torch.empty(k, dtype=torch.float64, device=dev),
                    gap=torch.empty(k, dtype=torch.float64, device=dev),
                    status=torch.empty(k, dtype=torch.int32, device=dev),
                    probes=torch.empty(k, dtype=torch.int32, device=dev),
                    iters=torch.empty(k, dtype=torch.int32, device=dev))

    main_buf = buffers(w.x)

    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    warm, _, root = args.warm.partition("+")
    root = root or "bisect"
    train_info = None
    if warm.startswith("mlp"):
        # learned warm start: trained on separate drift-planted queries (not timed)
        wt = make(npts=args.train_npts, seed=seed + 100)
        solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], warm="cont", check_every=ce_run)
        t0 = time.perf_counter()
        tr = solver.warm_train(wt.x, epochs=args.epochs, batch=4096, lr=1e-3, seed=7)
        train_info = {"train_queries": args.train_npts, "pairs": tr["pairs"], "epochs": args.epochs,
                      "loss_first_last": [round(float(tr["epoch_loss"][0]), 5), round(float(tr["epoch_loss"][-1]), 5)],
                      "seconds": round(time.perf_counter() - t0, 2)}
        log(f"warm-start network trained: {train_info}")

    def run_leg(name, wmode, buf, nwarm, max_steps, budget_s=None):
        """nwarm untimed steps, then timed steps: max_steps of them, or (with
        a budget) as many as fit in budget_s, at least one."""
        extra = {} if args.tail_max is None else {"tail_max": args.tail_max}
        if args.wide_min is not None:
            extra["wide_min"] = args.wide_min
        if args.deep_max is not None:
            extra["deep_max"] = args.deep_max
        solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], warm=wmode, root=root, check_every=ce_run,
                        **extra)

        def step():
            solver.min_time_dev(buf["x"], buf["T"], buf["gap"], buf["status"], probes=buf["probes"],
                                iters=buf["iters"], stream=stream)

        for i in range(nwarm):
            step()
            log(f"[{name}] warmup step {i + 1}/{nwarm} done")
        torch.cuda.synchronize()
        acc = dict(tk=0.0, launches=0, rows=0.0, ttail=0.0, tpts=0, dev_s=0.0, tw=0.0, nw=0, rw=0.0)
        done = 0
        t0 = time.perf_counter()
        while done < max_steps:
            step()
            tm = solver.last_timing()
            acc["tk"] += tm["iter_kernel_s"]
            acc["launches"] += tm["iter_launches"]
            acc["rows"] += tm["point_rows"]
            acc["ttail"] += tm["tail_kernel_s"]
            acc["tpts"] += tm["tail_points"]
            acc["dev_s"] += tm["total_s"]
            acc["tw"] += tm["wide_kernel_s"]
            acc["nw"] += tm["wide_launches"]
            acc["rw"] += tm["wide_point_rows"]
            done += 1
            log(f"[{name}] step {done}: device {tm['total_s']:.3f} s")
            if budget_s is not None and time.perf_counter() - t0 >= budget_s:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        k = buf["x"].shape[0]
        st = buf["status"].cpu().numpy()
        return dict(qps=k * done / dt, ms=1e3 * dt / done, steps=done, status=st, T=buf["T"].cpu().numpy(),
                    gap=buf["gap"].cpu().numpy(), iters=buf["iters"].cpu().numpy(),
                    probes=buf["probes"].cpu().numpy(), **acc)

    def summary(r):
        st, it = r["status"], r["iters"]
        ok = st == 0
        return {"queries_per_s": round(r["qps"], 2), "ms_per_step": round(r["ms"], 1), "steps_timed": r["steps"],
                "statuses_ok_inside_unreach_noconv_nonfinite": np.bincount(st, minlength=5).tolist(),
                "mean_iters": round(float(it.mean()), 1),
                "iters_p50_p90_p99_max": [float(v) for v in np.percentile(it, [50, 90, 99, 100])],
                "mean_probes": round(float(r["probes"].mean()), 3),
                "max_gap_reached": float(r["gap"][ok].max()) if ok.any() else None,
                "iter_kernel_s_per_step": round(r["tk"] / r["steps"], 3),
                "iter_launches_per_step": int(r["launches"] // r["steps"]),
                "tail_kernel_s_per_step": round(r["ttail"] / r["steps"], 3),
                "tail_points_per_step": int(r["tpts"] // r["steps"])}

    R = run_leg(args.warm, warm, main_buf, args.warmup, args.steps)
    head = summary(R)
    ok = R["status"] == 0
    head["T_le_T0_frac"] = (round(float(np.mean(R["T"][ok] <= T0[ok] * (1 + 1e-4))), 6)
                            if ok.any() and planted else None)

    plain = None
    if not args.no_plain and warm != "cold":
        P = run_leg("plain", "cold", main_buf, 0, args.steps, args.plain_budget)
        plain = summary(P)
        okb = (P["status"] == 0) & (R["status"] == 0)
        plain["same_results_as_value"] = bool(np.array_equal(P["status"], R["status"]) and np.all(
            np.abs(P["T"][okb] - R["T"][okb]) <= 1e-4 * R["T"][okb]))
        plain["value_over_plain"] = round(R["qps"] / P["qps"], 3)
    literal = None
    if not args.no_literal and planted:
        wl = make(npts=args.npts, literal=True)
        lb = buffers(wl.x)
        L = run_leg("literal", warm, lb, 0, args.steps, args.literal_budget)
        literal = summary(L)
        literal["points"] = wl.meta["points"]
        del lb

    # algorithmic flops: K lam and K^T y per point-row, 4 m n
    fpr = 4.0 * spec.m * spec.n
    bf = w.opts["prec"] == "bf16x3"
    peak = PEAK_BF16_MFMA_TFLOPS if bf else PEAK_FP64_TFLOPS if w.opts["prec"] == "fp64" else PEAK_FP32_MFMA_TFLOPS
    kern = {"k_pdhg_wide": (R["tw"], R["nw"], R["rw"]),
            "k_pdhg": (R["tk"] - R["tw"], R["launches"] - R["nw"], R["rows"] - R["rw"])}
    if bf:
        kern = {"k_pdhg_stream": (R["tk"], R["launches"], R["rows"])}
    dom = max(kern, key=lambda k: kern[k][0])
    tk, launches, rows = kern[dom]
    flops = fpr * rows
    achieved = flops / tk / 1e12 if tk > 0 else 0.0
    ct = None if bf else counter_traffic(args.warm, ce_run, w.opts["c_tau"], dom)
    traffic = None if ct is None else ct["hbm_bytes_per_launch"]
    desc = {"k_pdhg_wide": "k_pdhg_wide (fused FP32 PDHG iterations, 64 points per workgroup)",
            "k_pdhg": f"k_pdhg (fused {w.opts['prec'].upper()} PDHG iterations, 16-point tiles)",
            "k_pdhg_stream": "k_pdhg_stream<bf16 hi+lo> (3 bf16 MFMAs per product; achieved counts algorithmic flops)"}
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE counters, copy-calibrated)",
                "alg_flops_per_launch": round(flops / max(1, launches), 1),
                "kernel": desc[dom], "avg_launch_ms": round(1e3 * tk / max(1, launches), 4), "launches": launches,
                "iteration_kernels": {k: {"s_per_step": round(v[0] / R["steps"], 4),
                                          "launches_per_step": int(v[1] // R["steps"]),
                                          "avg_launch_ms": round(1e3 * v[0] / max(1, v[1]), 4),
                                          "tflops": round(fpr * v[2] / v[0] / 1e12, 3) if v[0] > 0 else None}
                                      for k, v in kern.items()}}
    metric = METRIC if args.workload == "c5" else \
        f"min-time queries/sec at dual gap≤1e-6 (n={spec.n},N={spec.N}): plain vs warm-start"
    out = {"metric": metric, "value": round(R["qps"], 2), "unit": "queries/s", "n_gpus": 1, "steps": R["steps"],
           "warmup": args.warmup, "ms_per_step": round(R["ms"], 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": w.opts["prec"], "data": "synthetic",
           "config": {"workload": f"min-time T(x), n={spec.n} m={spec.m} N={spec.N}, {spec.uset} control, "
                                  f"ellipsoid target, t_max={spec.t_max}, {spec.quad}, {npts} "
                                  f"{w.meta.get('points') or 'uniform in [-2,2]^2'} points "
                                  f"(value: warm start '{args.warm}'; plain: cold start at every probe)",
                      "npts": npts, "warm": args.warm, "scan": default_opts().scan,
                      "wide_min": args.wide_min if args.wide_min is not None else default_opts().wide_min,
                      "deep_max": args.deep_max if args.deep_max is not None else default_opts().deep_max,
                      "tail_max": args.tail_max if args.tail_max is not None else default_opts().tail_max,
                      "check_every": ce_run, "c_tau": w.opts["c_tau"], "gap_tol": 1e-6, "certificate": "fp64"},
           "results": head, "plain": plain, "literal": literal, "warm_start_training": train_info,
           "roofline": roofline}
    if not args.no_cpu:
        workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
        idx = (stratified_sample(T0, args.cpu_sample) if planted
               else np.unique(np.linspace(0, npts - 1, min(args.cpu_sample, npts)).astype(int)))
        copts = dict(c_tau=w.opts["c_tau"], warm=warm if warm in ("cold", "cont") else "cont", root=root)
        log(f"[cpu] oracle on {len(idx)} stratified queries, {workers} workers")
        rate, wall, per, cst = cpu_baseline(spec, w.x[idx], copts, workers)
        out["cpu_baseline"] = {"value": round(rate, 4), "unit": "queries/s", "cores": workers, "kind": "oracle",
                               "sample": f"{len(idx)} of the batch's queries spread evenly over "
                                         f"{'the planted times T0' if planted else 'the batch'}, each run to "
                                         f"completion on {workers} single-thread processes "
                                         f"({wall:.1f} s wall; per query mean {per.mean():.2f} s, max "
                                         f"{per.max():.2f} s)",
                               "options": copts, "statuses": cst, **host_info()}
    out["wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


def _oracle_value(args):
    """One oracle value solve (worker process): certified [phi_lo, phi_hi]."""
    spec, x, t, c_tau = args
    from oracle import hopf_oracle as O
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    pr = O.solve_value(S, x, t, O.Options(c_tau=c_tau))
    return pr.phi_lo, pr.phi_hi


def oracle_value_rate(spec, xs, t, c_tau, budget_s, workers):
    """The oracle's value solves phi(x_i, t), in order, one per single-thread
    worker process, for a wall-clock budget; returns (solves/s, seconds,
    finished)."""
    import multiprocessing as mp
    single_thread_workers()
    ctx = mp.get_context("spawn")
    pool = ctx.Pool(workers)
    done = 0
    t0 = time.perf_counter()
    try:
        it = pool.imap(_oracle_value, [(spec, x, float(t), c_tau) for x in xs], chunksize=1)
        while True:
            left = budget_s - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                it.next(timeout=left)
                done += 1
            except (mp.TimeoutError, StopIteration):
                break
    finally:
        el = time.perf_counter() - t0
        pool.terminate()
        pool.join()
    return done / el, el, done


def paper_scaling_ms(d):
    """The paper's least-squares fit of its per-solve time (ms) against the
    dimension d in the scaling experiment of Sec. VI-C (MATLAB, FP64, one
    laptop CPU, residual stop 1e-4): context, not a target."""
    return 2.382e-4 * d * d + 0.0414 * d + 2.598


def bench_tychastic(args):
    """The dimensional-scaling experiment of Sec. VI-C: value solves of the
    k-copy double integrator (d = 2k, m = 1, N = 100 left-rule nodes, t = 2)
    for every d of --dims, each over --npts points resident on the device,
    after the unscented five-sigma-point system of Sec. VI-B (d = 10, the
    first sweep entry).  `value` is the rate at the largest d with inputs
    and outputs resident on the device (hopf_value_dev); the oracle's rate
    on the host cores and the paper's times are reported beside it."""
    import numpy as np
    import torch
    from gen.configs import config_tychastic, config_unscented
    from paper_1712_08226_amd import Solver
    dims = [int(v) for v in args.dims.split(",")]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    solver = Solver(0)
    sweep = []
    cases = [(10, "unscented", lambda: config_unscented(npts=args.npts))]
    cases += [(d, "sampled", lambda d=d: config_tychastic(d, npts=args.npts)) for d in dims]
    for d, kind, make in cases:
        w = make()
        if args.c_tau is not None:
            w.opts["c_tau"] = args.c_tau
        spec, T, npts = w.systems[0], w.opts["t"], len(w.x)
        solver.set_systems([spec])
        # inputs and outputs resident on the device; the timed region is the call
        xd = torch.tensor(w.x, dtype=torch.float64, device=dev)
        td = torch.full((npts,), T, dtype=torch.float64, device=dev)
        lo, hi = torch.empty_like(td), torch.empty_like(td)
        itd = torch.empty(npts, dtype=torch.int32, device=dev)
        std = torch.empty(npts, dtype=torch.int32, device=dev)
        nw = min(npts, 4096)
        legs = {}
        # structure 1: the reduced system of the copies' mean (the default);
        # structure 0: the full d-dimensional system, as the paper solves it
        for structure in (1, 0):
            solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], structure=structure)
            for i in range(args.warmup):
                solver.value_dev(xd[:nw], td[:nw], lo[:nw], hi[:nw], std[:nw], iters=itd[:nw], stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.value_dev(xd, td, lo, hi, std, iters=itd, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tm = solver.last_timing()
            r = {"phi_lo": lo.cpu().numpy(), "phi_hi": hi.cpu().numpy(), "iters": itd.cpu().numpy(),
                 "status": std.cpu().numpy()}
            legs[structure] = (dt, tm, r)
            log(f"[{kind} d={d} structure={structure}] {npts} value solves: {dt:.3f} s")
        dt, tm, r = legs[1]
        df, tmf, rf = legs[0]
        gap = (r["phi_hi"] - r["phi_lo"]) / np.maximum(1.0, np.abs(r["phi_hi"]))
        achf = tmf["alg_flops"] / tmf["iter_kernel_s"] / 1e12 if tmf["iter_kernel_s"] > 0 else 0.0
        # the paper's fit for the sampled copies; 4.0 ms per point reported for the unscented system
        pms = paper_scaling_ms(d) if kind == "sampled" else 4.0
        agree = bool(np.all(np.maximum(r["phi_lo"], rf["phi_lo"]) <= np.minimum(r["phi_hi"], rf["phi_hi"]) +
                            1e-9 * np.maximum(1.0, np.abs(rf["phi_hi"]))))
        row = {"system": kind, "d": d, "points": npts, "device_s": round(dt, 4),
               "solves_per_s": round(npts / dt, 1),
               "solves_per_s_solver_events": round(npts / tm["total_s"], 1),
               "mean_iters": round(float(r["iters"].mean()), 1), "max_iters": int(r["iters"].max()),
               "statuses": np.bincount(r["status"], minlength=5).tolist(), "max_gap": float(gap.max()),
               "reached_frac": round(float(np.mean(r["phi_hi"] <= 0.0)), 4),
               "full_system": {"solves_per_s": round(npts / df, 1), "mean_iters": round(float(rf["iters"].mean()), 1),
                               "statuses": np.bincount(rf["status"], minlength=5).tolist(),
                               "k_pdhg_tflops": round(achf, 3),
                               "k_pdhg_frac_fp32_mfma": round(achf / PEAK_FP32_MFMA_TFLOPS, 4),
                               "intervals_overlap_reduced": agree},
               "paper_ms_per_solve": round(pms, 3), "paper_solves_per_s": round(1e3 / pms, 1)}
        sweep.append(row)

    # the unscented problem as Sec. VI-B poses it: minimum time to the
    # weighted target, reduced system (structure 1) and full system
    w = config_unscented(npts=args.npts)
    solver.set_systems(w.systems)
    xd = torch.tensor(w.x, dtype=torch.float64, device=dev)
    npts = len(w.x)
    Td, gd = (torch.empty(npts, dtype=torch.float64, device=dev) for _ in range(2))
    std, prd = (torch.empty(npts, dtype=torch.int32, device=dev) for _ in range(2))
    mt = {}
    for structure in (1, 0):
        solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], structure=structure, warm="cont")
        nw = min(npts, 4096)
        solver.min_time_dev(xd[:nw], Td[:nw], gd[:nw], std[:nw], probes=prd[:nw], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.min_time_dev(xd, Td, gd, std, probes=prd, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mt[structure] = (dt, Td.cpu().numpy(), std.cpu().numpy(), prd.cpu().numpy())
        log(f"[unscented min time structure={structure}] {npts} queries: {dt:.3f} s")
    (dt, T1, s1, p1), (dtf, T0, s0, _) = mt[1], mt[0]
    ok = (s1 == 0) & (s0 == 0)
    n_status = int(np.sum(s1 != s0))
    n_T = int(np.sum(np.abs(T1[ok] - T0[ok]) > 1e-4 * T0[ok] + 1e-6 * w.systems[0].t_max))
    unscented_mt = {"points": npts, "queries_per_s": round(npts / dt, 1), "device_s": round(dt, 4),
                    "statuses": np.bincount(s1, minlength=5).tolist(), "mean_probes": round(float(p1.mean()), 2),
                    "T_p50": round(float(np.median(T1[s1 == 0])), 4) if (s1 == 0).any() else None,
                    "full_system": {"queries_per_s": round(npts / dtf, 1), "device_s": round(dtf, 4),
                                    "points_with_other_status": n_status, "points_with_other_T": n_T},
                    "paper_ms_per_point": 4.0, "paper_points_per_s": 250.0}

    top = sweep[-1]
    cpu = None
    if not args.no_cpu:
        # the oracle on the host cores, value solves of the largest d, bounded
        w = config_tychastic(dims[-1], npts=256)
        workers = min(16, os.cpu_count() or 1)
        rate, el, done = oracle_value_rate(w.systems[0], w.x, w.opts["t"], w.opts["c_tau"], args.cpu_budget, workers)
        cpu = {"value": round(rate, 3), "unit": "solves/s", "cores": workers, "kind": "oracle",
               "sample": f"d={dims[-1]} value solves in order on {workers} single-thread processes for "
                         f"{args.cpu_budget:.0f} s wall; {done} finished"}
        print(f"[tychastic] oracle: {done} solves in {el:.1f} s", file=sys.stderr, flush=True)
    res = {"metric": f"value solves/sec at dual gap<=1e-6, sampled-copy double integrator (d={top['d']}, m=1, N=100; "
                     "value: the reduced system of the copies' mean, sweep[].full_system: the full system)",
           "value": top["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
           "ms_per_step": round(1e3 * top["device_s"], 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"value phi(x, t=2) of k = d/2 double integrators sharing one control in [-1,1], "
                                  f"starts ~ N((1,0), 0.0667^2 I), mean-squared target 0.04, left rule N=100, "
                                  f"{top['points']} points per d", "dims": dims,
                      "c_tau": args.c_tau if args.c_tau is not None else config_tychastic(dims[-1], npts=1).opts["c_tau"],
                      "certificate": "fp64"},
           "sweep": sweep,
           "unscented_min_time": unscented_mt,
           "paper_context": "Sec. VI-C fit of MATLAB time per value solve on a laptop CPU (FP64, residual stop "
                            "1e-4): paper_ms_per_solve; for the unscented row the Sec. VI-B average of 4.0 ms per "
                            "point (HJ solutions along trajectories); other hardware and a looser stop, not a target",
           "roofline": {"bound": "mfma", "achieved": top["full_system"]["k_pdhg_tflops"], "peak": PEAK_FP32_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": top["full_system"]["k_pdhg_frac_fp32_mfma"], "traffic": None,
                        "kernel": "k_pdhg<float, NT, 1> on the full system (algorithmic flops 4*m*n per point-row)"},
           "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def bench_grid(args):
    """The level-set experiment of Sec. VI-A: value solves of the double
    integrator on a grid over [-1, 1]^2 at ten horizons t_j = j T*/10, each
    horizon in the paper's per-horizon layout (a table over [0, t_j]), FP64
    iterations.  Grids of 50 x 50 (the paper's) and 512 x 512 points, inputs
    resident on the device; table builds are timed apart."""
    import numpy as np
    import torch
    from dataclasses import replace
    from gen.configs import config_grid
    from paper_1712_08226_amd import Solver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    solver = Solver(0)
    w0 = config_grid(50)
    spec, opts = w0.systems[0], w0.opts
    solver.set_systems([spec])
    solver.set_opts(prec=opts["prec"], c_tau=opts["c_tau"])
    r0 = solver.min_time(np.array([[1.0, 0.0]]))
    Ts = float(r0["T"][0])
    times = [Ts * j / 10 for j in range(1, 11)]
    print(f"[grid] T* from (1,0) = {Ts:.6f}", file=sys.stderr, flush=True)
    grids = []
    for per_axis in (50, 512):
        w = config_grid(per_axis)
        npts = len(w.x)
        xd = torch.tensor(w.x, dtype=torch.float64, device=dev)
        lo, hi = torch.empty(npts, dtype=torch.float64, device=dev), torch.empty(npts, dtype=torch.float64, device=dev)
        itd = torch.empty(npts, dtype=torch.int32, device=dev)
        std = torch.empty(npts, dtype=torch.int32, device=dev)
        solve_s, build_s, iters, stats, reached, maxgap = 0.0, 0.0, [], np.zeros(5, dtype=int), [], 0.0
        for k, t in enumerate(times):
            t0 = time.perf_counter()
            solver.set_systems([replace(spec, t_max=t)])
            build_s += time.perf_counter() - t0
            td = torch.full((npts,), t, dtype=torch.float64, device=dev)
            if k == 0:
                for i in range(args.warmup):
                    solver.value_dev(xd, td, lo, hi, std, iters=itd, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.value_dev(xd, td, lo, hi, std, iters=itd, stream=stream)
            torch.cuda.synchronize()
            solve_s += time.perf_counter() - t0
            st_h, lo_h, hi_h = std.cpu().numpy(), lo.cpu().numpy(), hi.cpu().numpy()
            stats += np.bincount(st_h, minlength=5)[:5]
            iters.append(float(itd.float().mean().item()))
            reached.append(round(float(np.mean(hi_h <= 0.0)), 4))
            maxgap = max(maxgap, float(np.max((hi_h - lo_h) / np.maximum(1.0, np.abs(hi_h)))))
        row = {"grid": f"{per_axis}x{per_axis}", "solves": npts * len(times), "solve_s": round(solve_s, 4),
               "solves_per_s": round(npts * len(times) / solve_s, 1), "table_builds_s": round(build_s, 3),
               "mean_iters_per_horizon": [round(v, 1) for v in iters], "statuses": stats.tolist(),
               "max_gap": maxgap, "reached_frac_per_horizon": reached}
        grids.append(row)
        print(f"[grid {per_axis}x{per_axis}] {row['solves']} value solves in {solve_s:.3f} s", file=sys.stderr,
              flush=True)
    cpu = None
    if not args.no_cpu:
        wc = config_grid(50)
        t = times[4]
        rate, el, done = oracle_value_rate(replace(spec, t_max=t), wc.x, t, opts["c_tau"], args.cpu_budget,
                                           min(16, os.cpu_count() or 1))
        cpu = {"value": round(rate, 2), "unit": "solves/s", "cores": min(16, os.cpu_count() or 1), "kind": "oracle",
               "sample": f"50x50 grid at t = T*/2 in order on single-thread processes for {args.cpu_budget:.0f} s "
                         f"wall; {done} finished"}
        print(f"[grid] oracle: {done} solves in {el:.1f} s", file=sys.stderr, flush=True)
    top = grids[-1]
    res = {"metric": "value solves/sec at dual gap<=1e-6, double-integrator level-set grid (Sec. VI-A)",
           "value": top["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
           "ms_per_step": round(1e3 * top["solve_s"], 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
           "config": {"workload": "value phi(x, t_j) of the double integrator, |u|<=1, disk r=0.2, on a grid over "
                                  "[-1,1]^2 at t_j = j T*/10 (j = 1..10, T* from (1,0)), per-horizon left rule "
                                  "N=100, FP64 iterations", "T_star": Ts, "c_tau": opts["c_tau"]},
           "grids": grids,
           "paper_context": "Sec. VI-A: 2.1 ms per grid point (476 solves/s) on a 50x50 grid, MATLAB on one laptop "
                            "CPU, residual stop 1e-4; other hardware and a looser stop, not a target",
           "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def bench_c3(args):
    """Precision workload (n=200, m=20, N=400, box): value solves phi(x, t) of
    16384 points in BF16 hi+lo (FP32 accumulate, FP32 escalation of stalled
    probes) and in FP32, both certified in FP64, inputs resident on the
    device; the BF16 / FP32 difference; the one-probe min-time queries; and
    (CPU leg) the FP64 oracle on an evenly spaced sample of the points at the
    full N = 400, timed, with each sampled point's error of the BF16 result
    against it: |dphi| of the interval midpoints, interval overlap, and
    ||dlam|| / ||lam||."""
    import numpy as np
    import torch
    from gen.configs import config3
    from paper_1712_08226_amd import Solver
    w = config3(npts=args.npts if args.npts != 65536 else 16384)
    if args.c_tau is not None:
        w.opts["c_tau"] = args.c_tau
    spec = w.systems[0]
    npts = len(w.x)
    t = np.asarray(w.meta["t"], dtype=np.float64)
    dev = torch.device("cuda:0")
    solver = Solver(0)
    t0 = time.perf_counter()
    solver.set_systems([spec])
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream(dev)
    xd = torch.tensor(w.x, dtype=torch.float64, device=dev)
    td = torch.tensor(t, dtype=torch.float64, device=dev)
    lo, hi = torch.empty_like(td), torch.empty_like(td)
    lam = torch.empty_like(xd)
    st = torch.empty(npts, dtype=torch.int32, device=dev)
    it = torch.empty(npts, dtype=torch.int32, device=dev)
    out = {}
    wmin = args.wide_min if args.wide_min is not None else w.opts.get("wide_min")
    extra = {} if wmin is None else {"wide_min": wmin}
    for prec in ("bf16x3", "fp32"):
        solver.set_opts(prec=prec, c_tau=w.opts["c_tau"], **extra)
        for i in range(args.warmup):
            solver.value(w.x[:256], t[:256])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.value_dev(xd, td, lo, hi, st, lam=lam, iters=it, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tm = solver.last_timing()
        out[prec] = dict(r=dict(phi_lo=lo.cpu().numpy(), phi_hi=hi.cpu().numpy(), lam=lam.cpu().numpy(),
                                status=st.cpu().numpy(), iters=it.cpu().numpy()), dt=dt, tm=tm)
        log(f"[c3 {prec}] {npts} value solves in {dt:.2f} s")
    solver.set_opts(prec="bf16x3", c_tau=w.opts["c_tau"])
    nmt = min(npts, 2048)
    t0 = time.perf_counter()
    rm = solver.min_time(w.x[:nmt])
    dtm = time.perf_counter() - t0
    log(f"[c3] {nmt} min-time queries in {dtm:.2f} s")
    b, f = out["bf16x3"]["r"], out["fp32"]["r"]
    mid_b = 0.5 * (b["phi_lo"] + b["phi_hi"])
    mid_f = 0.5 * (f["phi_lo"] + f["phi_hi"])
    tmb = out["bf16x3"]["tm"]

    def kern(tm):
        nw = tm["wide_launches"]
        ks = {"k_pdhg_swide": (tm["wide_kernel_s"], nw, tm["wide_point_rows"]),
              "k_pdhg_stream": (tm["iter_kernel_s"] - tm["wide_kernel_s"], tm["iter_launches"] - nw,
                                tm["point_rows"] - tm["wide_point_rows"])}
        fpr = 4.0 * spec.m * spec.n
        return {k: {"s": round(v[0], 4), "launches": int(v[1]),
                    "tflops": round(fpr * v[2] / v[0] / 1e12, 3) if v[0] > 0 else None} for k, v in ks.items()}
    kb = kern(tmb)
    dom = max(kb, key=lambda k: kb[k]["s"])
    ach = kb[dom]["tflops"] or 0.0
    res = {"metric": "value solves/sec at dual gap<=1e-6, BF16 hi+lo (n=200, m=20, N=400, box)",
           "value": round(npts / out["bf16x3"]["dt"], 2), "unit": "solves/s", "n_gpus": 1, "steps": 1,
           "warmup": args.warmup, "ms_per_step": round(1e3 * out["bf16x3"]["dt"], 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
           "config": {"workload": f"value phi(x,t), n=200 m=20 N=400 box control, {npts} points x~N(0,4I), "
                                  "t~U[0.5,10], K as bf16 hi+lo with fp32 accumulation, fp64 tables and certificate",
                      "c_tau": w.opts["c_tau"], "check_every": w.opts.get("check_every"),
                      "wide_min": wmin if wmin is not None else default_opts().wide_min},
           "fp32_solves_per_s": round(npts / out["fp32"]["dt"], 2),
           "bf16_over_fp32": round(out["fp32"]["dt"] / out["bf16x3"]["dt"], 3),
           "statuses_bf16": np.bincount(b["status"], minlength=5).tolist(),
           "statuses_fp32": np.bincount(f["status"], minlength=5).tolist(),
           "mean_iters_bf16_fp32": [float(b["iters"].mean()), float(f["iters"].mean())],
           "max_gap_bf16": float(np.max((b["phi_hi"] - b["phi_lo"]) / np.maximum(1, np.abs(b["phi_hi"])))),
           "error": {"max_abs_phi_bf16_vs_fp32_all": float(np.max(np.abs(mid_b - mid_f)))},
           "iteration_kernels": {"bf16x3": kb, "fp32": kern(out["fp32"]["tm"])},
           "min_time": {"queries": nmt, "queries_per_s": round(nmt / dtm, 2),
                        "statuses": np.bincount(rm["status"], minlength=5).tolist()},
           "setup_s": round(setup_s, 2),
           "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_BF16_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / PEAK_BF16_MFMA_TFLOPS, 4), "traffic": None,
                        "kernel": f"{dom}<bf16 hi+lo> (3 bf16 MFMAs per product; achieved counts algorithmic flops)"}}
    if not args.no_cpu and args.c3_sample > 0:
        import multiprocessing as mp
        idx = np.linspace(0, npts - 1, min(args.c3_sample, npts)).astype(int)
        workers = max(1, min(args.cpu_workers, os.cpu_count() or 1, len(idx)))
        single_thread_workers()
        opts = dict(c_tau=w.opts["c_tau"], max_iter=2_000_000)
        log(f"[c3 cpu] oracle on {len(idx)} points at N={spec.N}, {workers} workers")
        t0 = time.perf_counter()
        orc = [None] * len(idx)
        with mp.get_context("spawn").Pool(workers) as pool:
            jobs = [(k, spec, w.x[i], float(t[i]), opts) for k, i in enumerate(idx)]
            for done, r in enumerate(pool.imap_unordered(_oracle_value_full, jobs, chunksize=1)):
                orc[r[0]] = r[1:]
                log(f"[c3 cpu] oracle point {done + 1}/{len(idx)} (sample {r[0]}): {r[4]} iterations, {r[5]:.1f} s")
        wall = time.perf_counter() - t0
        per = []
        for k, i in enumerate(idx):
            olo, ohi, olam, oit, osec = orc[k]
            mo = 0.5 * (olo + ohi)
            dl = float(np.linalg.norm(b["lam"][i] - olam) / max(np.linalg.norm(olam), 1e-300))
            per.append({"idx": int(i), "t": round(float(t[i]), 4), "phi_oracle": mo,
                        "abs_dphi": abs(float(mid_b[i]) - mo),
                        "rel_dphi": abs(float(mid_b[i]) - mo) / max(1.0, abs(mo)),
                        "intervals_overlap": bool(max(b["phi_lo"][i], olo) <= min(b["phi_hi"][i], ohi) +
                                                  1e-9 * max(1.0, abs(mo))),
                        "rel_dlam": dl, "oracle_iters": int(oit), "oracle_s": round(osec, 2)})
        res["error"]["bf16_vs_fp64_oracle_sample"] = per
        res["error"]["max_rel_dphi_sample"] = max(e["rel_dphi"] for e in per)
        res["error"]["max_rel_dlam_sample"] = max(e["rel_dlam"] for e in per)
        res["cpu_baseline"] = {"value": round(len(idx) / wall, 4), "unit": "solves/s", "cores": workers,
                               "kind": "oracle", "sample": f"{len(idx)} evenly spaced points of the batch, "
                                                           f"value solves at N={spec.N} run to completion",
                               "host": host_info()}
    print(json.dumps(res), flush=True)


def bench_tune(args):
    """The launch-parameter tuner (paper_1712_08226_amd.tune) on the headline
    system: the drift-planted queries (--npts of them), continuation start,
    the workload's step ratio; prints the table and the chosen setting."""
    from gen.configs import config5
    from paper_1712_08226_amd import Solver
    from paper_1712_08226_amd.tune import tune
    w = config5(npts=args.npts)
    solver = Solver(0)
    solver.set_systems(w.systems)
    base = dict(prec=w.opts["prec"], c_tau=w.opts["c_tau"], warm="cont", check_every=w.opts["check_every"])
    solver.set_opts(**base)
    solver.min_time(w.x[:1024])                      # first-call costs out of the table
    res = tune(solver, w.x, mode="min_time", base=base, log=log)
    print(json.dumps({"workload": f"min-time n=100 m=10 N=300, {len(w.x)} drift-planted queries, warm cont",
                      **res}), flush=True)


def bench_c4(args):
    """64 uneven systems in one call (every system's points mixed in random
    order; each system's points run as a job with its own kernels, the jobs
    on a pool of streams).  Value solves phi(x, t), t ~ U[0.5, t_max], with
    an iteration cap per solve; point counts scaled by --c4-scale."""
    import numpy as np
    from gen.configs import config4
    from paper_1712_08226_amd import Solver
    w = config4(scale=args.c4_scale)
    npts = len(w.x)
    t = np.random.default_rng(44).uniform(0.5, 10.0, npts)
    solver = Solver(0)
    t0 = time.perf_counter()
    solver.set_systems(w.systems)
    setup_s = time.perf_counter() - t0
    print(f"[c4] {len(w.systems)} systems set up in {setup_s:.1f} s; {npts} {args.c4_mode} queries",
          file=sys.stderr, flush=True)
    solver.set_opts(prec=w.opts["prec"], c_tau=w.opts["c_tau"], max_iter=args.c4_max_iter, warm="cont")
    times = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        if args.c4_mode == "value":
            r = solver.value(w.x, t, sys_id=w.sys_id)
        else:
            r = solver.min_time(w.x, sys_id=w.sys_id)
        times.append(time.perf_counter() - t0)
        print(f"[c4] step {i + 1}/{args.steps}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    tm = solver.last_timing()
    dt = float(np.mean(times))
    st = r["status"]
    ach = tm["alg_flops"] / tm["total_s"] / 1e12 if tm["total_s"] > 0 else 0.0
    per_sys = []
    for k, s in enumerate(w.systems):
        sel = w.sys_id == k
        per_sys.append([int(s.A.shape[0]), int(s.B.shape[1]), int(s.N), s.uset, int(sel.sum()),
                        int((st[sel] == 0).sum()), float(r["iters"][sel].mean())])
    mt = args.c4_mode == "min_time"
    res = {"metric": ("min-time queries/sec at dual gap<=1e-6" if mt else "certified value solves/sec (gap<=1e-6)")
                     + ", 64 uneven systems in one call",
           "value": round(npts / dt, 2), "unit": "queries/s" if mt else "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 0, "ms_per_step": round(1e3 * dt, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": ("min-time T(x), continuation warm start" if mt else "value phi(x,t), t~U[0.5,10]")
                                  + f", 64 systems n log-uniform [4,256] (drawn "
                                  f"{min(s.A.shape[0] for s in w.systems)}-{max(s.A.shape[0] for s in w.systems)}), "
                                  f"m=max(1,n/4), N in 100..500, l2/box 32/32, {npts} drift-planted points "
                                  f"({args.c4_scale:g} x 256-4096 per system), step ratio 5 (l2) / 0.3 (box), "
                                  f"at most {args.c4_max_iter} iterations per solve (probe)"},
           "results": {"ok": int((st == 0).sum()), "unreachable": int((st == 2).sum()), "inside": int((st == 1).sum()),
                       "noconv": int((st == 3).sum()), "nonfinite": int((st == 4).sum()),
                       "mean_iters": float(r["iters"].mean()), "max_iters": int(r["iters"].max())},
           "timing": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in tm.items()},
           "setup_s": round(setup_s, 2),
           "per_system_n_m_N_uset_points_ok_meaniters": per_sys,
           "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(ach / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                        "basis": "algorithmic flops of all systems / device time of the whole call"}}
    print(json.dumps(res), flush=True)

if __name__ == "__main__":
    main()
