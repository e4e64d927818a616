"""Launch-parameter tuner for one system class.

For a system and a sample of its queries, every candidate setting of the
launch parameters (certificate interval, the active-point thresholds of the
64-point and 8-wave kernels, the tail-solver threshold) is run through the
library on the device and timed with the library's own event timing; a
candidate is eligible only if it returns the reference setting's results
(the same statuses, T within the search tolerance, every gap within the
tolerance).  The fastest eligible candidate is returned with the whole
table.  The step ratio c_tau is not tuned here: it changes the iteration
path, not the launch."""
from __future__ import annotations

import itertools

import numpy as np

DEFAULT_GRID = {"check_every": (50, 75, 100), "wide_min": (16384, 32768), "tail_max": (512, 2048)}


def _same(ref, r, mode, rel=1e-4):
    if not np.array_equal(ref["status"], r["status"]):
        return False
    ok = ref["status"] == 0
    if mode == "min_time":
        return bool(np.all(np.abs(ref["T"][ok] - r["T"][ok]) <= rel * ref["T"][ok]) and np.all(r["gap"][ok] <= 1e-6))
    lo = np.maximum(ref["phi_lo"], r["phi_lo"])
    hi = np.minimum(ref["phi_hi"], r["phi_hi"])
    return bool(np.all(lo[ok] <= hi[ok] + 1e-9 * np.maximum(1.0, np.abs(hi[ok]))))


def tune(solver, x, mode="min_time", t=None, base=None, grid=None, reps=1, log=None):
    """solver: a Solver with the system set (one system); x: (npts, n)
    sample queries; t: horizons for mode "value"; base: the options every
    candidate starts from (prec, c_tau, warm, ...); grid: {option: values}.
    Returns {"best": {...}, "table": [...], "reference": {...}}."""
    base = dict(base or {})
    grid = dict(grid or DEFAULT_GRID)
    keys = list(grid)

    def run(opts):
        solver.set_opts(**opts)
        best = None
        for _ in range(max(1, reps)):
            r = solver.min_time(x) if mode == "min_time" else solver.value(x, t)
            s = solver.last_timing()["total_s"]
            best = s if best is None else min(best, s)
        return r, best

    ref_opts = dict(base)
    ref, ref_s = run(ref_opts)
    table = []
    for vals in itertools.product(*(grid[k] for k in keys)):
        opts = dict(base, **dict(zip(keys, vals)))
        r, sec = run(opts)
        same = _same(ref, r, mode)
        row = dict(zip(keys, vals), device_s=round(sec, 4), queries_per_s=round(len(x) / sec, 1), same_results=same)
        table.append(row)
        if log:
            log(f"[tune] {row}")
    ok = [row for row in table if row["same_results"]]
    best = min(ok, key=lambda r: r["device_s"]) if ok else None
    return {"best": best, "table": table,
            "reference": dict({k: base.get(k) for k in keys}, device_s=round(ref_s, 4))}
