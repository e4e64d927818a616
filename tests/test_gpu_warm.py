"""Learned warm start on the GPU: the network's gradients against the FP64
oracle, training reduces the loss, the trained network's lam_0 needs fewer
iterations than the plain start lam_0 = 0, and warm-started minimum times are
the certified results of the plain method (the network only changes where
the iterations start)."""
import sys

import numpy as np
import pytest

from gen import random_system, gaussian_points
from gen.workloads import planted_drift_points
from oracle import hopf_oracle as O
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_1712_08226_amd import Solver
    s = Solver(0)
    yield s
    s.close()


def test_mlp_gradient_matches_oracle(solver):
    say("case: mlp gradient parity")
    spec = random_system(6, 2, 30, "l2", seed=3, t_max=3.0)
    solver.set_systems([spec])
    solver.warm_init(0, seed=7)
    theta, _ = solver.warm_get(0)
    n = 6
    rng = np.random.default_rng(0)
    B = 300
    Z = rng.normal(size=(B, n + 1)).astype(np.float32)
    Y = np.zeros((B, n + 2), dtype=np.float32)
    Y[:, :n] = rng.normal(size=(B, n))
    Y[:, n] = rng.normal(0, 0.5, B)
    Y[:, n + 1] = (rng.uniform(size=B) < 0.6)
    # the output layer is small at init; perturb it so every loss term is active
    th = theta.astype(np.float64)
    th[-(n + 2) * 257:] += rng.normal(0, 0.3, (n + 2) * 257)
    solver.warm_set(th.astype(np.float32), None, 0)
    loss_d, g_d = solver.warm_loss_grad(Z, Y, 0)
    loss_o, g_o = M.loss_and_grad(th.astype(np.float32).astype(np.float64), Z.astype(np.float64),
                                  Y.astype(np.float64), n, 256)
    assert abs(loss_d - loss_o) <= 1e-4 * max(1.0, abs(loss_o))
    scale = np.abs(g_o).max()
    assert np.max(np.abs(g_d - g_o)) <= 1e-3 * scale
    rel = np.linalg.norm(g_d - g_o) / np.linalg.norm(g_o)
    assert rel <= 1e-3


def test_training_and_warm_min_time(solver, tmp_path):
    """Train on solver-generated pairs, then solve held-out points with the
    warm start.  Every learned mode must return the plain search's results on
    every point (same status, |dT| <= 1e-4 T, gap <= 1e-6): the network only
    moves where the iterations start, or (mode "mlp") adds probe hints inside
    the first sign-change cell.  Sampled points also match the oracle.  The
    iteration counts of cold, continuation and the learned starts are
    reported; the network's lam_0 must beat the cold start."""
    say("case: warm start train + min_time")
    spec = random_system(20, 3, 60, "l2", seed=12, t_max=6.0)
    solver.set_systems([spec])
    solver.set_opts(prec="fp32", c_tau=2.0, warm="cont")
    xtr, _ = planted_drift_points(spec, 2048, 0.2, 3.0, seed=1)
    res = solver.warm_train(xtr, epochs=30, batch=1024, lr=1e-3, seed=3)
    say("pairs", res["pairs"], "loss first/last", res["epoch_loss"][0], res["epoch_loss"][-1])
    assert res["pairs"] > 2048
    assert res["epoch_loss"][-1] < 0.5 * res["epoch_loss"][0]
    xte, _ = planted_drift_points(spec, 512, 0.2, 3.0, seed=2)
    solver.set_opts(prec="fp32", c_tau=2.0, warm="cold")
    cold = solver.min_time(xte)
    solver.set_opts(prec="fp32", c_tau=2.0, warm="cont")
    base = solver.min_time(xte)
    assert np.array_equal(cold["status"], base["status"])
    ok = base["status"] == 0
    assert np.all(np.abs(cold["T"][ok] - base["T"][ok]) <= 1e-4 * base["T"][ok])
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset="l2", N=60, t_max=6.0)
    for k in np.flatnonzero(ok)[:3]:
        o = O.min_time(S, xte[k], O.Options(c_tau=2.0))
        assert o.status == O.PT_OK and abs(base["T"][k] - o.T) <= 1e-4 * o.T
    iters = {"cold": cold["iters"].mean(), "cont": base["iters"].mean()}
    for mode in ("mlp", "mlp_lam", "mlp_first"):
        solver.set_opts(prec="fp32", c_tau=2.0, warm=mode)
        warm = solver.min_time(xte)
        iters[mode] = warm["iters"].mean()
        say(mode, "iters", iters[mode], "probes cont", base["probes"].mean(), "warm", warm["probes"].mean())
        assert np.array_equal(base["status"], warm["status"]), mode
        assert np.all(warm["gap"][ok] <= 1e-6), mode
        assert np.all(np.abs(warm["T"][ok] - base["T"][ok]) <= 1e-4 * base["T"][ok]), mode
        assert np.all(np.isinf(warm["T"][base["status"] == 2])), mode
    say("mean iterations per query:", {k: round(float(v), 1) for k, v in iters.items()},
        "gain of the network's lam_0 over continuation:", round(float(iters["cont"] / iters["mlp_lam"]), 3),
        "of the network's first-probe start:", round(float(iters["cont"] / iters["mlp_first"]), 3))
    assert iters["mlp_lam"] < 0.9 * iters["cold"]
    # the first-probe start against continuation, the non-learned baseline:
    # measured and reported above; it must not cost more than a tenth
    assert iters["mlp_first"] <= 1.1 * iters["cont"]
    # the trained network survives a save and a load into a fresh context
    from paper_1712_08226_amd import Solver
    path = str(tmp_path / "net.npz")
    solver.warm_save(path)
    s2 = Solver(0)
    try:
        s2.set_systems([spec])
        s2.warm_load(path)
        for a, b in zip(solver.warm_get(), s2.warm_get()):
            assert np.array_equal(a, b)
        solver.set_opts(prec="fp32", c_tau=2.0, warm="mlp_first")
        s2.set_opts(prec="fp32", c_tau=2.0, warm="mlp_first")
        r1, r2 = solver.min_time(xte[:64]), s2.min_time(xte[:64])
        assert np.array_equal(r1["status"], r2["status"])
        assert np.array_equal(r1["T"], r2["T"], equal_nan=True)
    finally:
        s2.close()
