"""The C-ABI's error paths and the parts of the boundary beyond the solves:
invalid targets are refused, an iteration cap shows up per point, a damaged
warm-start network changes no result, checkpoint files round-trip and bad
ones are refused, and a target matrix that is not diagonal gives the
oracle's results in the caller's coordinates."""
import math
import sys

import numpy as np
import pytest

from gen import random_system, gaussian_points
from gen.workloads import planted_drift_points
from oracle import hopf_oracle as O

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


def with_W(spec, W):
    return dict(A=spec.A, B=spec.B, W=W, c=spec.c, uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)


def test_invalid_targets_are_rejected(solver):
    from paper_1712_08226_amd.hopfpd import HopfError
    say("case: invalid targets")
    spec = random_system(6, 2, 30, "l2", seed=3, t_max=3.0)
    W = np.eye(6)
    W[0, 1] = W[1, 0] = 2.0                      # eigenvalues 3 and -1: indefinite
    with pytest.raises(HopfError, match="positive definite"):
        solver.set_systems([with_W(spec, W)])
    W = np.eye(6)
    W[0, 1] = 0.3                                # not symmetric
    with pytest.raises(HopfError, match="symmetric"):
        solver.set_systems([with_W(spec, W)])
    W = np.diag([1.0, 0.5, 0.0, 1.0, 1.0, 1.0])  # singular
    with pytest.raises(HopfError, match="positive definite"):
        solver.set_systems([with_W(spec, W)])
    solver.set_systems([spec])                   # a valid system still works afterwards
    r = solver.min_time(np.zeros((1, 6)))
    assert r["status"][0] == 1


def test_iteration_cap_is_reported_per_point(solver):
    """max_iter = 1 with a certificate after every iteration: every query that
    needs iterations ends NOCONV with T = NaN, points inside the target still
    report INSIDE, and the call succeeds."""
    say("case: max_iter = 1")
    spec = random_system(12, 2, 50, "l2", seed=5, t_max=4.0)
    solver.set_systems([spec])
    solver.set_opts(prec="fp32", c_tau=1.0, warm="cont", max_iter=1, check_every=1)
    x, _ = planted_drift_points(spec, 40, 0.3, 2.5, seed=8)
    x[:3] = 0.0                                  # the target's centre: inside
    r = solver.min_time(x)
    assert np.all(r["status"][:3] == 1) and np.all(r["T"][:3] == 0.0)
    assert np.all(r["status"][3:] == 3), np.bincount(r["status"], minlength=5)
    assert np.all(np.isnan(r["T"][3:]))
    v = solver.value(x[3:], np.full(37, 2.0))
    assert np.all(v["status"] == 3)


def test_damaged_network_changes_no_result(solver, tmp_path):
    """A network with garbage or non-finite parameters can only cost
    iterations: every learned start returns the cold search's statuses and
    minimum times."""
    from paper_1712_08226_amd.hopfpd import HopfError
    say("case: damaged warm-start network")
    spec = random_system(12, 2, 50, "l2", seed=5, t_max=4.0)
    solver.set_systems([spec])
    x, _ = planted_drift_points(spec, 64, 0.3, 2.5, seed=9)
    solver.set_opts(prec="fp32", c_tau=1.0, warm="cold")
    cold = solver.min_time(x)
    solver.warm_init(0, seed=1)
    theta, norm = solver.warm_get(0)
    rng = np.random.default_rng(4)
    n = spec.A.shape[0]
    norm = np.concatenate([np.zeros(n), np.ones(n), [spec.t_max, 1.0]]).astype(np.float32)
    for label, th in (("garbage", (rng.normal(0, 30.0, theta.size)).astype(np.float32)),
                      ("nan", np.full(theta.size, np.nan, dtype=np.float32))):
        solver.warm_set(th, norm, 0)
        for mode in ("mlp", "mlp_lam", "mlp_first"):
            solver.set_opts(prec="fp32", c_tau=1.0, warm=mode)
            r = solver.min_time(x)
            say(label, mode, "status", np.bincount(r["status"], minlength=5))
            assert np.array_equal(r["status"], cold["status"]), (label, mode)
            ok = cold["status"] == 0
            assert np.all(np.abs(r["T"][ok] - cold["T"][ok]) <= 1e-4 * cold["T"][ok]), (label, mode)
    # checkpoints: a round trip keeps the parameters; bad files are refused
    solver.warm_set(theta, norm, 0)
    path = str(tmp_path / "net.bin")
    solver.warm_save(path)
    solver.warm_init(0, seed=2)
    solver.warm_load(path)
    th2, nm2 = solver.warm_get(0)
    assert np.array_equal(th2, theta) and np.array_equal(nm2, norm)
    data = open(path, "rb").read()
    trunc = str(tmp_path / "trunc.bin")
    open(trunc, "wb").write(data[: len(data) // 2])
    with pytest.raises(HopfError):
        solver.warm_load(trunc)
    solver.set_systems([random_system(8, 2, 30, "l2", seed=6, t_max=3.0)])
    with pytest.raises(HopfError):
        solver.warm_load(path)                   # a network for another n
    solver.set_systems([spec])
    with pytest.raises(HopfError):
        solver.warm_load(str(tmp_path / "missing.bin"))


def test_target_that_is_not_diagonal_vs_oracle(solver):
    """W = Q diag(q) Q^T with a random rotation Q: the library solves in the
    rotated state and answers in the caller's coordinates; minimum times,
    values, costates and trajectories match the oracle, which uses W as
    given."""
    say("case: non-diagonal target")
    spec = random_system(8, 2, 60, "l2", seed=14, t_max=4.0)
    rng = np.random.default_rng(15)
    Q, _ = np.linalg.qr(rng.normal(size=(8, 8)))
    W = Q @ np.diag(rng.uniform(0.05, 0.2, 8)) @ Q.T
    W = 0.5 * (W + W.T)
    c = 0.05 * rng.normal(size=8)
    sysd = dict(A=spec.A, B=spec.B, W=W, c=c, uset="l2", N=60, t_max=4.0, quad="trap")
    solver.set_systems([sysd])
    solver.set_opts(prec="fp32", c_tau=1.0, warm="cont")
    S = O.System(spec.A, spec.B, W, c, uset="l2", N=60, t_max=4.0)
    x = gaussian_points(24, 8, 0.12, seed=16)
    r = solver.min_time(x)
    for k in range(0, 24, 4):
        o = O.min_time(S, x[k], O.Options(c_tau=1.0, warm="cont"))
        assert r["status"][k] == o.status, (k, r["status"][k], o.status)
        if o.status == O.PT_OK:
            assert abs(r["T"][k] - o.T) <= 1e-4 * o.T, (k, r["T"][k], o.T)
    t = np.linspace(0.3, 3.5, 24)
    v = solver.value(x, t)
    for k in (0, 7, 23):
        pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=1.0, gap_tol=1e-10, max_iter=400000))
        assert max(v["phi_lo"][k], pr.phi_lo) <= min(v["phi_hi"][k], pr.phi_hi) + 1e-9
        # lam* is unique (J* strongly convex): the certified gaps bound the distance
        mu = float(np.linalg.eigvalsh(W).min())
        gd = v["phi_hi"][k] - v["phi_lo"][k]
        dl = math.sqrt(2 * gd / mu) + math.sqrt(2 * max(pr.phi_hi - pr.phi_lo, 0) / mu)
        assert np.linalg.norm(v["lam"][k] - pr.lam) <= dl + 1e-6
    T = 1.9
    tr = solver.trajectory(x[3], T)
    pr = O.solve_value(S, x[3], T, O.Options(c_tau=1.0, gap_tol=1e-11, max_iter=400000))
    xT = O.terminal_state(S, pr.xf, pr.Ks, pr.y)
    np.testing.assert_allclose(tr["xs"][-1], xT, atol=2e-4 * max(1.0, np.abs(xT).max()))
    # x_T = W lam* + c in the caller's coordinates (grad J* at the optimum)
    np.testing.assert_allclose(tr["xs"][-1], W @ pr.lam + c, atol=2e-3)
