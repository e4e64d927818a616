"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the
same seeded inputs.

Bar (per result): certified value intervals [phi_lo, phi_hi] of the device
and the oracle overlap (both contain phi_N), the device gap is <= 1e-6, and
minimum times agree to |dT| <= 1e-4 T with identical per-point statuses.
Iterates are not compared: the device iterates in FP32 (or FP64), the
oracle in FP64, and both results are certified independently.
"""
import math
import sys

import numpy as np
import pytest
from scipy.linalg import expm

from gen import double_integrator, random_system, uniform_box_points, gaussian_points
from oracle import hopf_oracle as O

pytestmark = pytest.mark.gpu

GAP = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_1712_08226_amd import Solver
    s = Solver(0)
    yield s
    s.close()


def osys(spec, **kw):
    d = dict(uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    d.update(kw)
    return O.System(spec.A, spec.B, spec.W, spec.c, **d)


def overlap(a_lo, a_hi, b_lo, b_hi, tol=1e-9):
    return max(a_lo, b_lo) <= min(a_hi, b_hi) + tol * max(1.0, abs(a_hi), abs(b_hi))


def integrator(n, r, uset, N=40, t_max=5.0):
    return dict(A=np.zeros((n, n)), B=np.eye(n), W=(r * r) * np.eye(n), c=np.zeros(n), uset=uset,
                N=N, t_max=t_max, quad="trap")


# ------------------------------------------------------------------ value

@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_value_integrator_closed_form(solver, prec):
    """dx/dt = u: phi = 1/2 (max(0, ||x|| - t)^2 / r^2 - 1) inside the certified interval."""
    say("case: value integrator", prec)
    sysd = integrator(3, 0.3, "l2")
    solver.set_systems([sysd])
    solver.set_opts(prec=prec, c_tau=1.0)
    x = np.array([[0.9, -0.4, 0.2], [0.2, 0.1, 0.0], [1.5, 1.0, -1.0], [0.5, 0.5, 0.5]])
    t = np.array([0.3, 0.5, 1.2, 0.0])
    r = solver.value(x, t)
    for k in range(len(t)):
        exact = 0.5 * (max(0.0, np.linalg.norm(x[k]) - t[k]) ** 2 / 0.09 - 1.0)
        assert r["status"][k] == 0
        assert r["phi_lo"][k] - 1e-9 <= exact <= r["phi_hi"][k] + 1e-9, (k, r["phi_lo"][k], exact, r["phi_hi"][k])
        assert (r["phi_hi"][k] - r["phi_lo"][k]) / max(1.0, abs(r["phi_hi"][k])) <= GAP


@pytest.mark.parametrize("tail", [0, 512])
@pytest.mark.parametrize("uset,quad,n,m,prec", [("l2", "trap", 6, 2, "fp32"), ("box", "trap", 6, 2, "fp32"),
                                                ("l2", "left", 20, 3, "fp32"), ("box", "left", 6, 1, "fp64"),
                                                ("l2", "trap", 35, 5, "fp32")])
def test_value_random_system_vs_oracle(solver, uset, quad, n, m, prec, tail):
    """tail=0: 16-point tiles throughout; tail=512: the per-point tail solver
    (FP32 only; FP64 always runs on the tiles)."""
    say("case: value random", uset, quad, n, m, prec, "tail", tail)
    spec = random_system(n, m, 40, uset, seed=21, t_max=3.0, quad=quad)
    solver.set_systems([spec])
    solver.set_opts(prec=prec, c_tau=1.0, tail_max=tail)
    x = gaussian_points(70, n, 0.15, seed=4)          # 70 points: one full tile + a ragged one
    t = np.linspace(0.0, 3.0, 70)
    r = solver.value(x, t)
    S = osys(spec)
    for k in list(range(0, 70, 9)) + [69]:
        pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=1.0, gap_tol=1e-9, max_iter=400000))
        assert r["status"][k] == 0, (k, r["status"][k])
        assert overlap(r["phi_lo"][k], r["phi_hi"][k], pr.phi_lo, pr.phi_hi), (k, r["phi_lo"][k], r["phi_hi"][k], pr.phi_lo, pr.phi_hi)
        assert (r["phi_hi"][k] - r["phi_lo"][k]) / max(1.0, abs(r["phi_hi"][k])) <= GAP


# ------------------------------------------------------------------ minimum time

@pytest.mark.parametrize("prec,tail", [("fp64", 0), ("fp32", 0), ("fp32", 512)])
def test_min_time_double_integrator(solver, prec, tail):
    """Sec. VI-A system, r = 0.1, N = 100 trapezoid, 24 points of the
    [-2,2]^2 workload; every point is reachable (T <= 6)."""
    say("case: min_time double integrator", prec, "tail", tail)
    spec = double_integrator(0.1, 100)
    solver.set_systems([spec])
    solver.set_opts(prec=prec, c_tau=30.0, tail_max=tail)
    x = uniform_box_points(24, 2, -2.0, 2.0, seed=1)
    r = solver.min_time(x)
    S = osys(spec)
    for k in range(0, 24, 3):
        o = O.min_time(S, x[k], O.Options(c_tau=30.0))
        assert r["status"][k] == o.status, (k, r["status"][k], o.status)
        if o.status == O.PT_OK:
            assert abs(r["T"][k] - o.T) <= 1e-4 * o.T, (k, r["T"][k], o.T)
            assert r["gap"][k] <= GAP


@pytest.mark.parametrize("tail", [0, 512])
def test_min_time_integrator_closed_form(solver, tail):
    say("case: min_time integrator closed form", "tail", tail)
    solver.set_systems([integrator(3, 0.3, "l2", N=40, t_max=5.0)])
    solver.set_opts(prec="fp32", c_tau=1.0, tail_max=tail)
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1.0, size=(100, 3))
    r = solver.min_time(x)
    exact = np.maximum(0.0, np.linalg.norm(x, axis=1) - 0.3)
    for k in range(100):
        if exact[k] == 0.0:
            assert r["status"][k] == 1 and r["T"][k] == 0.0
        elif exact[k] > 5.0:
            assert r["status"][k] == 2 and math.isinf(r["T"][k])
        else:
            assert r["status"][k] == 0
            assert abs(r["T"][k] - exact[k]) <= 1e-4 * exact[k], (k, r["T"][k], exact[k])


@pytest.mark.parametrize("tail", [0, 512])
@pytest.mark.parametrize("uset,n,m,N", [("l2", 12, 2, 50), ("box", 12, 3, 50)])
def test_min_time_random_system_vs_oracle(solver, uset, n, m, N, tail):
    """tail=0: every round on the 16-point tiles; tail=512: the per-point
    tail solver takes the points after the first round group."""
    say("case: min_time random", uset, n, m, N, "tail", tail)
    spec = random_system(n, m, N, uset, seed=5, t_max=4.0)
    solver.set_systems([spec])
    solver.set_opts(prec="fp32", c_tau=1.0, tail_max=tail)
    x = gaussian_points(20, n, 0.12, seed=8)
    r = solver.min_time(x)
    S = osys(spec)
    for k in range(0, 20, 4):
        o = O.min_time(S, x[k], O.Options(c_tau=1.0))
        assert r["status"][k] == o.status, (k, r["status"][k], o.status)
        if o.status == O.PT_OK:
            assert abs(r["T"][k] - o.T) <= 1e-4 * o.T, (k, r["T"][k], o.T)
            assert r["gap"][k] <= GAP


def test_edge_cases(solver):
    say("case: edge cases")
    solver.set_systems([integrator(2, 0.3, "l2", N=20, t_max=1.0)])
    solver.set_opts(prec="fp32", c_tau=1.0)
    x = np.array([[3.0, 0.0], [0.1, 0.1], [np.nan, 0.0], [0.5, 0.2]])
    r = solver.min_time(x)
    assert list(r["status"]) == [2, 1, 4, 0]
    assert math.isinf(r["T"][0]) and r["T"][1] == 0.0 and math.isnan(r["T"][2])
    empty = solver.min_time(np.zeros((0, 2)))
    assert empty["T"].shape == (0,)


@pytest.mark.parametrize("quad,T", [("trap", 1.377), ("left", 1.9), ("trap", 1.6)])
def test_trajectory_readout_vs_oracle(solver, quad, T):
    """Control and trajectory read-out (Sec. IV eq. (27), Sec. V eq. (33)):
    node times, the terminal state (= certified x_T), the control where it is
    unique (nodes with ||K_k lam*|| not small), and p* = e^{T A^T} lam*."""
    say("case: trajectory", quad, T)
    spec = random_system(5, 2, 30, "l2", seed=17, t_max=3.0, quad=quad)
    solver.set_systems([spec])
    solver.set_opts(prec="fp32", c_tau=1.0, gap_tol=1e-7)
    x0 = np.array([0.4, -0.3, 0.25, 0.1, -0.2])
    tr = solver.trajectory(x0, T)
    S = osys(spec)
    pr = O.solve_value(S, x0, T, O.Options(c_tau=1.0, gap_tol=1e-11, max_iter=400000))
    s, u, xs, p = O.readout(S, x0, pr)
    assert len(tr["s"]) == len(s)
    np.testing.assert_allclose(tr["s"], s, atol=1e-12)
    xT = O.terminal_state(S, pr.xf, pr.Ks, pr.y)
    scale = max(1.0, np.abs(xT).max())
    np.testing.assert_allclose(tr["xs"][-1], xT, atol=2e-4 * scale)
    np.testing.assert_allclose(tr["p_star"], p, atol=2e-3 * max(1.0, np.abs(p).max()))
    # u_k is unique where K_k lam* != 0 (the unit vector along K_k lam* for the
    # l2 ball).  P is mu-strongly convex (mu = lambda_min(W)), so a certified
    # gap g bounds ||lam - lam*|| <= sqrt(2 g / mu), and the direction of
    # K_k lam moves by at most 2 ||K_k|| ||dlam|| / ||K_k lam*||; the
    # tolerance below is that bound for both solves (x2 for the dual read-out).
    mu = float(np.min(np.diag(spec.W)))
    g_dev = (tr["phi_hi"] - tr["phi_lo"])
    g_or = pr.phi_hi - pr.phi_lo
    dlam = math.sqrt(2 * max(g_dev, 0) / mu) + math.sqrt(2 * max(g_or, 0) / mu)
    Kl = O.apply_K(pr.Ks, pr.lam)
    order = np.argsort(-np.asarray(pr.tau), kind="stable")
    nKl = np.linalg.norm(Kl[order], axis=1)
    nK = np.array([np.linalg.norm(pr.Ks[k], 2) for k in order])
    big = nKl > 0.2 * nKl.max()
    assert big.sum() >= 3
    tol = 4.0 * nK[big] * dlam / nKl[big] + 5e-3
    err = np.linalg.norm(tr["u"][big] - u[big], axis=1)
    assert np.all(err <= tol), (err, tol)
    assert np.all(np.linalg.norm(tr["u"], axis=1) <= 1.0 + 1e-9)
    # the device's trajectory interior is the impulse march of its own
    # controls: x_j = e^{(s_j - s_{j-1}) A} x_{j-1} + w_j B u_j (Sec. V eq. (33))
    w_of = {round(T - t, 10): wk for t, wk in zip(pr.tau, pr.w)}
    cur, sp = x0.copy(), 0.0
    for j in range(len(s)):
        cur = expm((tr["s"][j] - sp) * spec.A) @ cur + w_of[round(tr["s"][j], 10)] * spec.B @ tr["u"][j]
        sp = tr["s"][j]
        np.testing.assert_allclose(tr["xs"][j], cur, atol=1e-9 * scale)
    # and it matches the oracle's interior within what the controls allow:
    # |dx_j| <= sum_{k <= j} w_k ||e^{(s_j - s_k) A} B|| du_k, with du_k the
    # bound above where u_k is unique and 2 (the ball's diameter) elsewhere
    du = np.full(len(s), 2.0)
    du[big] = np.minimum(2.0, tol)
    for j in range(len(s)):
        bound = sum(w_of[round(s[k], 10)] * np.linalg.norm(expm((s[j] - s[k]) * spec.A) @ spec.B, 2) * du[k]
                    for k in range(j + 1))
        assert np.linalg.norm(tr["xs"][j] - xs[j]) <= bound + 2e-4 * scale, (j, np.linalg.norm(tr["xs"][j] - xs[j]), bound)


# ------------------------------------------------------------------ streaming kernel and BF16 hi+lo

@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("uset,n,m", [("l2", 40, 20), ("box", 40, 20), ("l2", 30, 5)])
def test_value_streaming_and_bf16_vs_oracle(solver, prec, uset, n, m):
    """Large m (streaming kernel) and the BF16 hi+lo split: the certified
    interval must still contain phi_N and reach the gap tolerance."""
    say("case: value streaming", prec, uset, n, m)
    spec = random_system(n, m, 40, uset, seed=31, t_max=3.0)
    solver.set_systems([spec])
    solver.set_opts(prec=prec, c_tau=1.0, tail_max=0)    # every iteration in the streaming kernel
    x = gaussian_points(40, n, 0.1, seed=6)
    t = np.linspace(0.2, 3.0, 40)
    r = solver.value(x, t)
    S = osys(spec)
    for k in [0, 13, 27, 39]:
        pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=1.0, gap_tol=1e-9, max_iter=400000))
        assert r["status"][k] == 0, (k, r["status"][k])
        assert overlap(r["phi_lo"][k], r["phi_hi"][k], pr.phi_lo, pr.phi_hi), (k, r["phi_lo"][k], r["phi_hi"][k], pr.phi_lo, pr.phi_hi)
        assert (r["phi_hi"][k] - r["phi_lo"][k]) / max(1.0, abs(r["phi_hi"][k])) <= GAP


def test_value_bf16_c3_shape(solver):
    """n=200, m=20, box control, x ~ N(0, 4I) (the precision workload's
    shape and points, N reduced to 60 for test time): BF16 hi+lo, FP32 and the
    FP64 oracle give overlapping certified intervals at gap <= 1e-6."""
    say("case: value bf16 c3 shape")
    spec = random_system(200, 20, 60, "box", seed=1003, t_max=10.0)
    solver.set_systems([spec])
    x = gaussian_points(64, 200, 2.0, seed=3)
    t = np.linspace(0.5, 10.0, 64)
    res = {}
    for prec in ("fp32", "bf16x3"):
        solver.set_opts(prec=prec, c_tau=5.0)
        res[prec] = r = solver.value(x, t)
        say(prec, "status", np.bincount(r["status"], minlength=5), "iters", r["iters"].mean())
        assert np.all(r["status"] == 0)
        assert np.all((r["phi_hi"] - r["phi_lo"]) / np.maximum(1.0, np.abs(r["phi_hi"])) <= GAP)
    a, b = res["fp32"], res["bf16x3"]
    for k in range(64):
        assert overlap(a["phi_lo"][k], a["phi_hi"][k], b["phi_lo"][k], b["phi_hi"][k]), k
    S = osys(spec)
    for k in (0, 21, 63):
        pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=5.0))
        assert overlap(b["phi_lo"][k], b["phi_hi"][k], pr.phi_lo, pr.phi_hi), (k, b["phi_lo"][k], b["phi_hi"][k], pr.phi_lo, pr.phi_hi)

# ------------------------------------------------------------------ hybrid Newton-bisection

@pytest.mark.parametrize("prec,case,tail", [("fp64", "di", 0), ("fp32", "di", 512), ("fp32", "l2", 0),
                                           ("fp32", "l2", 512), ("fp32", "box", 512)])
def test_min_time_newton_vs_oracle(solver, prec, case, tail):
    """Sec. IV hybrid on the device against the oracle's hybrid: same
    statuses, |dT| <= 1e-4 T, gap <= 1e-6; fewer probes than bisection."""
    say("case: min_time newton", prec, case, "tail", tail)
    if case == "di":
        spec, c_tau = double_integrator(0.1, 100), 30.0
        x = uniform_box_points(24, 2, -2.0, 2.0, seed=1)
    else:
        spec, c_tau = random_system(12, 2 if case == "l2" else 3, 50, case, seed=5, t_max=4.0), 1.0
        x = gaussian_points(20, 12, 0.12, seed=8)
    solver.set_systems([spec])
    solver.set_opts(prec=prec, c_tau=c_tau, warm="cont", tail_max=tail)
    rb = solver.min_time(x)
    solver.set_opts(prec=prec, c_tau=c_tau, warm="cont", root="newton", tail_max=tail)
    rn = solver.min_time(x)
    say("probes bisect", rb["probes"].mean(), "newton", rn["probes"].mean(),
        "iters", rb["iters"].mean(), rn["iters"].mean())
    assert np.array_equal(rb["status"], rn["status"])
    ok = rn["status"] == 0
    assert rn["probes"][ok].mean() < rb["probes"][ok].mean()
    assert np.all(rn["gap"][ok] <= GAP)
    S = osys(spec)
    for k in range(0, len(x), 4):
        o = O.min_time(S, x[k], O.Options(c_tau=c_tau, warm="cont", root="newton"))
        assert rn["status"][k] == o.status, (k, rn["status"][k], o.status)
        if o.status == O.PT_OK:
            assert abs(rn["T"][k] - o.T) <= 1e-4 * o.T, (k, rn["T"][k], o.T)



# ------------------------------------------------------------------ per-point tail solver

def test_tail_solver_beyond_resident_workgroups(solver):
    """More tail points than workgroups resident at once (two per compute
    unit): the later workgroups queue behind the first and every point is
    still solved as on the tiles."""
    say("case: tail beyond residency")
    spec = random_system(24, 4, 60, "l2", seed=78, t_max=4.0)
    solver.set_systems([spec])
    from gen.workloads import planted_drift_points
    x, _ = planted_drift_points(spec, 1500, 0.2, 3.0, seed=14)
    res = {}
    for tail in (0, 2048):
        solver.set_opts(prec="fp32", c_tau=1.0, warm="cont", tail_max=tail, adapt=0)
        res[tail] = solver.min_time(x)
        tm = solver.last_timing()
        say("tail", tail, "points", tm["tail_points"], "s", tm["tail_kernel_s"])
        assert tm["tail_points"] == (len(x) if tail else 0)
    a, b = res[0], res[2048]
    assert np.array_equal(a["status"], b["status"])
    ok = a["status"] == 0
    assert ok.mean() > 0.9
    assert np.all(b["gap"][ok] <= GAP)
    # a horizon where |phi| is within the gap tolerance counts as reached, so
    # inside a cell where phi changes sign more than once the two summation
    # orders may close on different crossings; each T must still be one
    diff = np.flatnonzero(ok & (np.abs(a["T"] - b["T"]) > 1e-4 * a["T"]))
    say("points with different T:", len(diff))
    assert len(diff) <= 0.01 * len(x)
    if len(diff):
        solver.set_opts(prec="fp32", c_tau=1.0, max_iter=400000)
        for r in (a, b):
            v = solver.value(x[diff], r["T"][diff])
            assert np.all(v["status"] == 0)
            assert np.all(v["phi_lo"] <= 2e-6 * np.maximum(1.0, np.abs(v["phi_hi"]))), (diff, v["phi_lo"])


@pytest.mark.parametrize("mode,uset,quad", [("min_time", "l2", "trap"), ("min_time", "box", "trap"),
                                            ("min_time", "l2", "left"), ("value", "l2", "trap"),
                                            ("value", "box", "left")])
def test_tail_solver_matches_tiles(solver, mode, uset, quad):
    """The tail solver (matrix-vector FP32 iterations, in-kernel certificate,
    search step and probe setup) against the tiled rounds on the same points,
    both with fixed steps: identical statuses, certified results to the same
    tolerances; and it did take the points."""
    say("case: tail vs tiles", mode, uset, quad)
    spec = random_system(24, 4, 60, uset, seed=77, t_max=4.0, quad=quad)
    solver.set_systems([spec])
    from gen.workloads import planted_drift_points
    x, _ = planted_drift_points(spec, 70, 0.2, 3.0, seed=12)
    t = np.linspace(0.1, 4.0, 70)
    res = {}
    c_tau = 0.3 if uset == "box" else 1.0      # the step ratio the box control set is run with
    for tail in (0, 512):
        solver.set_opts(prec="fp32", c_tau=c_tau, warm="cont", tail_max=tail, adapt=0)
        res[tail] = solver.min_time(x) if mode == "min_time" else solver.value(x, t)
        tm = solver.last_timing()
        say("tail", tail, "points", tm["tail_points"], "rows", tm["tail_point_rows"], "s", tm["tail_kernel_s"])
        assert (tm["tail_points"] > 0) == (tail > 0)
    a, b = res[0], res[512]
    assert np.array_equal(a["status"], b["status"])
    ok = a["status"] == 0
    if mode == "min_time":
        assert np.all(np.abs(a["T"][ok] - b["T"][ok]) <= 1e-4 * a["T"][ok])
        assert np.all(b["gap"][ok] <= GAP)
    else:
        for k in np.flatnonzero(ok):
            assert overlap(a["phi_lo"][k], a["phi_hi"][k], b["phi_lo"][k], b["phi_hi"][k]), k
        assert np.all((b["phi_hi"] - b["phi_lo"])[ok] / np.maximum(1.0, np.abs(b["phi_hi"][ok])) <= GAP)
    S = osys(spec)
    for k in (0, 13, 33, 69):
        if mode == "min_time":
            o = O.min_time(S, x[k], O.Options(c_tau=c_tau, warm="cont"))
            assert b["status"][k] == o.status, (k, b["status"][k], o.status)
            if o.status == O.PT_OK:
                assert abs(b["T"][k] - o.T) <= 1e-4 * o.T, (k, b["T"][k], o.T)
        else:
            pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=c_tau, gap_tol=1e-9, max_iter=400000))
            assert overlap(b["phi_lo"][k], b["phi_hi"][k], pr.phi_lo, pr.phi_hi), k



@pytest.mark.parametrize("uset,quad,c_tau", [("box", "left", 1.0), ("box", "trap", 0.3), ("l2", "trap", 1.0)])
def test_adaptive_steps_converge_at_least_as_often(solver, uset, quad, c_tau):
    """Step adaptation in the tail solver (restarts with the primal-weight
    update) changes only the iteration path: every point certified with fixed
    steps is certified with adaptation too, the certified intervals overlap
    each other and the oracle's, and no more points hit max_iter."""
    say("case: adaptive steps", uset, quad, c_tau)
    spec = random_system(24, 4, 60, uset, seed=77, t_max=4.0, quad=quad)
    solver.set_systems([spec])
    from gen.workloads import planted_drift_points
    x, _ = planted_drift_points(spec, 70, 0.2, 3.0, seed=12)
    t = np.linspace(0.1, 4.0, 70)
    res = {}
    for adapt in (0, 1):
        solver.set_opts(prec="fp32", c_tau=c_tau, tail_max=512, adapt=adapt, max_iter=60000)
        res[adapt] = solver.value(x, t)
        say("adapt", adapt, "status", np.bincount(res[adapt]["status"], minlength=5), "iters", res[adapt]["iters"].mean())
    a, b = res[0], res[1]
    assert np.sum(b["status"] == 3) <= np.sum(a["status"] == 3)
    assert np.all(b["status"][a["status"] == 0] == 0)
    ok = b["status"] == 0
    assert np.all((b["phi_hi"] - b["phi_lo"])[ok] / np.maximum(1.0, np.abs(b["phi_hi"][ok])) <= GAP)
    for k in np.flatnonzero((a["status"] == 0) & ok):
        assert overlap(a["phi_lo"][k], a["phi_hi"][k], b["phi_lo"][k], b["phi_hi"][k]), k
    S = osys(spec)
    for k in np.flatnonzero(ok)[::17]:
        pr = O.solve_value(S, x[k], t[k], O.Options(c_tau=c_tau, gap_tol=1e-9, max_iter=400000))
        assert overlap(b["phi_lo"][k], b["phi_hi"][k], pr.phi_lo, pr.phi_hi), k


def test_value_dev_matches_host_call(solver):
    """hopf_value_dev (device buffers, caller's stream) gives the host call's
    results; a horizon outside [0, t_max] is rejected before any kernel runs,
    and a tensor of the wrong dtype is refused by the binding."""
    import torch
    from paper_1712_08226_amd.hopfpd import HopfError
    say("case: value_dev vs value")
    spec = random_system(20, 3, 40, "l2", seed=23, t_max=3.0)
    solver.set_systems([spec])
    solver.set_opts(prec="fp32", c_tau=1.0)
    x = gaussian_points(70, 20, 0.15, seed=6)
    t = np.linspace(0.0, 3.0, 70)
    r = solver.value(x, t)
    dev = torch.device("cuda:0")
    xd = torch.tensor(x, dtype=torch.float64, device=dev)
    td = torch.tensor(t, dtype=torch.float64, device=dev)
    lo = torch.empty(70, dtype=torch.float64, device=dev)
    hi = torch.empty_like(lo)
    lam = torch.empty(70, 20, dtype=torch.float64, device=dev)
    it = torch.empty(70, dtype=torch.int32, device=dev)
    st = torch.empty(70, dtype=torch.int32, device=dev)
    solver.value_dev(xd, td, lo, hi, st, lam=lam, iters=it, stream=torch.cuda.current_stream(dev))
    np.testing.assert_array_equal(st.cpu().numpy(), r["status"])
    np.testing.assert_array_equal(it.cpu().numpy(), r["iters"])
    np.testing.assert_allclose(lo.cpu().numpy(), r["phi_lo"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(hi.cpu().numpy(), r["phi_hi"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(lam.cpu().numpy(), r["lam"], rtol=1e-12, atol=1e-14)
    bad = td.clone()
    bad[5] = 3.5
    with pytest.raises(HopfError):
        solver.value_dev(xd, bad, lo, hi, st)
    with pytest.raises(ValueError):
        solver.value_dev(xd.float(), td, lo, hi, st)


def test_value_at_horizon_grid_vs_oracle(solver):
    """The paper's per-horizon layout (Sec. III-A: N left-rule nodes spread
    over [0, t]) on the Sec. VI-A level-set grid, FP64 iterations: every grid
    point certified, sampled points against the oracle's solve on the same
    nodes (which are i t / N, the paper's)."""
    from gen.configs import config_grid
    say("case: value at horizon, 50x50 grid")
    w = config_grid(50)
    spec = w.systems[0]
    t = 1.2
    solver.set_opts(prec="fp64", c_tau=10.0)
    r = solver.value_at_horizon(spec, w.x, t)
    assert np.all(r["status"] == 0), np.unique(r["status"], return_counts=True)
    gap = (r["phi_hi"] - r["phi_lo"]) / np.maximum(1.0, np.abs(r["phi_hi"]))
    assert gap.max() <= GAP
    S = O.System(spec.A, spec.B, spec.W, spec.c, uset=spec.uset, N=spec.N, t_max=t, quad=spec.quad)
    tau, wts, _ = O.nodes_and_weights(S, t)
    np.testing.assert_allclose(tau, np.arange(spec.N) * t / spec.N, rtol=0, atol=1e-12)
    np.testing.assert_allclose(wts, np.full(spec.N, t / spec.N), rtol=0, atol=1e-12)
    for i in [0, 1224, 1275, 2499] + list(range(37, 2500, 401)):
        pr = O.solve_value(S, w.x[i], t, O.Options(c_tau=10.0, gap_tol=1e-9, max_iter=400000))
        assert overlap(r["phi_lo"][i], r["phi_hi"][i], pr.phi_lo, pr.phi_hi), \
            (i, r["phi_lo"][i], r["phi_hi"][i], pr.phi_lo, pr.phi_hi)
