"""Pins for the FP64 oracle: closed forms, brute force, strong duality,
invariants and special cases.  Each test would fail under a plausible mistake
in the oracle (dropped term, wrong sign or index, transposed operand)."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import hopf_oracle as O
from gen import (double_integrator, random_system, tychastic_double_integrator, tychastic_points,
                 unscented_weights, unscented_double_integrator, unscented_points)
from tests import pin_helpers as PH


def sysobj(spec, **kw):
    d = dict(uset=spec.uset, N=spec.N, t_max=spec.t_max, quad=spec.quad)
    d.update(kw)
    return O.System(spec.A, spec.B, spec.W, spec.c, **d)


def ball_system(n, r, uset, N=40, t_max=5.0, quad=O.TRAP):
    """dx/dt = u (A = 0, B = I): the time-independent Hamiltonian case of
    Sec. II-A, where the quadrature is exact."""
    return O.System(np.zeros((n, n)), np.eye(n), (r * r) * np.eye(n), None, None,
                    uset, N, t_max, quad)


# ------------------------------------------------------------------ table / expm

def test_K_rows_double_integrator_closed_form():
    """e^{tau A} for the nilpotent A = [[0,1],[0,0]] is [[1,tau],[0,1]], so
    K_k = -B^T e^{tau_k A^T} = -[tau_k, 1]."""
    S = sysobj(double_integrator(0.1, 100))
    tau = np.array([0.0, 0.3, 1.7, 9.9])
    Ks = O.K_blocks(S, tau)
    for k, t in enumerate(tau):
        np.testing.assert_allclose(Ks[k], -np.array([[t, 1.0]]), rtol=0, atol=1e-14)


def test_K_rows_rotation_and_diagonal_closed_form():
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    B = np.array([[0.0], [1.0]])
    S = O.System(A, B, np.eye(2), uset=O.BOX, N=10, t_max=1.0)
    t = 0.7
    E = np.array([[math.cos(t), math.sin(t)], [-math.sin(t), math.cos(t)]])
    np.testing.assert_allclose(O.K_blocks(S, [t])[0], -(E @ B).T, atol=1e-14)
    d = np.array([-1.0, -0.25, 0.2])
    S2 = O.System(np.diag(d), np.eye(3)[:, :2], np.eye(3), uset=O.L2, N=10, t_max=1.0)
    np.testing.assert_allclose(O.K_blocks(S2, [t])[0], -(np.diag(np.exp(t * d))[:, :2]).T, atol=1e-14)


# ------------------------------------------------------------------ quadrature

@pytest.mark.parametrize("quad", [O.TRAP, O.LEFT])
def test_weights_sum_to_horizon_and_are_nonnegative(quad):
    S = ball_system(2, 0.3, O.L2, N=11, t_max=5.0, quad=quad)
    for T in [0.0, 0.1, 0.5, 0.51, 1.234, 3.0, 4.99, 5.0]:
        tau, w, partial = O.nodes_and_weights(S, T)
        assert np.all(w >= 0.0)
        assert abs(np.sum(w) - T) <= 1e-13
        assert np.all(tau <= T + 1e-13)


def test_trapezoid_weights_on_grid_and_exactness():
    """On a grid horizon the weights are the composite trapezoid rule, which
    integrates linear functions of tau exactly at every horizon."""
    S = ball_system(2, 0.3, O.L2, N=11, t_max=5.0)
    h = 0.5
    tau, w, partial = O.nodes_and_weights(S, 2.0)
    assert not partial
    np.testing.assert_allclose(w, [h / 2, h, h, h, h / 2], atol=1e-15)
    for T in [0.3, 1.7, 2.0, 4.6]:
        tau, w, _ = O.nodes_and_weights(S, T)
        assert abs(np.dot(w, 3.0 + 2.0 * tau) - (3.0 * T + T * T)) <= 1e-12


def test_left_rule_matches_paper_layout_at_tmax():
    """At T = t_max the left rule is the paper's t_i = i T/N, i = 0..N-1,
    each with weight T/N (eq. (17))."""
    S = ball_system(2, 0.3, O.L2, N=8, t_max=4.0, quad=O.LEFT)
    tau, w, _ = O.nodes_and_weights(S, 4.0)
    np.testing.assert_allclose(tau, np.arange(8) * 0.5, atol=1e-15)
    np.testing.assert_allclose(w, np.full(8, 0.5), atol=1e-15)


@pytest.mark.parametrize("quad", [O.TRAP, O.LEFT])
def test_weights_continuous_across_grid_points(quad):
    """phi_N must be continuous in T for bisection: the weight of every time
    value is continuous as T crosses a grid point."""
    S = ball_system(2, 0.3, O.L2, N=11, t_max=5.0, quad=quad)
    h = O.grid_step(S)

    def weight_map(T):
        tau, w, _ = O.nodes_and_weights(S, T)
        out = {}
        for t, x in zip(tau, w):
            out[round(t, 6)] = out.get(round(t, 6), 0.0) + x
        return out
    for k in [1, 3, 7]:
        a, b = weight_map(k * h - 1e-9), weight_map(k * h + 1e-9)
        keys = set(a) | set(b)
        for key in keys:
            assert abs(a.get(key, 0.0) - b.get(key, 0.0)) < 1e-8


# ------------------------------------------------------------------ closed forms (A = 0)

@pytest.mark.parametrize("x,t", [([0.9, -0.4, 0.2], 0.3), ([0.2, 0.1, 0.0], 0.5),
                                 ([1.5, 1.0, -1.0], 1.2), ([0.5, 0.5, 0.5], 0.0)])
def test_value_l2_ball_closed_form(x, t):
    """dx/dt = u, ||u||_2 <= 1, ball target of radius r:
    phi(x,t) = 1/2 (max(0, ||x|| - t)^2 / r^2 - 1)  (Hopf formula, eq. (6))."""
    r = 0.3
    S = ball_system(3, r, O.L2)
    pr = O.solve_value(S, np.array(x), t, O.Options(c_tau=1.0, gap_tol=1e-9))
    exact = 0.5 * (max(0.0, np.linalg.norm(x) - t) ** 2 / r ** 2 - 1.0)
    assert pr.phi_lo - 1e-9 <= exact <= pr.phi_hi + 1e-9
    assert pr.phi_hi - pr.phi_lo <= 1e-8 * max(1.0, abs(exact))


@pytest.mark.parametrize("x,t", [([0.9, -0.4], 0.3), ([0.2, 0.7], 0.25), ([1.5, -1.0], 1.1)])
def test_value_box_closed_form(x, t):
    """dx/dt = u, ||u||_inf <= 1: each coordinate moves by at most t, so
    phi = 1/2 (sum_i max(0, |x_i| - t)^2 / r^2 - 1)."""
    r = 0.3
    S = ball_system(2, r, O.BOX)
    pr = O.solve_value(S, np.array(x), t, O.Options(c_tau=1.0, gap_tol=1e-9))
    exact = 0.5 * (np.sum(np.maximum(0.0, np.abs(x) - t) ** 2) / r ** 2 - 1.0)
    assert pr.phi_lo - 1e-9 <= exact <= pr.phi_hi + 1e-9


@pytest.mark.parametrize("x", [[0.9, -0.4, 0.2], [2.0, 1.0, 0.5], [0.25, 0.0, 0.1]])
def test_min_time_l2_ball_closed_form(x):
    """T* = max(0, ||x|| - r) for dx/dt = u with the l2-ball control."""
    r = 0.3
    S = ball_system(3, r, O.L2, N=40, t_max=5.0)
    res = O.min_time(S, np.array(x), O.Options(c_tau=1.0))
    exact = max(0.0, np.linalg.norm(x) - r)
    if exact == 0.0:
        assert res.status == O.PT_INSIDE and res.T == 0.0
        return
    assert res.status == O.PT_OK
    assert res.lo <= exact + 1e-9 and exact <= res.hi + 1e-9
    assert abs(res.T - exact) <= 1e-4 * exact
    assert res.gap_n <= 1e-6


def test_min_time_off_centre_target():
    """dx/dt = u with the target centred at c: T* = max(0, ||x - c|| - r)."""
    r = 0.3
    c = np.array([0.5, -1.0, 0.25])
    S = O.System(np.zeros((3, 3)), np.eye(3), (r * r) * np.eye(3), c, None, O.L2, 40, 5.0)
    x = np.array([1.5, 0.0, -0.5])
    res = O.min_time(S, x, O.Options(c_tau=1.0))
    exact = np.linalg.norm(x - c) - r
    assert res.status == O.PT_OK and abs(res.T - exact) <= 1e-4 * exact


def test_min_time_box_closed_form():
    """Box control: T* solves sum_i max(0, |x_i| - T)^2 = r^2."""
    r = 0.3
    x = np.array([1.0, 0.6])
    S = ball_system(2, r, O.BOX, N=40, t_max=5.0)
    res = O.min_time(S, x, O.Options(c_tau=1.0))
    f = lambda T: np.sum(np.maximum(0.0, np.abs(x) - T) ** 2) - r * r   # noqa: E731
    lo, hi = 0.0, 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    assert abs(res.T - hi) <= 1e-4 * hi


def test_phi_monotone_in_t_for_integrator():
    """For dx/dt = u the value is nonincreasing in t."""
    S = ball_system(3, 0.3, O.L2)
    x = np.array([1.0, -0.5, 0.3])
    prev = math.inf
    for t in [0.0, 0.2, 0.4, 0.8, 1.2, 1.6]:
        pr = O.solve_value(S, x, t, O.Options(gap_tol=1e-9))
        assert pr.phi_lo <= prev + 1e-9
        prev = pr.phi_hi


# ------------------------------------------------------------------ special values

def test_phi_at_zero_horizon_is_terminal_cost():
    """phi(x, 0) = J(x), the initial condition of eq. (4)."""
    spec = random_system(6, 2, 20, "l2", seed=3)
    S = sysobj(spec)
    x = np.linspace(-1, 1, 6)
    pr = O.solve_value(S, x, 0.0)
    d = x - spec.c
    exact = 0.5 * (d @ np.linalg.solve(spec.W, d) - 1.0)
    assert abs(pr.phi_lo - exact) <= 1e-12 and abs(pr.phi_hi - exact) <= 1e-12


# ------------------------------------------------------------------ strong duality vs an independent solver

@pytest.mark.parametrize("uset,quad,T,shift", [("l2", O.TRAP, 1.37, 0.0), ("box", O.TRAP, 0.9, 0.2),
                                               ("l2", O.LEFT, 2.2, -0.15), ("box", O.TRAP, 2.0, 0.0)])
def test_strong_duality_against_independent_primal_solve(uset, quad, T, shift):
    """phi_N equals the optimum of the primal control problem over discrete
    controls (Fenchel-Rockafellar); the primal is solved here by projected
    gradient with expm from scipy, independently of the primal-dual method.
    Some cases move the target centre off the origin."""
    spec = random_system(4, 2, 16, uset, seed=11, t_max=3.0, quad=quad)
    c = shift * np.array([1.0, -2.0, 0.5, 1.0])
    S = O.System(spec.A, spec.B, spec.W, c, None, uset, spec.N, spec.t_max, quad)
    rng = np.random.default_rng(0)
    x = rng.normal(0, 0.6, 4)
    pr = O.solve_value(S, x, T, O.Options(c_tau=1.0, gap_tol=1e-10, max_iter=400000))
    assert pr.gap_n() <= 1e-10
    fval, _ = PH.primal_fista(spec.A, spec.B, spec.W, c, np.eye(2), uset, x, T,
                              pr.tau, pr.w, iters=40000)
    assert pr.phi_lo - 1e-9 <= fval + 1e-9
    assert abs(fval - pr.phi_hi) <= 1e-7 * max(1.0, abs(fval))


@pytest.mark.parametrize("steps", ["accel", "precond"])
@pytest.mark.parametrize("uset,quad,T,shift", [("l2", O.TRAP, 1.37, 0.0), ("box", O.TRAP, 0.9, 0.2),
                                               ("l2", O.LEFT, 2.2, -0.15)])
def test_step_variants_reach_the_primal_optimum(steps, uset, quad, T, shift):
    """The accelerated and the diagonally preconditioned iterations (Sec. III,
    Sec. III-A) converge to the same phi_N: the independent projected-gradient
    solve of the primal control problem lies in their certified interval,
    which is as tight as the fixed-step one."""
    spec = random_system(4, 2, 16, uset, seed=11, t_max=3.0, quad=quad)
    c = shift * np.array([1.0, -2.0, 0.5, 1.0])
    S = O.System(spec.A, spec.B, spec.W, c, None, uset, spec.N, spec.t_max, quad)
    x = np.random.default_rng(0).normal(0, 0.6, 4)
    pr = O.solve_value(S, x, T, O.Options(c_tau=1.0, gap_tol=1e-9, max_iter=2_000_000, steps=steps))
    assert pr.gap_n() <= 1e-9
    fval, _ = PH.primal_fista(spec.A, spec.B, spec.W, c, np.eye(2), uset, x, T, pr.tau, pr.w, iters=40000)
    assert pr.phi_lo - 1e-8 <= fval <= pr.phi_hi + 1e-8 * max(1.0, abs(fval))


def test_accelerated_steps_follow_the_schedule():
    """One accelerated step from (tau, sigma): theta = 1/sqrt(1 + 2 gamma tau),
    tau' = theta tau, sigma' = sigma / theta (tau sigma is kept), and the
    extrapolation is lam+ + theta (lam+ - lam); gamma = lambda_min(W)."""
    spec = random_system(5, 2, 12, "l2", seed=5, t_max=2.0)
    S = sysobj(spec)
    x = np.linspace(-0.5, 0.5, 5)
    pr = O.make_probe(S, x, 1.1, O.Options(c_tau=1.0, steps="accel"))
    assert abs(pr.gamma - np.min(np.linalg.eigvalsh(spec.W))) <= 1e-15
    t0, s0, lam0 = pr.tau_p, pr.sigma_d, pr.lam.copy()
    O.pdhg_iteration(S, pr)
    th = 1.0 / math.sqrt(1.0 + 2.0 * pr.gamma * t0)
    assert abs(pr.tau_p - th * t0) <= 1e-15 * t0 and abs(pr.sigma_d - s0 / th) <= 1e-12 * s0
    np.testing.assert_allclose(pr.lam_bar, pr.lam + th * (pr.lam - lam0), rtol=0, atol=1e-15)


def test_terminal_state_matches_costate():
    """At the optimum x_T = grad J*(lam*) = W lam* + c (Sec. V, eq. (29)), and
    the read-out trajectory ends at x_T; p* = e^{T A^T} lam*."""
    spec = random_system(4, 2, 16, "l2", seed=2, t_max=3.0)
    S = sysobj(spec)
    x = np.array([0.5, -0.3, 0.2, 0.4])
    T = 1.3
    pr = O.solve_value(S, x, T, O.Options(gap_tol=1e-11, max_iter=400000))
    xT = O.terminal_state(S, pr.xf, pr.Ks, pr.y)
    np.testing.assert_allclose(xT, spec.W @ pr.lam + spec.c, atol=1e-5)
    s, u, xs, p = O.readout(S, x, pr)
    np.testing.assert_allclose(xs[-1], xT, atol=1e-10)
    np.testing.assert_allclose(p, expm(T * spec.A.T) @ pr.lam, atol=1e-12)
    assert np.all(np.linalg.norm(u, axis=1) <= 1.0 + 1e-12)
    assert abs(s[-1] - T) < 1e-12 and s[0] >= -1e-12


def test_dphi_dT_equals_minus_hamiltonian():
    """d phi/dT = -H_x(p*, x0) with H_x(p, x) = -x^T A^T p + ||Qu^T B^T p||_*
    (Sec. IV); the discrete phi_N agrees up to the quadrature error."""
    spec = random_system(4, 2, 400, "l2", seed=4, t_max=4.0)
    S = sysobj(spec)
    x = np.array([0.6, -0.5, 0.4, 0.3])
    T, dT = 1.5, 1e-3
    opt = O.Options(gap_tol=1e-12, max_iter=2000000, check_every=50)
    a = O.solve_value(S, x, T - dT, opt)
    b = O.solve_value(S, x, T + dT, opt)
    mid = O.solve_value(S, x, T, opt)
    fd = (b.phi_hi - a.phi_hi) / (2 * dT)
    p = expm(T * spec.A.T) @ mid.lam
    H = O.hamiltonian_x(S, p, x)
    assert abs(fd + H) <= 2e-2 * max(1.0, abs(H))


# ------------------------------------------------------------------ invariants

def test_similarity_invariance():
    """x' = S x, A' = S A S^-1, B' = S B, W' = S W S^T, c' = S c leave phi
    and T* unchanged."""
    spec = random_system(3, 1, 30, "l2", seed=8, t_max=4.0)
    rng = np.random.default_rng(1)
    Sm = rng.normal(size=(3, 3)) + 2 * np.eye(3)
    S1 = sysobj(spec)
    S2 = O.System(Sm @ spec.A @ np.linalg.inv(Sm), Sm @ spec.B, Sm @ spec.W @ Sm.T, Sm @ spec.c,
                  uset="l2", N=30, t_max=4.0)
    x = np.array([0.4, -0.35, 0.3])
    opt = O.Options(gap_tol=1e-9, max_iter=400000)
    a = O.solve_value(S1, x, 1.1, opt)
    b = O.solve_value(S2, Sm @ x, 1.1, opt)
    assert max(a.phi_lo, b.phi_lo) <= min(a.phi_hi, b.phi_hi) + 1e-9


def test_control_scaling_equivalence():
    """U = Qu C with Qu = 2 I equals B' = 2 B with Qu = I."""
    spec = random_system(3, 2, 20, "box", seed=9, t_max=3.0)
    S1 = O.System(spec.A, spec.B, spec.W, spec.c, 2 * np.eye(2), "box", 20, 3.0)
    S2 = O.System(spec.A, 2 * spec.B, spec.W, spec.c, None, "box", 20, 3.0)
    x = np.array([0.8, -0.6, 0.5])
    opt = O.Options(gap_tol=1e-9, max_iter=400000)
    a = O.solve_value(S1, x, 0.8, opt)
    b = O.solve_value(S2, x, 0.8, opt)
    assert max(a.phi_lo, b.phi_lo) <= min(a.phi_hi, b.phi_hi) + 1e-9


def test_planted_point_value_bound():
    """Plant x0 = e^{-T0 A}(x_T - sum_k w_k e^{tau_k A} B u_k) with x_T inside
    the target and feasible u_k: then phi_N(x0, T0) <= J(x_T) < 0."""
    spec = random_system(5, 2, 40, "l2", seed=6, t_max=3.0)
    S = sysobj(spec)
    rng = np.random.default_rng(5)
    T0 = 1.7
    tau, w, _ = O.nodes_and_weights(S, T0)
    u = rng.normal(size=(len(tau), 2))
    u /= np.maximum(1.0, np.linalg.norm(u, axis=1, keepdims=True))
    xT = 0.5 * np.sqrt(np.diag(spec.W)) * rng.uniform(-1, 1, 5)
    drive = sum(wk * expm(t * spec.A) @ spec.B @ uk for t, wk, uk in zip(tau, w, u))
    x0 = expm(-T0 * spec.A) @ (xT - drive)
    pr = O.solve_value(S, x0, T0, O.Options(gap_tol=1e-9, max_iter=400000))
    JxT = 0.5 * (xT @ np.linalg.solve(spec.W, xT) - 1.0)
    assert pr.phi_lo <= JxT + 1e-9


# ------------------------------------------------------------------ double integrator (Sec. VI-A)

def test_double_integrator_textbook_anchors():
    """Closed-form anchors of the double integrator (the paper chose it
    because closed-form optimal solutions exist, Sec. VI-A)."""
    with open("tests/golden/double_integrator_origin.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for p, v, T in rows:
        assert abs(PH.di_time_to_origin(float(p), float(v)) - float(T)) < 1e-12


@pytest.mark.slow
def test_double_integrator_min_time_vs_bang_bang():
    """Discrete T_N* (trapezoid, N=100, r=0.1) against the continuous minimum
    time from one-switch bang-bang brute force; the quadrature error is
    O(h^2) with h = 10/99."""
    spec = double_integrator(0.1, 100)
    S = sysobj(spec)
    opt = O.Options(c_tau=30.0)
    for x in [(1.0, 0.0), (-0.5, 1.0), (1.2, -0.8)]:
        Tc = PH.di_min_time_ball(x[0], x[1], 0.1)
        res = O.min_time(S, np.array(x), opt)
        assert res.status == O.PT_OK
        assert abs(res.T - Tc) <= 3e-4 * Tc + 0.02 * O.grid_step(S) ** 2, (x, res.T, Tc)


@pytest.mark.slow
def test_double_integrator_converges_in_N():
    """Convergence to the continuous minimum time as N grows: the left
    rule's error is first order (doubling N roughly halves it once N >= 100)
    and the trapezoid's error is smaller at every N."""
    Tc = PH.di_min_time_ball(1.0, 0.0, 0.1)
    errs = {O.LEFT: [], O.TRAP: []}
    for quad in (O.LEFT, O.TRAP):
        for N in [100, 200, 400]:
            S = sysobj(double_integrator(0.1, N, quad=quad))
            res = O.min_time(S, np.array([1.0, 0.0]), O.Options(c_tau=30.0, t_rel_tol=2e-7))
            errs[quad].append(abs(res.T - Tc))
    e = errs[O.LEFT]
    assert e[0] > e[1] > e[2]
    assert 1.3 < e[0] / e[1] < 2.6 and 1.3 < e[1] / e[2] < 2.6
    t = errs[O.TRAP]
    assert t[0] > t[1] > t[2]
    assert all(a < b for a, b in zip(t, e))


@pytest.mark.slow
def test_double_integrator_vs_grid_hamilton_jacobi():
    """Brute-force grid HJ (semi-Lagrangian dynamic programming) on 2-D
    inputs: agreement within the grid's own error (a few cells of time)."""
    g, Tg = PH.di_grid_min_time()
    S = sysobj(double_integrator(0.1, 100))
    for x in [(1.0, 0.0), (-1.0, 0.5), (0.5, -1.0), (1.5, 1.0)]:
        res = O.min_time(S, np.array(x), O.Options(c_tau=30.0))
        Tgrid = PH.grid_lookup(g, Tg, *x)
        assert abs(res.T - Tgrid) <= 0.08 + 0.03 * res.T, (x, res.T, Tgrid)


def test_unreachable_and_inside_statuses():
    S = ball_system(2, 0.3, O.L2, N=20, t_max=1.0)
    r = O.min_time(S, np.array([3.0, 0.0]))
    assert r.status == O.PT_UNREACH and math.isinf(r.T)
    r = O.min_time(S, np.array([0.1, 0.1]))
    assert r.status == O.PT_INSIDE and r.T == 0.0
    r = O.min_time(S, np.array([np.nan, 0.0]))
    assert r.status == O.PT_NONFINITE


# ------------------------------------------------------------------ hybrid Newton-bisection (Sec. IV)

def test_value_slope_is_exact_left_rule_derivative():
    """For the left rule the discrete value is differentiable between grid
    points with d phi_N/dT = <A x_f, lam*> - sigma_C(K_M lam*) (envelope
    theorem: only x_f and the last weight r depend on T).  Central finite
    differences of tightly solved values must match the slope from lam*."""
    spec = random_system(5, 2, 40, "l2", seed=14, t_max=4.0, quad="left")
    S = sysobj(spec)
    x = np.array([0.7, -0.4, 0.5, 0.2, -0.3])
    opt = O.Options(gap_tol=1e-13, max_iter=3000000, check_every=50)
    h = O.grid_step(S)
    for T in (0.37 * 4.0 + 0.3 * h, 2.0 + 0.55 * h):
        d = 1e-4 * h                   # stays between two grid points
        a = O.solve_value(S, x, T - d, opt)
        b = O.solve_value(S, x, T + d, opt)
        mid = O.solve_value(S, x, T, opt)
        fd = (-0.5 * (b.P + b.D) + 0.5 * (a.P + a.D)) / (2 * d)
        s = O.value_slope(S, mid)
        assert abs(fd - s) <= 1e-5 * max(1.0, abs(s)), (T, fd, s)


def test_value_slope_sign_flip_fails():
    """The slope is negative where the target is being approached: a flipped
    sign of either term would break the Newton step (integrator closed form
    d phi/dT = -(||x|| - T)/r^2 for the unit l2 ball)."""
    r = 0.3
    S = ball_system(3, r, O.L2, N=40, t_max=5.0)
    x = np.array([0.9, -0.4, 0.2])
    T = 0.5
    pr = O.solve_value(S, x, T, O.Options(gap_tol=1e-12, max_iter=400000))
    exact = -(np.linalg.norm(x) - T) / (r * r)
    assert abs(O.value_slope(S, pr) - exact) <= 1e-5 * abs(exact)


@pytest.mark.parametrize("x", [[0.9, -0.4, 0.2], [2.0, 1.0, 0.5], [1.1, 0.3, -0.7]])
def test_newton_min_time_l2_ball_closed_form(x):
    """Hybrid Newton-bisection finds T* = ||x|| - r within the stopping
    tolerance, in fewer probes than bisection."""
    r = 0.3
    S = ball_system(3, r, O.L2, N=40, t_max=5.0)
    exact = np.linalg.norm(x) - r
    rn = O.min_time(S, np.array(x), O.Options(c_tau=1.0, root="newton", warm="cont"))
    rb = O.min_time(S, np.array(x), O.Options(c_tau=1.0, warm="cont"))
    assert rn.status == O.PT_OK and rn.lo <= exact + 1e-9 <= rn.hi + 2e-9
    assert abs(rn.T - exact) <= 1e-4 * exact and rn.gap_n <= 1e-6
    assert rn.probes < rb.probes


def test_newton_double_integrator_vs_bang_bang():
    """Same bang-bang anchors as bisection (Sec. VI-A system)."""
    spec = double_integrator(0.1, 100)
    S = sysobj(spec)
    for x in [(1.0, 0.0), (-0.5, 1.0), (1.2, -0.8)]:
        Tc = PH.di_min_time_ball(x[0], x[1], 0.1)
        res = O.min_time(S, np.array(x), O.Options(c_tau=30.0, root="newton", warm="cont"))
        assert res.status == O.PT_OK
        assert abs(res.T - Tc) <= 3e-4 * Tc + 0.02 * O.grid_step(S) ** 2, (x, res.T, Tc)


def test_newton_and_bisection_bracket_the_same_crossing():
    """On a random system the two searches end on brackets of width <= tol
    that overlap (the same sign change of phi_N)."""
    spec = random_system(8, 2, 50, "l2", seed=5, t_max=4.0)
    S = sysobj(spec)
    from gen.workloads import planted_drift_points
    xs, _ = planted_drift_points(spec, 4, 0.3, 2.5, seed=2)
    for x in xs:
        rb = O.min_time(S, x, O.Options(c_tau=1.0, warm="cont"))
        rn = O.min_time(S, x, O.Options(c_tau=1.0, warm="cont", root="newton"))
        assert rb.status == rn.status == O.PT_OK
        assert max(rb.lo, rn.lo) <= min(rb.hi, rn.hi) + 1e-12
        assert abs(rb.T - rn.T) <= 1e-4 * rb.T


# ------------------------------------------------------------------ tychastic double integrator (Sec. VI-B/C)

@pytest.mark.slow
def test_tychastic_identical_copies_reduce_to_double_integrator():
    """k equal copies that share one control, with the mean-squared target
    ell = r^2: the problem is the double integrator with the disk of radius
    r, so the discrete minimum time matches one-switch bang-bang brute force
    within the same quadrature bound as the single system."""
    k, r = 3, 0.1
    S = sysobj(tychastic_double_integrator(k, ell=r * r, N=100, t_max=10.0, quad="trap"))
    res = O.min_time(S, np.tile([1.0, 0.0], k), O.Options(c_tau=30.0))
    Tc = PH.di_min_time_ball(1.0, 0.0, r)
    assert res.status == O.PT_OK
    assert abs(res.T - Tc) <= 3e-4 * Tc + 0.02 * O.grid_step(S) ** 2, (res.T, Tc)


def test_tychastic_value_splits_into_mean_and_spread():
    """All copies share the control, so each copy's deviation delta_i from the
    sample mean evolves as e^{tA} delta_i whatever the control.  With the
    mean-squared target ell the value therefore splits exactly (also after
    discretisation) into the double integrator's value at the mean, with the
    disk of radius sqrt(ell), plus s(T) / (2 ell), s(T) = mean_i |e^{TA} delta_i|^2,
    where e^{TA} = [[1, T], [0, 1]]."""
    k, ell = 4, 0.04
    S = sysobj(tychastic_double_integrator(k, ell=ell, N=100, t_max=2.0, quad="left"))
    S2 = sysobj(double_integrator(math.sqrt(ell), 100, t_max=2.0, quad="left"))
    opt = O.Options(c_tau=0.5, gap_tol=1e-10, max_iter=400000)
    X = tychastic_points(k, 3, (1.0, 0.0), 0.0667, 21)
    for x in X:
        chi = x.reshape(k, 2)
        mean = chi.mean(axis=0)
        for T in (0.7, 2.0):
            E = np.array([[1.0, T], [0.0, 1.0]])
            s = float(np.mean(np.sum(((chi - mean) @ E.T) ** 2, axis=1)))
            a = O.solve_value(S, x, T, opt)
            b = O.solve_value(S2, mean, T, opt)
            assert a.gap_n() <= 1e-10 and b.gap_n() <= 1e-10
            lo, hi = b.phi_lo + s / (2 * ell), b.phi_hi + s / (2 * ell)
            assert max(a.phi_lo, lo) <= min(a.phi_hi, hi) + 1e-9, (T, a.phi_lo, a.phi_hi, lo, hi)
            assert abs(s / (2 * ell)) > 1e-3     # the spread term is not negligible


@pytest.mark.slow
def test_unscented_with_no_spread_is_the_double_integrator():
    """Five equal sigma points (zero covariance): the weights sum to one, so
    the weighted target is the disk of radius sqrt(ell) and the 10-state
    problem's minimum time is the double integrator's, against one-switch
    bang-bang brute force within the single system's quadrature bound."""
    r = 0.1
    S = sysobj(unscented_double_integrator(ell=r * r, N=100, t_max=10.0, quad="trap"))
    res = O.min_time(S, np.tile([1.0, 0.0], 5), O.Options(c_tau=30.0))
    Tc = PH.di_min_time_ball(1.0, 0.0, r)
    assert res.status == O.PT_OK
    assert abs(res.T - Tc) <= 3e-4 * Tc + 0.02 * O.grid_step(S) ** 2, (res.T, Tc)


@pytest.mark.slow
def test_unscented_min_time_is_the_crossing_of_reduced_value_plus_spread():
    """The reduced minimum-time search rests on phi(x, T) = phi_red(mean, T) +
    s(T) at every horizon: at the full 10-state system's first crossing T*
    the reduced value plus the weighted spread is reached (<= 0), and one
    stopping tolerance earlier it is not, with s(T) of the size that makes
    the difference."""
    ell = 0.04
    w, _ = unscented_weights(2)
    S = sysobj(unscented_double_integrator(ell, N=100, t_max=2.0, quad="left"))
    S2 = sysobj(double_integrator(math.sqrt(ell), 100, t_max=2.0, quad="left"))
    opt = O.Options(c_tau=0.5, gap_tol=1e-10, max_iter=400000)
    X = unscented_points(2, (0.7, -0.2), (1.0, 0.1), 0.0667, 24)
    X = X + 0.03 * np.random.default_rng(6).normal(size=X.shape)
    for x in X:
        r = O.min_time(S, x, O.Options(c_tau=0.5))
        assert r.status == O.PT_OK
        chi = x.reshape(5, 2)
        mean = w @ chi

        def reduced(T):
            E = np.array([[1.0, T], [0.0, 1.0]])
            s = float(w @ np.sum(((chi - mean) @ E.T) ** 2, axis=1)) / (2 * ell)
            b = O.solve_value(S2, mean, T, opt)
            return b.phi_hi + s, s
        at, s_at = reduced(r.T)
        before, _ = reduced(r.T - 2e-4 * r.T - 2e-6)
        assert at <= 1e-6 and before > 0.0, (r.T, at, before)
        assert s_at > 1e-2


def test_unscented_costates_from_the_reduced_solve():
    """The full system's optimal costate per sigma point is rebuilt from the
    reduced solve at the weighted mean: lam_c = a_c (W_b^-1 e^{TA}(chi_c -
    mean) + lam_red / a), a_c = w_c / w_0, a = sum_c a_c (W_b = ell/w_0 I, the
    first block).  Dropping a_c or the 1/a share fails by a factor of two or
    more on the four outer points."""
    ell, T = 0.04, 1.3
    w, _ = unscented_weights(2)
    S = sysobj(unscented_double_integrator(ell, N=100, t_max=2.0, quad="left"))
    S2 = sysobj(double_integrator(math.sqrt(ell), 100, t_max=2.0, quad="left"))
    opt = O.Options(c_tau=0.5, gap_tol=1e-12, max_iter=800000)
    x = unscented_points(1, (0.8, -0.2), (1.2, 0.2), 0.0667, 25)[0] + 0.05 * np.random.default_rng(9).normal(size=10)
    full = O.solve_value(S, x, T, opt)
    chi = x.reshape(5, 2)
    mean = w @ chi
    red = O.solve_value(S2, mean, T, opt)
    E = np.array([[1.0, T], [0.0, 1.0]])
    a = w / w[0]
    wb_inv = w[0] / ell
    lam = np.concatenate([a[c] * (wb_inv * (E @ (chi[c] - mean)) + red.lam / a.sum()) for c in range(5)])
    assert np.max(np.abs(full.lam - lam)) <= 1e-4 * np.max(np.abs(full.lam)), np.max(np.abs(full.lam - lam))


def test_sigma_points_reproduce_the_moments():
    """The 2n+1 sigma points with their mean weights reproduce the mean and
    covariance of N(mu, std^2 I_2) exactly; the weights sum to one and, with
    kappa = 3 - n, are all positive (so the weighted target is an ellipsoid)."""
    w, lam = unscented_weights(2)
    assert abs(w.sum() - 1.0) <= 1e-15 and np.all(w > 0) and lam == 1.0
    X = unscented_points(4, (0.5, -0.3), (1.5, 0.3), 0.0667, 3).reshape(4, 5, 2)
    mu = np.einsum("i,qia->qa", w, X)
    assert np.allclose(mu, X[:, 0, :], atol=1e-15)
    D = X - mu[:, None, :]
    C = np.einsum("i,qia,qib->qab", w, D, D)
    assert np.allclose(C, 0.0667 ** 2 * np.eye(2)[None], atol=1e-15)


def test_unscented_value_splits_into_weighted_mean_and_spread():
    """Sigma points weighted by w_i in the target (W blocks ell / w_i): as for
    equal samples the copies share the control, so the value of the 10-dim
    system splits exactly into the double integrator's value at the weighted
    mean with the disk of radius sqrt(ell) (sum_i w_i = 1) plus
    sum_i w_i |e^{TA}(chi_i - mean)|^2 / (2 ell).  Points with their sigma
    points off-centre (mean != chi_0) make the weighting matter."""
    ell = 0.04
    w, _ = unscented_weights(2)
    S = sysobj(unscented_double_integrator(ell, N=100, t_max=2.0, quad="left"))
    S2 = sysobj(double_integrator(math.sqrt(ell), 100, t_max=2.0, quad="left"))
    opt = O.Options(c_tau=0.5, gap_tol=1e-10, max_iter=400000)
    rng = np.random.default_rng(5)
    X = unscented_points(2, (0.8, -0.2), (1.2, 0.2), 0.0667, 22)
    X = X + 0.05 * rng.normal(size=X.shape)          # a general stack of 5 states
    for x in X:
        chi = x.reshape(5, 2)
        mean = w @ chi
        for T in (0.7, 2.0):
            E = np.array([[1.0, T], [0.0, 1.0]])
            s = float(w @ np.sum(((chi - mean) @ E.T) ** 2, axis=1))
            a = O.solve_value(S, x, T, opt)
            b = O.solve_value(S2, mean, T, opt)
            assert a.gap_n() <= 1e-10 and b.gap_n() <= 1e-10
            lo, hi = b.phi_lo + s / (2 * ell), b.phi_hi + s / (2 * ell)
            assert max(a.phi_lo, lo) <= min(a.phi_hi, hi) + 1e-9, (T, a.phi_lo, a.phi_hi, lo, hi)
            # the plain (unweighted) mean and spread do not give the value
            um = chi.mean(axis=0)
            us = float(np.mean(np.sum(((chi - um) @ E.T) ** 2, axis=1)))
            c = O.solve_value(S2, um, T, opt)
            assert abs(c.phi_hi + us / (2 * ell) - a.phi_hi) > 1e-4


@pytest.mark.parametrize("T", [3.0, 1.37])
def test_operator_norm_bound_against_singular_values(T):
    """L (which sets both step sizes) is the spectral norm of the stacked K on
    the table nodes, from the largest singular value of the stacked matrix
    (a different computation from the oracle's eigenvalue of the Gram sum);
    with an off-grid horizon the extra node's Frobenius term keeps L an upper
    bound of ||K||."""
    spec = random_system(6, 2, 30, "l2", seed=31, t_max=3.0)
    S = sysobj(spec)
    tau, w, partial = O.nodes_and_weights(S, T)
    Ks = O.K_blocks(S, tau)
    L = O.op_norm_bound(S, Ks, partial)
    full = np.linalg.norm(Ks.reshape(-1, 6), 2)
    if partial:
        table = np.linalg.norm(Ks[:-1].reshape(-1, 6), 2)
        assert full <= L + 1e-12
        assert abs(L ** 2 - table ** 2 - np.sum(Ks[-1] ** 2)) <= 1e-10 * L ** 2
    else:
        assert abs(L - full) <= 1e-10 * full


# ------------------------------------------------------------------ first crossing (Sec. IV: the smallest T with phi = 0)

def rotation_system(eps=0.05, r=0.5, N=200, t_max=10.0):
    """Harmonic oscillator x1' = x2, x2' = -x1 (e^{tA} a rotation) with l2
    control of radius eps in both coordinates and the disk of radius r at
    c = (0, -2).  The free motion from (2, 0) is (2 cos t, -2 sin t): it
    passes through the disk near t = pi/2 + 2 pi k and leaves it again."""
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    return O.System(A, eps * np.eye(2), (r * r) * np.eye(2), np.array([0.0, -2.0]), None,
                    O.L2, N, t_max, O.TRAP)


def rotation_first_crossing(eps=0.05, r=0.5):
    """Closed form.  Because every e^{sA} is a rotation, the points reachable
    at time t are the disk of radius eps t around the free motion, and so
    are those of the quadrature form (sum_k w_k = t, every u_k can be turned
    to the same direction).  The target is reached exactly when
    |x_free(t) - c| = sqrt(8 - 8 sin t) <= r + eps t; T* is the first root."""
    from scipy.optimize import brentq
    f = lambda t: math.sqrt(max(8.0 - 8.0 * math.sin(t), 0.0)) - r - eps * t
    return brentq(f, 0.5, math.pi / 2, xtol=1e-14)


def test_rotation_reach_set_closed_form_sign_pattern():
    """phi_N(x, t) <= 0 exactly where the closed form says the disk is
    reached: twice in [0, 10] with an unreachable stretch in between and at
    t_max, so a search that looks only at t_max misses the first crossing."""
    S = rotation_system()
    x = np.array([2.0, 0.0])
    opt = O.Options(c_tau=1.0, max_iter=400000)
    for t in (1.0, 1.6, 4.0, 7.85, 10.0):
        dist = math.sqrt(max(8.0 - 8.0 * math.sin(t), 0.0))
        reach = dist <= 0.5 + 0.05 * t
        pr = O.make_probe(S, x, t, opt)
        out = O.sign_probe(S, pr, opt)
        assert out == (O.REACH if reach else O.UNREACH), (t, out, dist)


@pytest.mark.parametrize("root", ["bisect", "newton"])
def test_min_time_is_the_first_crossing(root):
    """On the rotation system the search returns the first crossing of the
    closed form (not +inf, which the value at t_max alone would suggest),
    within the search tolerance and the trapezoid's exactness."""
    S = rotation_system()
    Tc = rotation_first_crossing()
    res = O.min_time(S, np.array([2.0, 0.0]), O.Options(c_tau=1.0, warm="cont", root=root))
    assert res.status == O.PT_OK
    assert res.lo <= Tc + 1e-9 and abs(res.T - Tc) <= 1e-4 * Tc, (res.T, Tc)
    assert res.gap_n <= 1e-6


def test_min_time_unreachable_needs_every_scan_horizon():
    """UNREACH only when every scan horizon is certified unreachable: a
    start far from the target probes all of them."""
    S = rotation_system(eps=0.01)
    opt = O.Options(c_tau=1.0, warm="cont", scan=16)
    res = O.min_time(S, np.array([6.0, 0.0]), opt)
    assert res.status == O.PT_UNREACH and math.isinf(res.T)
    nodes = O.scan_nodes(S, opt)
    assert nodes[-1] == S.N - 1 and len(nodes) == 16 and all(np.diff(nodes) > 0)
    assert res.scan_probes == 16 and res.probes == 16


def test_scan_nodes_and_node_bisection_bookkeeping():
    """Scan horizons are table nodes, strictly ascending, ending at t_max;
    the nodes strictly inside a bracket are found exactly at node horizons
    and between them."""
    S = rotation_system(N=300)
    h = O.grid_step(S)
    nodes = O.scan_nodes(S, O.Options(scan=48))
    assert nodes[0] == 1 and nodes[-1] == 299 and all(np.diff(nodes) > 0)
    assert O.node_horizon(S, 299) == S.t_max
    assert O.inner_nodes(S, 5 * h, 9 * h) == (6, 8)
    assert O.inner_nodes(S, 5.5 * h, 9.2 * h) == (6, 9)
    ka, kb = O.inner_nodes(S, 5 * h, 6 * h)
    assert ka > kb


def test_min_time_hint_inside_the_cell_is_probed_first():
    """Hints t_bracket = (a, b) strictly inside the first cell are the first
    probes after the scan; the answer is unchanged (single crossing)."""
    S = rotation_system()
    Tc = rotation_first_crossing()
    a, b = Tc - 1e-3, Tc + 1e-3
    plain = O.min_time(S, np.array([2.0, 0.0]), O.Options(c_tau=1.0, warm="cont"))
    hinted = O.min_time(S, np.array([2.0, 0.0]), O.Options(c_tau=1.0, warm="cont"), t_bracket=(a, b))
    assert hinted.status == O.PT_OK and abs(hinted.T - Tc) <= 1e-4 * Tc
    assert hinted.probes < plain.probes


@pytest.mark.slow
def test_planted_points_of_the_n100_workload_reach_by_T0():
    """The drift-planted start points of the n=100, m=10, N=300 workload hit
    the target's boundary at T0 under zero control, so phi_N(x0, T0) <= 0
    and the first crossing is at most T0.  Every one of them must come back
    reached with T <= T0 (1 + 1e-4)."""
    from gen.configs import config5
    from gen.workloads import planted_drift_points
    wl = config5(npts=8)
    spec = wl.systems[0]
    S = sysobj(spec)
    x, T0 = planted_drift_points(spec, 8192, 0.2, 3.0, 5)
    # points whose reachable horizons form one short interval around T0
    # (about [0.85 T0, 1.4 T0]): a uniform scan of spacing t_max/32 steps over
    # them; 3788 is reached again near t = 9, a later crossing
    for k in (16, 1242, 3788, 8127, 100, 5000):
        res = O.min_time(S, x[k], O.Options(c_tau=2.0, warm="cont"))
        assert res.status == O.PT_OK, (k, res.status)
        assert res.T <= T0[k] * (1 + 1e-4), (k, res.T, T0[k])


# ------------------------------------------------------------------ read-out trajectory interior

def test_trajectory_interior_matches_impulse_march():
    """Every state of the read-out, not only the last, against an
    independent forward march: the quadrature form applies the control at
    node k as the impulse w_k B Qu u_k at physical time s_k and the state
    moves freely in between, so x_j = e^{(s_j - s_{j-1}) A} x_{j-1} + w_j B Qu u_j
    from x(0) = x0 (one matrix exponential per gap, no prefix sums)."""
    spec = random_system(4, 2, 16, "box", seed=12, t_max=3.0)
    S = O.System(spec.A, spec.B, spec.W, spec.c, np.diag([0.7, 1.3]), "box", 16, 3.0)
    x = np.array([0.5, -0.3, 0.2, 0.4])
    T = 1.37                        # off the grid: the extra node at tau = T is included
    pr = O.solve_value(S, x, T, O.Options(gap_tol=1e-9, max_iter=400000, c_tau=0.3))
    s, u, xs, p = O.readout(S, x, pr)
    w_by_s = {round(T - t, 12): wk for t, wk in zip(pr.tau, pr.w)}
    cur, s_prev = x.copy(), 0.0
    for j in range(len(s)):
        cur = expm((s[j] - s_prev) * spec.A) @ cur
        wk = w_by_s[round(s[j], 12)]
        cur = cur + wk * spec.B @ (u[j] if wk > 0 else np.zeros(2))
        s_prev = s[j]
        np.testing.assert_allclose(xs[j], cur, atol=1e-11)
    np.testing.assert_allclose(xs[-1], O.terminal_state(S, pr.xf, pr.Ks, pr.y), atol=1e-11)


def test_trajectory_converges_to_the_held_control_ode():
    """As N grows the read-out approaches the exact solution of the ODE under
    the same control held constant on each node's panel (zero-order hold,
    integrated with the augmented-matrix exponential).  With the left rule
    at T = t_max the node at physical time s_j closes the panel
    [s_j - h, s_j], so the held-control state at s_j is compared with the
    read-out state there; the gap is first order in h."""
    A = np.array([[0.0, 1.0], [0.0, 0.0]])
    B = np.array([[0.0], [1.0]])
    errs = []
    for N in (50, 200):
        S = O.System(A, B, 0.01 * np.eye(2), None, None, O.BOX, N, 2.0, O.LEFT)
        x = np.array([0.6, 0.1])
        pr = O.solve_value(S, x, 2.0, O.Options(gap_tol=1e-10, max_iter=400000, c_tau=10.0))
        s, u, xs, p = O.readout(S, x, pr)
        h = 2.0 / N
        assert abs(s[0] - h) < 1e-12
        cur, err = x.copy(), 0.0
        for j in range(len(s)):
            Aug = np.zeros((3, 3))
            Aug[:2, :2] = A
            Aug[:2, 2] = (B @ u[j]).ravel()
            E = expm(h * Aug)
            cur = E[:2, :2] @ cur + E[:2, 2]          # state at s_j
            err = max(err, float(np.max(np.abs(cur - xs[j]))))
        errs.append(err)
    assert errs[1] < 0.5 * errs[0] and errs[1] < 0.05, errs


# ------------------------------------------------------------------ golden values against the oracle

def test_oracle_min_time_against_golden_time_to_origin():
    """The golden textbook times to the origin bound the oracle's minimum time
    to a disk of radius r around it: T_r <= T_0, and since every point of the
    disk reaches the origin within r + 2 sqrt(r + r^2/2),
    T_r >= T_0 - r - 2 sqrt(r + r^2/2); the discrete search adds at most the
    trapezoid error and its tolerance."""
    r = 0.02
    spec = double_integrator(r, 160, t_max=8.0)
    S = sysobj(spec)
    with open("tests/golden/double_integrator_origin.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    h = O.grid_step(S)
    for p, v, T0 in rows:
        res = O.min_time(S, np.array([float(p), float(v)]), O.Options(c_tau=30.0, warm="cont"))
        T0 = float(T0)
        assert res.status == O.PT_OK
        slack = 0.02 * h * h + 1e-4 * T0
        assert T0 - r - 2 * math.sqrt(r + r * r / 2) - slack <= res.T <= T0 + slack, (p, v, res.T, T0)
