"""Planted mistakes in the oracle must be caught by its pins.

Each case patches one function of the oracle (on the CPU, for the duration
of the test only) with a plausible error -- a dropped term, a wrong sign or
exponent, a transposed operand, a wrong norm, the search rule that looks at
t_max only -- and checks that at least one of a fixed set of quick pins
fails.  The unpatched oracle passes all of them (the pin modules run them
as ordinary tests)."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import hopf_oracle as O
from oracle import mlp_oracle as M
from tests import test_oracle_pins as P
from tests import test_mlp_oracle_pins as PM


def quick_pins():
    return [
        lambda: P.test_K_rows_double_integrator_closed_form(),
        lambda: P.test_trapezoid_weights_on_grid_and_exactness(),
        lambda: P.test_value_l2_ball_closed_form([0.9, -0.4, 0.2], 0.3),
        lambda: P.test_value_box_closed_form([0.9, -0.4], 0.3),
        lambda: P.test_min_time_l2_ball_closed_form([0.9, -0.4, 0.2]),
        lambda: P.test_min_time_is_the_first_crossing("bisect"),
        lambda: P.test_strong_duality_against_independent_primal_solve("l2", O.TRAP, 1.37, 0.0),
        lambda: P.test_planted_point_value_bound(),
        lambda: P.test_trajectory_interior_matches_impulse_march(),
        lambda: PM.test_adam_bias_correction_over_several_steps(),
    ]


def some_pin_fails():
    for pin in quick_pins():
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError, ValueError, FloatingPointError):
            return True
    return False


def _support_wrong_norm(v, uset):
    return float(np.sum(np.abs(v))) if uset == O.L2 else float(np.linalg.norm(v, 2))


def _K_transposed(sys, tau):
    Ks = np.zeros((len(tau), sys.m, sys.n))
    for k, t in enumerate(tau):
        Ks[k] = -(expm(t * sys.A.T) @ sys.B @ sys.Qu).T
    return Ks


def _primal_no_weights(sys, xf, Ks, w, lam):
    Kl = O.apply_K(Ks, lam)
    return O.J_star(sys, lam) - xf @ lam + sum(O.support(Kl[k], sys.uset) for k in range(len(w)))


def _J_with_W(sys, x):
    d = np.asarray(x, dtype=np.float64) - sys.c
    return 0.5 * (d @ sys.W @ d - 1.0)


def _scan_t_max_only(sys, opt):
    return [O.last_node(sys)]


def _trap_full_end_weight(sys, T):
    tau, w, partial = _ORIG_NW(sys, T)
    if sys.quad == O.TRAP and len(w):
        w = w.copy()
        w[0] = 2 * w[0]
    return tau, w, partial


def _adam_first_power(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    return _ORIG_ADAM(theta, g, m, v, 1, lr, b1, b2, eps)


def _xf_wrong_sign(sys, x0, T, opt, lam0=None, y0=None):
    pr = _ORIG_MP(sys, x0, T, opt, lam0, y0)
    pr.xf = expm(-T * sys.A) @ np.asarray(x0, dtype=np.float64)
    return pr


_ORIG_NW = O.nodes_and_weights
_ORIG_MP = O.make_probe
_ORIG_ADAM = M.adam_step

MUTATIONS = {
    "support function of the wrong norm": (O, "support", _support_wrong_norm),
    "transposed matrix exponential in K": (O, "K_blocks", _K_transposed),
    "quadrature weights dropped from P": (O, "primal_obj", _primal_no_weights),
    "W in place of W^-1 in the terminal cost": (O, "J", _J_with_W),
    "search that looks at t_max only": (O, "scan_nodes", _scan_t_max_only),
    "full trapezoid weight at tau = 0": (O, "nodes_and_weights", _trap_full_end_weight),
    "Adam bias correction with power 1": (M, "adam_step", _adam_first_power),
    "free motion e^{-TA} x0 in place of e^{TA} x0": (O, "make_probe", _xf_wrong_sign),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    mod, attr, fn = MUTATIONS[name]
    monkeypatch.setattr(mod, attr, fn)
    assert some_pin_fails(), f"no pin caught: {name}"
