"""FP64 CPU oracle for the primal-dual solution of the generalized Hopf formula.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP path.

Method: Kirchner, Hewer, Darbon, Osher, "A Primal-Dual Method for Optimal
Control and Trajectory Generation in High-Dimensional Systems" (arXiv
1712.08226).  Every function below is written plainly, one point at a time, in
float64, citing the passage it follows.

Problem (Sec. II-B, eqs. (8)-(13); Sec. III-A, eqs. (16)-(23)).
    dx/dt = A x + B u,  u in U = Qu * C with C the unit l2 ball or unit box.
    Target Omega = {x : (x-c)^T W^{-1} (x-c) <= 1}   (Sec. VI-A, eq. (34)).
    Terminal cost J(x) = 1/2 ((x-c)^T W^{-1} (x-c) - 1), negative inside Omega,
    positive outside, zero on its boundary (Sec. IV).  The paper's example uses
    twice this function; the zero level set, hence the minimum time, is the
    same.

Terminal-costate form.  Substituting p = e^{T A^T} lam in the quadrature form
of the generalized Hopf formula (eq. (18)) gives, with x_f = e^{T A} x0 and
time-to-go nodes tau_k with weights w_k,
    P(lam) = J*(lam) - <x_f, lam> + sum_k w_k sigma_C(K_k lam),
    K_k    = -Qu^T B^T e^{tau_k A^T}                     (eq. (20) in lam),
    phi_N(x0, T) = -min_lam P(lam).
J*(lam) = 1/2 lam^T W lam + <c, lam> + 1/2 is the conjugate of J (the ellipsoid
analogue of eq. (35)); sigma_C is the support function of C (the dual norm of
eq. (16)): the l2 norm for the l2 ball, the l1 norm for the box.  The
Fenchel dual of min P (Sec. III, the saddle form of eq. (14)) is
    D(y) = -J(x_f - sum_k K_k^T y_k),   y_k in w_k C         (eq. (22)),
so for every lam and every feasible y:  -P(lam) <= phi_N <= -D(y).  The point
x_f - K^T y is the terminal state reached under the piecewise-constant control
u_k = y_k / w_k.

Quadrature ("fixed time-to-go table", the reading used throughout this
project).  The table holds nodes tau_k = k h, k = 0..N-1, with
h = t_max/(N-1) (trapezoid rule) or h = t_max/N (left rule of eq. (17)).  A
probe at horizon T uses the nodes with tau_k <= T plus, for the trapezoid rule
and a horizon that is not a multiple of h, one extra node at tau = T.  At
T = t_max both rules reduce to the paper's layout with N equally spaced
samples; see ``nodes_and_weights``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.linalg import expm, eigvalsh, cho_factor, cho_solve

L2, BOX = "l2", "box"
TRAP, LEFT = "trap", "left"

# per-point status codes (same meaning as the C-ABI's, values chosen here)
PT_OK, PT_INSIDE, PT_UNREACH, PT_NOCONV, PT_NONFINITE = 0, 1, 2, 3, 4


@dataclass
class System:
    """One linear system with its control set, target and quadrature table."""
    A: np.ndarray
    B: np.ndarray
    W: np.ndarray
    c: np.ndarray | None = None
    Qu: np.ndarray | None = None
    uset: str = L2
    N: int = 100
    t_max: float = 10.0
    quad: str = TRAP

    def __post_init__(self):
        self.A = np.asarray(self.A, dtype=np.float64)
        self.B = np.asarray(self.B, dtype=np.float64)
        if self.B.ndim == 1:
            self.B = self.B[:, None]
        self.W = np.asarray(self.W, dtype=np.float64)
        n, m = self.B.shape
        self.c = np.zeros(n) if self.c is None else np.asarray(self.c, dtype=np.float64)
        self.Qu = np.eye(m) if self.Qu is None else np.asarray(self.Qu, dtype=np.float64)
        self._Wchol = cho_factor(self.W)

    @property
    def n(self):
        return self.B.shape[0]

    @property
    def m(self):
        return self.B.shape[1]


@dataclass
class Options:
    """Solver settings.  Paper: theta = 1 and sigma = 1/(tau ||K||^2)
    (Sec. VI); here sigma carries a 0.999 factor so that the strict step
    condition tau sigma ||K||^2 < 1 of Sec. III holds, and tau = c_tau/||K||.

    Minimum-time search (Sec. IV: T* is the smallest horizon with
    phi(x0, T) = 0): the table nodes nearest to t_max (j / scan)^2,
    j = 1..scan, are probed in ascending order until the first certified
    reach; the search then refines the cell between the last
    certified-unreachable scan horizon and that reach (bisection over the
    table nodes inside it, then bisection or the Newton hybrid of Sec. IV)."""
    c_tau: float = 1.0
    gap_tol: float = 1e-6
    t_rel_tol: float = 0.5e-4
    t_abs_tol_frac: float = 1e-6
    max_iter: int = 200000
    check_every: int = 25
    warm: str = "cold"          # "cold": lam0 = 0 at every probe; "cont": previous probe's iterate
    root: str = "bisect"        # "bisect": midpoint; "newton": Sec. IV hybrid Newton-bisection step
    newton_rho: float = 0.5     # hybrid: a probe also runs until gap <= rho |phi| (Newton accuracy)
    newton_after: int = 1       # hybrid: midpoint probes inside the cell before Newton steps start
    scan: int = 48              # scan horizons: table nodes nearest t_max (j/scan)^2, j = 1..scan
    steps: str = "fixed"        # "fixed": tau, sigma as above; "accel": Sec. III's accelerated
                                # variant for a strongly convex G; "precond": diagonal
                                # preconditioning (Sec. III-A); see pdhg_iteration


# ---------------------------------------------------------------- terminal data

def J(sys: System, x):
    """Terminal cost, quadratic and zero on the ellipsoid boundary (Sec. IV,
    Sec. VI-A eq. (34))."""
    d = np.asarray(x, dtype=np.float64) - sys.c
    return 0.5 * (d @ cho_solve(sys._Wchol, d) - 1.0)


def J_star(sys: System, lam):
    """Fenchel conjugate of J (eq. (7) applied to J): 1/2 lam^T W lam + <c,lam> + 1/2."""
    return 0.5 * lam @ sys.W @ lam + sys.c @ lam + 0.5


def support(v, uset):
    """sigma_C(v) = max_{u in C} <v,u>: the dual norm of Sec. III-A, eq. (16)."""
    return float(np.linalg.norm(v, 2)) if uset == L2 else float(np.sum(np.abs(v)))


def project(v, radius, uset):
    """Euclidean projection onto radius*C: the prox of the indicator F_i* of
    eq. (22) (Sec. VI-A gives the interval case: clamp to +-Delta t)."""
    v = np.asarray(v, dtype=np.float64)
    if radius <= 0.0:
        return np.zeros_like(v)
    if uset == L2:
        nv = np.linalg.norm(v)
        return v if nv <= radius else v * (radius / nv)
    return np.clip(v, -radius, radius)


# ---------------------------------------------------------------- quadrature

def grid_step(sys: System):
    return sys.t_max / (sys.N - 1) if sys.quad == TRAP else sys.t_max / sys.N


def split_horizon(sys: System, T):
    """T = M h + r with 0 <= r < h; a T within 1e-12 relative of a grid point
    snaps to it."""
    h = grid_step(sys)
    q = T / h
    qr = round(q)
    if abs(q - qr) <= 1e-12 * max(1.0, q):
        return int(qr), 0.0
    M = int(math.floor(q))
    return M, T - M * h


def nodes_and_weights(sys: System, T):
    """Time-to-go nodes and quadrature weights for horizon T.

    Returns (tau, w, partial) where tau[k], w[k] list the nodes in the order
    table nodes 0..M (ascending tau) then, if present, the extra node at
    tau = T; ``partial`` tells whether the last entry is that extra node.

    Trapezoid: composite trapezoid on [0, M h] plus one trapezoid panel on
    [M h, T].  Left rule: each panel [k h, (k+1) h] (and [M h, T]) uses its
    node of smaller time-to-go, which is the paper's left Riemann sum with
    t_i = i dt (eq. (17)) read in time-to-go.
    """
    h = grid_step(sys)
    if T <= 0.0:
        return np.zeros(0), np.zeros(0), False
    M, r = split_horizon(sys, T)
    if sys.quad == TRAP:
        M = min(M, sys.N - 1)
        tau = [k * h for k in range(M + 1)]
        w = [0.0] * (M + 1)
        for k in range(M):              # panels [k h, (k+1) h]
            w[k] += 0.5 * h
            w[k + 1] += 0.5 * h
        partial = r > 0.0
        if partial:                     # panel [M h, T]
            w[M] += 0.5 * r
            tau.append(T)
            w.append(0.5 * r)
        return np.array(tau), np.array(w), partial
    # left rule
    tau = [k * h for k in range(M)]
    w = [h] * M
    if r > 0.0:
        tau.append(M * h)
        w.append(r)
    return np.array(tau), np.array(w), False


def K_blocks(sys: System, tau):
    """K_k = -Qu^T B^T e^{tau_k A^T} for every node (eq. (20), lam form); each
    block is m x n and is computed by a direct matrix exponential.  Returned
    as an array of shape (nodes, m, n)."""
    Ks = np.zeros((len(tau), sys.m, sys.n))
    for k, t in enumerate(tau):
        Ks[k] = -(expm(t * sys.A) @ sys.B @ sys.Qu).T
    return Ks


def apply_K(Ks, lam):
    """(K lam)_k = K_k lam, shape (nodes, m)."""
    return np.einsum("kij,j->ki", Ks, lam)


def apply_KT(Ks, y):
    """K^T y = sum_k K_k^T y_k, shape (n,)."""
    return np.einsum("kij,ki->j", Ks, y)


# ---------------------------------------------------------------- objectives

def primal_obj(sys, xf, Ks, w, lam):
    """P(lam) = J*(lam) - <x_f, lam> + sum_k w_k sigma_C(K_k lam): the function
    minimised in eq. (18), in the terminal costate."""
    Kl = apply_K(Ks, lam)
    s = sum(w[k] * support(Kl[k], sys.uset) for k in range(len(w)))
    return J_star(sys, lam) - xf @ lam + s


def terminal_state(sys, xf, Ks, y):
    """x_f - sum_k K_k^T y_k: the terminal state under u_k = y_k / w_k."""
    if len(Ks) == 0:
        return xf.copy()
    return xf - apply_KT(Ks, y)


def dual_obj(sys, xf, Ks, y):
    """D(y) = -J(x_f - K^T y) for feasible y (Fenchel dual of eq. (18))."""
    return -J(sys, terminal_state(sys, xf, Ks, y))


def op_norm_bound(sys, Ks, partial):
    """Upper bound L >= ||K||: exact on the table nodes, plus the Frobenius
    norm of the extra node's block when present."""
    if len(Ks) == 0:
        return 0.0
    table = Ks[:-1] if partial else Ks
    S = np.zeros((sys.n, sys.n))
    for k in range(len(table)):
        S += table[k].T @ table[k]
    L2sq = float(eigvalsh(S)[-1]) if len(table) else 0.0
    if partial:
        L2sq += float(np.sum(Ks[-1] ** 2))
    return math.sqrt(max(L2sq, 0.0))


# ---------------------------------------------------------------- PDHG

@dataclass
class Probe:
    """State and result of one Hopf solve at a fixed horizon T."""
    T: float
    tau: np.ndarray
    w: np.ndarray
    partial: bool
    Ks: list
    xf: np.ndarray
    L: float
    tau_p: float
    sigma_d: float
    lam: np.ndarray
    lam_bar: np.ndarray
    y: np.ndarray
    iters: int = 0
    P: float = math.inf
    D: float = -math.inf
    tight: bool = False          # run to the hybrid's relative accuracy as well as the sign
    history: list = field(default_factory=list)
    steps: str = "fixed"         # step rule (Options.steps)
    gamma: float = 0.0           # "accel": strong-convexity modulus of G, lambda_min(W)
    tau_vec: np.ndarray | None = None    # "precond": per-component primal steps
    sig_node: np.ndarray | None = None   # "precond": per-node dual steps

    @property
    def phi_lo(self):
        return -self.P

    @property
    def phi_hi(self):
        return -self.D

    def gap_n(self):
        return (self.P - self.D) / max(1.0, abs(self.D))


def make_probe(sys: System, x0, T, opt: Options, lam0=None, y0=None):
    """Set up one solve: nodes, weights, K, x_f = e^{T A} x0 (eq. (9)), step
    sizes, and the starting point (lam0 = 0 unless given)."""
    tau, w, partial = nodes_and_weights(sys, T)
    Ks = K_blocks(sys, tau)
    xf = expm(T * sys.A) @ np.asarray(x0, dtype=np.float64)
    L = op_norm_bound(sys, Ks, partial)
    if L > 0.0:
        tau_p = opt.c_tau / L
        sigma_d = 0.999 / (tau_p * L * L)
    else:
        tau_p, sigma_d = 1.0, 0.0
    lam = np.zeros(sys.n) if lam0 is None else np.array(lam0, dtype=np.float64)
    y = np.zeros((len(tau), sys.m))
    gamma, tau_vec, sig_node = 0.0, None, None
    if opt.steps == "accel":
        gamma = float(eigvalsh(sys.W)[0])
    elif opt.steps == "precond" and len(tau):
        # Pock-Chambolle diagonal steps with alpha = 1, the ratio c_tau moved
        # between the two sides: tau_i = c_tau / sum_r |K_ri|, and for node k
        # the smallest 1 / (c_tau sum_i |K_ri|) over its rows r, so that the
        # projection onto w_k C stays Euclidean (a smaller step per row keeps
        # the convergence condition)
        Kall = np.vstack(Ks)
        col = np.abs(Kall).sum(axis=0)
        tau_vec = np.where(col > 0.0, opt.c_tau / np.where(col > 0.0, col, 1.0), opt.c_tau)
        sig_node = np.array([0.999 / (opt.c_tau * max(np.abs(Kk).sum(axis=1).max(), 1e-300)) for Kk in Ks])
    if y0 is not None:
        # table nodes keep their rows, re-projected onto the new weights; the
        # extra node at tau = T starts from zero
        ntab = len(tau) - (1 if partial else 0)
        for k in range(min(ntab, y0.shape[0])):
            y[k] = project(y0[k], w[k], sys.uset)
    return Probe(T, tau, w, partial, Ks, xf, L, tau_p, sigma_d, lam, lam.copy(), y, steps=opt.steps,
                 gamma=gamma, tau_vec=tau_vec, sig_node=sig_node)


def pdhg_iteration(sys: System, pr: Probe):
    """One Chambolle-Pock step, Sec. III eq. (15) with theta = 1:
      y   <- prox_{sigma F*}(y + sigma K lam_bar)    (blockwise projection, eq. (23))
      lam+ <- prox_{tau G}(lam - tau K^T y)           (G = J* - <x_f,.>)
      lam_bar <- lam+ + (lam+ - lam).
    The prox of G solves (I + tau W) lam+ = lam - tau K^T y + tau (x_f - c),
    the terminal-costate form of eq. (37).

    The variants Sec. III names (Options.steps): "accel", the accelerated
    step for a G that is strongly convex with modulus gamma (here
    lambda_min(W)): theta = 1 / sqrt(1 + 2 gamma tau), then tau <- theta tau,
    sigma <- sigma / theta and lam_bar <- lam+ + theta (lam+ - lam);
    "precond", diagonal steps T (per component) and Sigma (per node): the
    dual step uses sigma_k on node k, the prox of G becomes
    (I + T W) lam+ = lam - T K^T y + T (x_f - c)."""
    if pr.steps == "precond":
        Kl = apply_K(pr.Ks, pr.lam_bar)
        v = pr.y + pr.sig_node[:, None] * Kl
        y_new = np.zeros_like(v)
        for k in range(len(pr.w)):
            y_new[k] = project(v[k], pr.w[k], sys.uset)
        g = apply_KT(pr.Ks, y_new)
        Tv = pr.tau_vec
        rhs = pr.lam - Tv * g + Tv * (pr.xf - sys.c)
        lam_new = np.linalg.solve(np.eye(sys.n) + Tv[:, None] * sys.W, rhs)
        pr.lam_bar = 2.0 * lam_new - pr.lam
        pr.lam = lam_new
        pr.y = y_new
        pr.iters += 1
        return
    v = pr.y + pr.sigma_d * apply_K(pr.Ks, pr.lam_bar)
    y_new = np.zeros_like(v)
    for k in range(len(pr.w)):
        y_new[k] = project(v[k], pr.w[k], sys.uset)
    g = apply_KT(pr.Ks, y_new)
    rhs = pr.lam - pr.tau_p * g + pr.tau_p * (pr.xf - sys.c)
    lam_new = np.linalg.solve(np.eye(sys.n) + pr.tau_p * sys.W, rhs)
    if pr.steps == "accel":
        theta = 1.0 / math.sqrt(1.0 + 2.0 * pr.gamma * pr.tau_p)
        pr.lam_bar = lam_new + theta * (lam_new - pr.lam)
        pr.tau_p *= theta
        pr.sigma_d /= theta
    else:
        pr.lam_bar = 2.0 * lam_new - pr.lam
    pr.lam = lam_new
    pr.y = y_new
    pr.iters += 1


def certify(sys: System, pr: Probe):
    """Primal value P(lam), dual value D(y) and the certified interval.  The
    primal bound takes the better of the iterate and lam = 0: P(0) = J*(0)
    = 1/2 = -min J (the terminal cost of Sec. IV is at least -1/2), which
    certifies phi >= -1/2 exactly when the target's centre is reachable."""
    pr.P = min(primal_obj(sys, pr.xf, pr.Ks, pr.w, pr.lam), 0.5)
    pr.D = dual_obj(sys, pr.xf, pr.Ks, pr.y)
    pr.history.append((pr.iters, pr.P, pr.D))


def solve_value(sys: System, x0, T, opt: Options = Options(), lam0=None, y0=None,
                pr: Probe | None = None):
    """phi_N(x0, T) to normalised gap (P-D)/max(1,|D|) <= gap_tol.

    Returns the probe; [phi_lo, phi_hi] = [-P, -D] brackets phi_N.  With no
    quadrature nodes (T = 0) the minimiser is lam = W^{-1}(x0 - c) and
    phi = J(x0) exactly (the initial condition of eq. (4))."""
    if pr is None:
        pr = make_probe(sys, x0, T, opt, lam0, y0)
    if len(pr.tau) == 0:
        pr.lam = cho_solve(sys._Wchol, pr.xf - sys.c)
        pr.P = primal_obj(sys, pr.xf, pr.Ks, pr.w, pr.lam)
        pr.D = dual_obj(sys, pr.xf, pr.Ks, pr.y)
        return pr
    while pr.iters < opt.max_iter:
        pdhg_iteration(sys, pr)
        if pr.iters % opt.check_every == 0:
            certify(sys, pr)
            if pr.gap_n() <= opt.gap_tol:
                break
    return pr


REACH, UNREACH, NOCONV = "reach", "unreach", "noconv"


def sign_decision(pr: Probe, opt: Options, tight: bool):
    """Sign of phi_N(x, T) from the probe's current certified interval
    [-P, -D] (Sec. IV: phi <= 0 means the target is reachable at T):
    -D <= 0 certifies reachable, -P > 0 certifies unreachable, and a gap
    below tolerance with neither counts as reachable (a zero of phi).  With
    `tight` (the Newton hybrid) the interval must also be narrower than
    newton_rho |phi| first.  Returns REACH, UNREACH or None (undecided)."""
    if pr.gap_n() <= opt.gap_tol:
        return UNREACH if -pr.P > 0.0 else REACH
    if tight and pr.P - pr.D > opt.newton_rho * 0.5 * abs(pr.P + pr.D):
        return None                     # the Newton step needs a tighter value
    if -pr.D <= 0.0:
        return REACH
    if -pr.P > 0.0:
        return UNREACH
    return None


def sign_probe(sys: System, pr: Probe, opt: Options, tight: bool = False):
    """Run a probe until the sign of phi_N is certified.  The starting point
    is certified before the first iteration (a probe continued from a nearby
    horizon often already decides), then every check_every iterations.
    Returns REACH, UNREACH or NOCONV."""
    if len(pr.tau) == 0:
        solve_value(sys, None, pr.T, opt, pr=pr)
        return REACH if -pr.D <= 0.0 else UNREACH
    certify(sys, pr)
    out = sign_decision(pr, opt, tight)
    if out is not None:
        return out
    while pr.iters < opt.max_iter:
        pdhg_iteration(sys, pr)
        if pr.iters % opt.check_every == 0:
            certify(sys, pr)
            out = sign_decision(pr, opt, tight)
            if out is not None:
                return out
    return NOCONV


@dataclass
class MinTimeResult:
    T: float
    status: int
    probes: int
    iters: int
    lam: np.ndarray
    y: np.ndarray | None
    P: float
    D: float
    gap_n: float
    lo: float
    hi: float
    final: Probe | None = None
    scan_probes: int = 0


def value_slope(sys: System, pr: Probe):
    """d phi_N / dT at the probe's horizon from its iterate (Sec. IV: the
    time derivative of the value is -H_x(p*, x0); with p = e^{T A^T} lam the
    two terms are <A x_f, lam> and the support function of the node at
    time-to-go T).  The node used is the one with the largest time-to-go and
    a positive weight (the last entry of the node list): for the left rule
    this is the exact one-sided derivative of the discretised value, for the
    trapezoid rule the derivative up to a term of order r = T - M h."""
    if len(pr.tau) == 0:
        return math.nan
    lam = pr.lam
    return float((sys.A @ pr.xf) @ lam - support(pr.Ks[-1] @ lam, sys.uset))


def last_node(sys: System):
    """Index K of the table node at t_max (K h = t_max)."""
    return sys.N - 1 if sys.quad == TRAP else sys.N


def node_horizon(sys: System, k: int):
    """Horizon of table node k (t_max exactly for the last node)."""
    return sys.t_max if k >= last_node(sys) else k * grid_step(sys)


def scan_nodes(sys: System, opt: Options):
    """The scan horizons as table nodes, ascending: node round(K (j/scan)^2)
    (at least 1) for j = 1..scan, repeats dropped, the last one K (t_max).
    The spacing grows like sqrt(t): a reachable interval of horizons near
    t = 0 is short (the control has acted only briefly), so the scan is
    finest there.  At a table node the quadrature needs no extra node."""
    K = last_node(sys)
    out = []
    for j in range(1, opt.scan + 1):
        if j == opt.scan:
            k = K
        else:
            s = j / opt.scan
            k = min(K, max(1, int(round(K * s * s))))
        if not out or k > out[-1]:
            out.append(k)
    return out


def node_floor(sys: System, t: float):
    """(k, exact): the table node at t when t is one (within 1e-12 relative,
    the snapping of split_horizon), else the node just below t."""
    q = t / grid_step(sys)
    qr = round(q)
    if abs(q - qr) <= 1e-12 * max(1.0, q):
        return int(qr), True
    return int(math.floor(q)), False


def inner_nodes(sys: System, lo: float, hi: float):
    """First and last table node strictly inside (lo, hi) (empty if ka > kb)."""
    ka = node_floor(sys, lo)[0] + 1
    kh, exact = node_floor(sys, hi)
    kb = min(kh - 1 if exact else kh, last_node(sys))
    return ka, kb


def search_tol(sys: System, opt: Options, hi: float):
    """Width at which the refinement stops (bracket [lo, hi], T = hi)."""
    return max(opt.t_rel_tol * hi, opt.t_abs_tol_frac * sys.t_max)


def newton_proposal(sys: System, opt: Options, pr: Probe, lo: float, hi: float):
    """The Sec. IV hybrid step from the probe just certified: T - phi/(d phi/dT)
    with phi the midpoint of its certified interval [-P, -D] and the slope of
    value_slope.  The probe is moved off that root estimate r towards the end
    of the bracket farther from it (above r when hi - r > r - lo, else below),
    by 0.4 of the stopping tolerance plus the estimate's own uncertainty, the
    interval's half-width (P - D)/2 divided by |slope|: it then lands on that
    side of the root, and with an accurate estimate the bracket closes on the
    next probe.  None when the slope is not negative or the probe would leave
    (lo, hi)."""
    s = value_slope(sys, pr)
    if not (s < 0.0) or not math.isfinite(s):
        return None
    r = pr.T - (-0.5 * (pr.P + pr.D)) / s
    shift = 0.4 * search_tol(sys, opt, hi) + 0.5 * (pr.P - pr.D) / abs(s)
    t = r + shift if hi - r > r - lo else r - shift
    return t if lo < t < hi else None


def min_time(sys: System, x0, opt: Options = Options(), lam0=None, t_bracket=None):
    """Minimum time to reach Omega (Sec. IV): the smallest horizon where phi_N
    falls to zero, searched with certified signs.

    1. Inside the target (J(x0) <= 0): T = 0.
    2. Scan: probe the scan nodes (scan_nodes) in ascending order until the
       first certified reach.  Every scan horizon certified unreachable,
       t_max included: T = +inf.  A reachable interval of horizons that lies
       strictly between two neighbouring scan horizons is not seen.
    3. Refine the cell [lo, hi] between the last certified-unreachable horizon
       (0 when the first scan horizon already reaches) and the first certified
       reach until hi - lo <= max(t_rel_tol hi, t_abs_tol_frac t_max):
         - a caller's hint t_bracket = (a, b) is probed first: b, then a,
           each only when it lies inside the current bracket;
         - then, while table nodes lie strictly inside the bracket, the
           middle one of them (bisection over the nodes);
         - then the midpoint, or with root = "newton" the hybrid step
           (newton_proposal) from a probe that ran to the Newton accuracy
           (probes between nodes, from the newton_after-th probe of the cell
           on); a Newton probe that leaves the bracket wider than half its
           width before the step forces the next probe to the midpoint, so
           the width halves at least every two probes (termination);
       a certified reach moves hi, a certified unreachable moves lo.
    4. T = hi; the solve at hi is continued to the gap tolerance.
    Probes start at lam = 0 (warm = "cold") or from the previous probe's
    iterate ("cont"); the first probe starts from lam0 when given."""
    x0 = np.asarray(x0, dtype=np.float64)
    if not np.all(np.isfinite(x0)):
        return MinTimeResult(math.nan, PT_NONFINITE, 0, 0, np.full(sys.n, math.nan), None,
                             math.nan, math.nan, math.nan, math.nan, math.nan)
    if J(sys, x0) <= 0.0:
        lam = cho_solve(sys._Wchol, x0 - sys.c)
        return MinTimeResult(0.0, PT_INSIDE, 0, 0, lam, None, J_star(sys, lam) - x0 @ lam,
                             -J(sys, x0), 0.0, 0.0, 0.0)
    probes, iters = 0, 0
    last = None

    def start(T, tight=False):
        nonlocal probes
        if last is None:
            pr = make_probe(sys, x0, T, opt, lam0)
        elif opt.warm == "cont":
            pr = make_probe(sys, x0, T, opt, last.lam, last.y)
        else:
            pr = make_probe(sys, x0, T, opt)
        pr.tight = tight
        probes += 1
        return pr

    # ---- scan for the first certified reach
    lo, hi = 0.0, math.inf
    nscan = 0
    for k in scan_nodes(sys, opt):
        T = node_horizon(sys, k)
        pr = start(T)
        out = sign_probe(sys, pr, opt)
        iters += pr.iters
        nscan += 1
        last = pr
        if out == NOCONV:
            return MinTimeResult(math.nan, PT_NOCONV, probes, iters, pr.lam, pr.y, pr.P, pr.D,
                                 pr.gap_n(), lo, T, pr, nscan)
        if out == REACH:
            hi = T
            break
        lo = T
    if not math.isfinite(hi):
        return MinTimeResult(math.inf, PT_UNREACH, probes, iters, last.lam, last.y, last.P, last.D,
                             last.gap_n(), lo, math.inf, last, nscan)

    # ---- refine the first cell
    hints = [] if t_bracket is None else [float(t_bracket[1]), float(t_bracket[0])]
    last_is_hi = True
    ncell = 0                 # probes inside the cell so far
    guard_w = None            # bracket width before the last Newton probe
    while hi - lo > search_tol(sys, opt, hi):
        nxt, newton, cont = 0.5 * (lo + hi), False, True
        while hints:
            t = hints.pop(0)
            if lo < t < hi:
                nxt = t
                break
        else:
            ka, kb = inner_nodes(sys, lo, hi)
            if ka <= kb:                      # table nodes inside: bisect over them
                nxt, cont = node_horizon(sys, (ka + kb) // 2), False
            elif opt.root == "newton" and last.tight and guard_w is None:
                t = newton_proposal(sys, opt, last, lo, hi)
                if t is not None:
                    nxt, newton = t, True
        width = hi - lo
        pr = start(nxt, tight=opt.root == "newton" and cont and ncell + 1 >= opt.newton_after)
        out = sign_probe(sys, pr, opt, pr.tight)
        iters += pr.iters
        ncell += 1
        if out == NOCONV:
            return MinTimeResult(math.nan, PT_NOCONV, probes, iters, pr.lam, pr.y, pr.P, pr.D,
                                 pr.gap_n(), lo, hi, pr, nscan)
        if out == REACH:
            hi, last_is_hi = nxt, True
        else:
            lo, last_is_hi = nxt, False
        last = pr
        if newton:
            guard_w = width if hi - lo > 0.5 * width else None
        else:
            guard_w = None

    # ---- the solve at T = hi to the gap tolerance
    if last_is_hi:
        fin = last
        before = fin.iters
    else:
        fin = start(hi)
        before = 0
    solve_value(sys, x0, hi, opt, pr=fin)
    iters += fin.iters - before
    st = PT_OK if fin.gap_n() <= opt.gap_tol else PT_NOCONV
    return MinTimeResult(hi, st, probes, iters, fin.lam, fin.y, fin.P, fin.D, fin.gap_n(),
                         lo, hi, fin, nscan)


def readout(sys: System, x0, pr: Probe):
    """Control, trajectory and costate from a solved probe.

    Control (Sec. IV, eq. (27)): at node k the control is u_k = Qu y_k / w_k,
    applied at physical time s_k = T - tau_k.  Trajectory (Sec. V,
    eq. (33)): the state after each node's contribution, marching forward in
    physical time, x(s_j) = e^{s_j A}(x0 + sum_{s_k <= s_j} w_k e^{-s_k A} B u_k);
    its last point equals the terminal state x_f - K^T y.  Costate:
    p* = e^{T A^T} lam* (the paper's minimiser, eq. (24)).
    Returns (s, u, xs, p_star) with rows sorted by increasing s."""
    x0 = np.asarray(x0, dtype=np.float64)
    T = pr.T
    order = np.argsort(-np.asarray(pr.tau), kind="stable")     # largest time-to-go first
    s = np.array([T - pr.tau[k] for k in order])
    u = np.array([sys.Qu @ pr.y[k] / pr.w[k] if pr.w[k] > 0 else np.zeros(sys.m)
                  for k in order]).reshape(len(order), sys.m)
    xs = []
    for j, k_j in enumerate(order):
        acc = x0.copy()
        for i in range(j + 1):
            k = order[i]
            acc = acc + pr.w[k] * expm(-s[i] * sys.A) @ sys.B @ u[i]
        xs.append(expm(s[j] * sys.A) @ acc)
    xs = np.array(xs).reshape(len(order), sys.n)
    p_star = expm(T * sys.A.T) @ pr.lam
    return s, u, xs, p_star


def hamiltonian_x(sys: System, p, x0):
    """H_x(p, x0) = -x0^T A^T p + sigma_C(-Qu^T B^T p) (Sec. IV), so that
    d phi / dT = -H_x(grad phi, x0)."""
    return -(x0 @ sys.A.T @ p) + support(-(sys.Qu.T @ sys.B.T @ p), sys.uset)
