"""Independent reference computations used to pin the oracle.

None of these share code with the oracle: they are brute-force, closed-form or
different-algorithm computations of quantities the oracle also produces.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm


# ---------------------------------------------------------------- double integrator

def di_time_to_origin(p, v):
    """Textbook minimum time of the double integrator (|u| <= 1) to the origin:
    one bang-bang switch on the curve p = -v|v|/2."""
    s = p + v * abs(v) / 2.0
    if s > 0:
        return v + 2.0 * math.sqrt(p + v * v / 2.0)
    if s < 0:
        return -v + 2.0 * math.sqrt(-p + v * v / 2.0)
    return abs(v)


def _di_endpoints(p0, v0, T, t1, s):
    """State at T under u = s on [0, t1], u = -s on [t1, T]."""
    t2 = T - t1
    p1 = p0 + v0 * t1 + 0.5 * s * t1 * t1
    v1 = v0 + s * t1
    p2 = p1 + v1 * t2 - 0.5 * s * t2 * t2
    v2 = v1 - s * t2
    return p2, v2


def di_dist_to_reach_set(p0, v0, T, ngrid=4001):
    """Distance from the origin to the boundary of the exact-time reachable
    set R(T); the boundary is traced by one-switch bang-bang controls.  Valid
    as the distance to R(T) while the origin is outside R(T), i.e. for
    T < time to origin."""
    best = math.inf
    for s in (1.0, -1.0):
        t1 = np.linspace(0.0, T, ngrid)
        p2, v2 = _di_endpoints(p0, v0, T, t1, s)
        d = np.hypot(p2, v2)
        i = int(np.argmin(d))
        lo, hi = t1[max(i - 1, 0)], t1[min(i + 1, ngrid - 1)]
        for _ in range(80):                       # golden-section refinement
            a = hi - (hi - lo) / 1.618033988749895
            b = lo + (hi - lo) / 1.618033988749895
            da = np.hypot(*_di_endpoints(p0, v0, T, a, s))
            db = np.hypot(*_di_endpoints(p0, v0, T, b, s))
            if da < db:
                hi = b
            else:
                lo = a
        best = min(best, float(np.hypot(*_di_endpoints(p0, v0, T, 0.5 * (lo + hi), s))), float(d[i]))
    return best


def di_min_time_ball(p0, v0, r):
    """Continuous-time minimum time of the double integrator to the disk of
    radius r at the origin, by scanning T up to the time to the origin and
    bisecting the first crossing of dist(0, R(T)) = r."""
    if math.hypot(p0, v0) <= r:
        return 0.0
    Tor = di_time_to_origin(p0, v0)
    Ts = np.linspace(0.0, Tor, 801)
    prev = 0.0
    for T in Ts[1:]:
        if di_dist_to_reach_set(p0, v0, T, 801) <= r:
            lo, hi = prev, T
            for _ in range(50):
                mid = 0.5 * (lo + hi)
                if di_dist_to_reach_set(p0, v0, mid) <= r:
                    hi = mid
                else:
                    lo = mid
            return hi
        prev = T
    return Tor


def di_grid_min_time(L=2.5, n=251, dt=0.02, tmax=8.0):
    """Semi-Lagrangian dynamic programming for the double integrator's
    minimum-time function on an n x n grid over [-L, L]^2 (target: disk of
    radius 0.1 at the origin).  T(x) = min_u dt + T(x + exact step under u),
    with u in {-1, 0, 1}, bilinear interpolation, iterated to a fixed point."""
    g = np.linspace(-L, L, n)
    dx = g[1] - g[0]
    P, V = np.meshgrid(g, g, indexing="ij")
    inside = np.hypot(P, V) <= 0.1
    BIG = 1e3                      # finite "not reached yet" so interpolation stays finite
    Tg = np.where(inside, 0.0, BIG)

    def interp(Tgrid, p, v):
        fi = (p + L) / dx
        fj = (v + L) / dx
        i0 = np.floor(fi).astype(int)
        j0 = np.floor(fj).astype(int)
        ok = (i0 >= 0) & (j0 >= 0) & (i0 < n - 1) & (j0 < n - 1)
        i0c = np.clip(i0, 0, n - 2)
        j0c = np.clip(j0, 0, n - 2)
        a = fi - i0c
        b = fj - j0c
        val = ((1 - a) * (1 - b) * Tgrid[i0c, j0c] + a * (1 - b) * Tgrid[i0c + 1, j0c]
               + (1 - a) * b * Tgrid[i0c, j0c + 1] + a * b * Tgrid[i0c + 1, j0c + 1])
        return np.where(ok, val, BIG)

    for _ in range(int(tmax / dt) + 50):
        best = np.full_like(Tg, BIG)
        for u in (-1.0, 0.0, 1.0):
            pn = P + V * dt + 0.5 * u * dt * dt
            vn = V + u * dt
            best = np.minimum(best, dt + interp(Tg, pn, vn))
        new = np.where(inside, 0.0, np.minimum(best, BIG))
        if np.max(np.abs(new - Tg)) < 1e-12:
            Tg = new
            break
        Tg = new
    return g, np.where(Tg >= 0.5 * BIG, np.inf, Tg)


def grid_lookup(g, Tg, p, v):
    dx = g[1] - g[0]
    i = int(round((p - g[0]) / dx))
    j = int(round((v - g[0]) / dx))
    return float(Tg[i, j])


# ---------------------------------------------------------------- independent primal solve

def primal_fista(A, B, W, c, Qu, uset, x0, T, tau, w, iters=30000):
    """Minimise J(e^{TA} x0 + sum_k w_k e^{tau_k A} B Qu u_k) over u_k in C by
    accelerated projected gradient (FISTA with restart): the primal problem
    whose optimal value is phi_N by Fenchel-Rockafellar duality.  Uses scipy's
    expm directly; shares nothing with the oracle's primal-dual iteration."""
    n, m = B.shape
    Winv = np.linalg.inv(W)
    G = np.stack([wk * (expm(t * A) @ B @ Qu) for t, wk in zip(tau, w)])   # (K, n, m)
    xf = expm(T * A) @ x0

    def terminal(u):
        return xf + np.einsum("knm,km->n", G, u)

    def f(u):
        d = terminal(u) - c
        return 0.5 * (d @ Winv @ d - 1.0)

    def grad(u):
        gx = Winv @ (terminal(u) - c)
        return np.einsum("knm,n->km", G, gx)

    def proj(u):
        if uset == "l2":
            nr = np.linalg.norm(u, axis=1, keepdims=True)
            return u / np.maximum(1.0, nr)
        return np.clip(u, -1.0, 1.0)

    Gm = G.transpose(1, 0, 2).reshape(n, -1)
    Lf = np.linalg.norm(Gm, 2) ** 2 * np.linalg.eigvalsh(Winv)[-1]
    u = np.zeros((len(tau), m))
    z = u.copy()
    t = 1.0
    fu = f(u)
    for _ in range(iters):
        un = proj(z - grad(z) / Lf)
        fn = f(un)
        if fn > fu:                     # restart
            z = u.copy()
            t = 1.0
            continue
        tn = 0.5 * (1 + math.sqrt(1 + 4 * t * t))
        z = un + ((t - 1) / tn) * (un - u)
        u, fu, t = un, fn, tn
    return fu, u
