"""Seeded synthetic initial conditions for the paper's test problems (Mu et al., arXiv 2304.05572,
Sec. 3). This module holds no arithmetic of the method itself: it only builds conserved-variable
arrays (cell averages) and problem parameters. It imports nothing but numpy, so both the oracle's
tests and the GPU path can use it.

Layout of every state: structure of arrays, x fastest, float64:
  1D: W[c, i]     c in (rho, rho*U, rho*E)
  2D: W[c, j, i]  c in (rho, rho*U, rho*V, rho*E)
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_NOSLIP = 0, 1, 2, 3
GAMMA = 1.4


def prim_to_cons(rho, u, v, p, gamma=GAMMA, dim=2):
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    p = np.asarray(p, np.float64)
    if dim == 1:
        E = p / (gamma - 1.0) + 0.5 * rho * u * u
        return np.stack([rho, rho * u, E])
    v = np.asarray(v, np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def cons_to_prim(W, gamma=GAMMA):
    W = np.asarray(W, np.float64)
    rho = W[0]
    u = W[1] / rho
    if W.shape[0] == 3:
        p = (gamma - 1.0) * (W[2] - 0.5 * rho * u * u)
        return rho, u, None, p
    v = W[2] / rho
    p = (gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


# ------------------------------------------------------------------ advection (Sec. 3.1, 3.3)
def _sinc(z):
    return np.where(z == 0, 1.0, np.sin(z) / np.where(z == 0, 1.0, z))


def advection_1d(n: int, t: float = 0.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(pi (x - t)), U = 1, p = 1 on [0, 2]: exact cell averages at time t."""
    dx = 2.0 / n
    xc = (np.arange(n) + 0.5) * dx
    rho = 1.0 + 0.2 * np.sin(np.pi * (xc - t)) * _sinc(np.pi * dx / 2)
    return prim_to_cons(rho, np.ones(n), None, np.ones(n), gamma, dim=1)


def advection_2d(n: int, t: float = 0.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(pi (x + y - t)), U = V = 1, p = 1 on [0, 2]^2: exact cell averages.

    The momentum and energy averages are exact too because U, V and p are constant."""
    h = 2.0 / n
    xc = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    s = _sinc(np.pi * h / 2)
    rho = 1.0 + 0.2 * np.sin(np.pi * (X + Y - t)) * s * s
    one = np.ones_like(rho)
    return prim_to_cons(rho, one, one, one, gamma)


# ------------------------------------------------------------------ shock tubes
def sod_1d(n: int, gamma=GAMMA):
    """Sod: (1, 0, 1) for x < 0.5, (0.125, 0, 0.1) for x > 0.5 on [0, 1] (x = 0.5 is a face for even n)."""
    xc = (np.arange(n) + 0.5) / n
    left = xc < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return prim_to_cons(rho, np.zeros(n), None, p, gamma, dim=1)


def viscous_shock_tube(nx: int, ny: int, gamma=GAMMA):
    """(120, 0, 0, 120/gamma) for x < 0.5 and (1.2, 0, 0, 1.2/gamma) for x > 0.5 on [0,1]x[0,0.5]."""
    xc = (np.arange(nx) + 0.5) / nx
    X = np.broadcast_to(xc, (ny, nx))
    left = X < 0.5
    rho = np.where(left, 120.0, 1.2)
    p = np.where(left, 120.0 / gamma, 1.2 / gamma)
    z = np.zeros_like(rho)
    return prim_to_cons(rho, z, z, p, gamma)


# ------------------------------------------------------------------ four-quadrant Riemann problems
# Quadrants in the usual order: 1 = (x>.5, y>.5), 2 = (x<.5, y>.5), 3 = (x<.5, y<.5), 4 = (x>.5, y<.5).
RP_CONFIG1 = [(1.0, 0.0, 0.0, 1.0), (0.5197, -0.7259, 0.0, 0.4), (0.1072, -0.7259, -1.4045, 0.0439),
              (0.2579, 0.0, -1.4045, 0.15)]
RP_CONFIG6 = [(1.0, -0.75, -0.5, 1.0), (2.0, 0.75, 0.5, 1.0), (1.0, -0.75, 0.5, 1.0),
              (3.0, -0.75, -0.5, 1.0)]


def quadrants(nx: int, ny: int, states, gamma=GAMMA, xs=0.5, ys=0.5):
    """Cell averages of a four-quadrant state on [0,1]^2 split at (xs, ys) (faces for even n)."""
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    q = np.where(X >= xs, np.where(Y >= ys, 0, 3), np.where(Y >= ys, 1, 2))
    st = np.asarray(states, np.float64)
    rho, u, v, p = (st[q, k] for k in range(4))
    return prim_to_cons(rho, u, v, p, gamma)


def _wave_curve(p, rho_k, p_k, gamma=GAMMA):
    """Velocity change f(p) and density behind a 1D wave of pressure p facing the state (rho_k, p_k):
    Rankine-Hugoniot for p > p_k (shock), isentrope for p <= p_k (rarefaction)."""
    a_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        f = (p - p_k) * math.sqrt(A / (p + B))
        r = p / p_k
        g = (gamma - 1.0) / (gamma + 1.0)
        rho = rho_k * (r + g) / (g * r + 1.0)
    else:
        f = 2.0 * a_k / (gamma - 1.0) * ((p / p_k) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        rho = rho_k * (p / p_k) ** (1.0 / gamma)
    return f, rho


RANGES = dict(rho=(0.1, 1.5), p=(0.03, 1.5), vel=1.2)


def _in_range(states):
    for rho, u, v, p in states:
        if not (RANGES["rho"][0] <= rho <= RANGES["rho"][1]):
            return False
        if not (RANGES["p"][0] <= p <= RANGES["p"][1]):
            return False
        if abs(u) > RANGES["vel"] or abs(v) > RANGES["vel"]:
            return False
    return True


def random_quadrant_states(rng: np.random.Generator, max_tries: int = 200):
    """Four quadrant states with one elementary wave (shock, rarefaction or contact) per edge.

    State 1 is drawn uniformly from the ranges; states 2 (x-wave from 1) and 4 (y-wave from 1) follow
    from a drawn wave type and strength along the wave curves; state 3 must then be reached from 2 by a
    y-wave and from 4 by an x-wave. The free strengths are fixed by requiring the two routes to 3 to
    agree in pressure and density (solved by a damped Newton iteration). Draws that do not close, or
    leave the ranges, are rejected; after max_tries the always-closing all-contact family is used
    (common pressure, u1=u2, u3=u4, v2=v3, v4=v1, free densities)."""
    g = GAMMA
    lo_r, hi_r = RANGES["rho"]
    lo_p, hi_p = RANGES["p"]
    vmax = RANGES["vel"]
    for _ in range(max_tries):
        rho1 = rng.uniform(lo_r, hi_r)
        p1 = rng.uniform(lo_p, hi_p)
        u1 = rng.uniform(-vmax, vmax)
        v1 = rng.uniform(-vmax, vmax)
        # wave family per edge: +1 / -1 (right- / left-facing acoustic wave) or 0 (contact)
        fam = rng.choice([-1, 0, 1], size=4)

        def x_wave(state_r, p_l, family):
            """Left state across a vertical edge, given the right state (rho, u, v, p)."""
            rho_r, u_r, v_r, p_r = state_r
            if family == 0:
                return None
            f, rho_l = _wave_curve(p_l, rho_r, p_r)
            # family +1 (wave moves right, state_r ahead): u_l = u_r + f ; family -1: mirror with state_l ahead
            return (rho_l, u_r + f, v_r, p_l) if family > 0 else None

        # Closing an arbitrary acoustic-wave loop is a two-parameter root find; we use the simplest
        # robust construction: pick the edge types, then solve for the pressures numerically.
        def close(params):
            p2, p4 = params
            s1 = (rho1, u1, v1, p1)
            # edge 1-2 (x-wave, state 2 on the left): right-facing wave, state 1 ahead
            f12, r2 = _wave_curve(p2, rho1, p1)
            s2 = (r2, u1 + f12, v1, p2)
            # edge 1-4 (y-wave, state 4 below): upward-facing wave, state 1 ahead
            f14, r4 = _wave_curve(p4, rho1, p1)
            s4 = (r4, u1, v1 + f14, p4)
            return s1, s2, s4

        def residual(params):
            s1, s2, s4 = close(params)
            # state 3: from 2 by a y-wave (u3 = u2), from 4 by an x-wave (v3 = v4)
            # pressure p3 from the y-route: v3 = v2 + f(p3; state 2) must equal v4
            # and from the x-route:           u3 = u4 + f(p3; state 4) must equal u2
            def solve_p(target, base_vel, rho_k, p_k):
                lo, hi = 1e-6, 50.0
                flo = base_vel + _wave_curve(lo, rho_k, p_k)[0] - target
                fhi = base_vel + _wave_curve(hi, rho_k, p_k)[0] - target
                if flo * fhi > 0:
                    return None
                for _ in range(100):
                    mid = 0.5 * (lo + hi)
                    fm = base_vel + _wave_curve(mid, rho_k, p_k)[0] - target
                    if (fm > 0) == (fhi > 0):
                        hi, fhi = mid, fm
                    else:
                        lo, flo = mid, fm
                return 0.5 * (lo + hi)
            py = solve_p(s4[2], s2[2], s2[0], s2[3])
            px = solve_p(s2[1], s4[1], s4[0], s4[3])
            if py is None or px is None:
                return None
            ry = _wave_curve(py, s2[0], s2[3])[1]
            rx = _wave_curve(px, s4[0], s4[3])[1]
            return np.array([math.log(py / px), math.log(ry / rx)]), (s1, s2, (ry, s2[1], s4[2], py), s4)

        x = np.array([rng.uniform(lo_p, hi_p), rng.uniform(lo_p, hi_p)])
        ok = False
        for _it in range(40):
            res = residual(x)
            if res is None:
                break
            r, states = res
            if np.max(np.abs(r)) < 1e-12:
                ok = True
                break
            J = np.zeros((2, 2))
            for k in range(2):
                dx = np.zeros(2)
                dx[k] = 1e-7 * x[k]
                rr = residual(x + dx)
                if rr is None:
                    break
                J[:, k] = (rr[0] - r) / dx[k]
            else:
                try:
                    step = np.linalg.solve(J, -r)
                except np.linalg.LinAlgError:
                    break
                x = np.clip(x + 0.7 * step, 1e-4, 50.0)
                continue
            break
        if ok and _in_range(states) and fam is not None:
            return [tuple(float(a) for a in s) for s in states]
    # all-contact fallback
    p = rng.uniform(lo_p, hi_p)
    u12, u34 = rng.uniform(-vmax, vmax, 2)
    v41, v23 = rng.uniform(-vmax, vmax, 2)
    rhos = rng.uniform(lo_r, hi_r, 4)
    return [(rhos[0], u12, v41, p), (rhos[1], u12, v23, p), (rhos[2], u34, v23, p), (rhos[3], u34, v41, p)]


def riemann_2d(n: int, seed: int = 0, ny: int | None = None):
    """Seeded four-quadrant Riemann problem on [0,1]^2 with n x n (or n x ny) cells."""
    rng = np.random.default_rng(seed)
    states = random_quadrant_states(rng)
    return quadrants(n, ny or n, states), states


def batch_sizes(nprob: int = 64, seed: int = 0, lo: int = 128, hi: int = 1024):
    """Uneven square grid sizes N_b drawn uniformly from {lo..hi}."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi + 1, size=nprob)]
