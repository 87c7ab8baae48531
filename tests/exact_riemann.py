"""Exact solution of the 1D Euler Riemann problem (textbook two-shock/rarefaction wave curves solved
by Newton's method on the star pressure), used as an independent pin of the oracle's Sod run."""
import math

import numpy as np


def _f(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:
        f = 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(L, R, gamma=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, gamma)
        fr, dfr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, x, t, x0=0.5, gamma=1.4):
    """(rho, u, p) at positions x and time t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3, len(x)))
    for n, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + g1) / (g1 * ps / pl + 1), us, ps)
            else:  # left rarefaction
                als = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                if s <= ul - al:
                    w = (rl, ul, pl)
                elif s >= us - als:
                    w = (rl * (ps / pl) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * (ul - s))
                    u = 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s)
                    rho = rl * (c / al) ** (2 / (gamma - 1))
                    w = (rho, u, pl * (c / al) ** (2 * gamma / (gamma - 1)))
        else:
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + g1) / (g1 * ps / pr + 1), us, ps)
            else:
                ars = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                if s >= ur + ar:
                    w = (rr, ur, pr)
                elif s <= us + ars:
                    w = (rr * (ps / pr) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) * (ar - (gamma - 1) / 2 * (ur - s))
                    u = 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s)
                    rho = rr * (c / ar) ** (2 / (gamma - 1))
                    w = (rho, u, pr * (c / ar) ** (2 * gamma / (gamma - 1)))
        out[:, n] = w
    return out


def cell_averages(L, R, n, t, x0=0.5, gamma=1.4, sub=64):
    """Cell averages of rho on [0,1] with n cells (sub-sampled midpoint rule)."""
    xs = ((np.arange(n * sub) + 0.5) / (n * sub))
    w = sample(L, R, xs, t, x0, gamma)
    return w.reshape(3, n, sub).mean(axis=2)
