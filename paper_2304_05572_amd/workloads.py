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

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_NOSLIP, BC_PRESCRIBED = 0, 1, 2, 3, 4
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


def advection_3d(n: int, t: float = 0.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(pi (x + y + z - 3 t)), U = V = W = 1, p = 1 on [0, 2]^3: exact cell averages,
    W[c][k][j][i] with c in (rho, rho U, rho V, rho W, rho E)."""
    h = 2.0 / n
    xc = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    s = _sinc(np.pi * h / 2)
    rho = 1.0 + 0.2 * np.sin(np.pi * (X + Y + Z - 3.0 * t)) * s ** 3
    return prim_to_cons3(rho, np.ones_like(rho), np.ones_like(rho), np.ones_like(rho), np.ones_like(rho), gamma)


def prim_to_cons3(rho, u, v, w, p, gamma=GAMMA):
    rho = np.asarray(rho, np.float64)
    E = np.asarray(p, np.float64) / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def octants_3d(nx: int, ny: int, nz: int, seed: int = 0, wiggle: float = 0.0, gamma=GAMMA):
    """Eight constant states (rho, p in [0.5, 1.5], each velocity component in [-0.3, 0.3]) on the octants of
    the unit cube split at its centre, times 1 + wiggle * (a smooth seeded product of sines) in rho and p:
    planar discontinuities meeting at a point, smooth regions in between. W[c][k][j][i]."""
    rng = np.random.default_rng(seed)
    zc, yc, xc = ((np.arange(n) + 0.5) / n for n in (nz, ny, nx))
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    code = (X >= 0.5).astype(int) * 4 + (Y >= 0.5).astype(int) * 2 + (Z >= 0.5).astype(int)
    rho, p = rng.uniform(0.5, 1.5, 8)[code], rng.uniform(0.5, 1.5, 8)[code]
    vel = [rng.uniform(-0.3, 0.3, 8)[code] for _ in range(3)]
    ph = rng.uniform(0.0, 2.0 * np.pi, 3)
    bump = np.sin(2 * np.pi * X + ph[0]) * np.sin(2 * np.pi * Y + ph[1]) * np.sin(2 * np.pi * Z + ph[2])
    return prim_to_cons3(rho * (1.0 + wiggle * bump), *vel, p * (1.0 + wiggle * bump), gamma)


def embed_2d_in_3d(W2, nz: int, axis: int = 2):
    """A 2D state W2[c][j][i] (c in rho, rho U, rho V, rho E) as a 3D state uniform along `axis`: axis 2 keeps
    (x, y) -> (x, y); axis 0 maps (x, y) -> (y, z); axis 1 maps (x, y) -> (z, x). Returns W3[c][k][j][i]."""
    rho, mu, mv, E = W2
    zero = np.zeros_like(rho)
    if axis == 2:   # uniform in z: W3[c][k][j][i] = W2[c][j][i]
        comps = [rho, mu, mv, zero, E]
        return np.stack([np.broadcast_to(q[None, :, :], (nz,) + rho.shape) for q in comps]).copy()
    if axis == 0:   # uniform in x: 2D x -> y, 2D y -> z: W3[c][k][j][i] = W2[c][k][j]
        comps = [rho, zero, mu, mv, E]
        return np.stack([np.broadcast_to(q[:, :, None], rho.shape + (nz,)) for q in comps]).copy()
    # uniform in y: 2D x -> z, 2D y -> x: W3[c][k][j][i] = W2[c][i][k]
    comps = [rho, mv, zero, mu, E]
    return np.stack([np.broadcast_to(q.T[:, None, :], (rho.shape[1], nz, rho.shape[0])) for q in comps]).copy()


# ------------------------------------------------------------------ shock tubes
def sod_1d(n: int, gamma=GAMMA):
    """Sod: (1, 0, 1) for x < 0.5, (0.125, 0, 0.1) for x > 0.5 on [0, 1] (x = 0.5 is a face for even n)."""
    xc = (np.arange(n) + 0.5) / n
    left = xc < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return prim_to_cons(rho, np.zeros(n), None, p, gamma, dim=1)


def shu_osher_1d(n: int = 400, gamma=GAMMA):
    """Shu-Osher shock / entropy-wave interaction (Sec. 3.2(b)) on [0, 10]: (3.857134, 2.629369, 10.33333)
    for x < 1, (1 + 0.2 sin(5 x), 0, 1) beyond, as values at the cell centres (x = 1 is a face for n
    divisible by 10)."""
    xc = (np.arange(n) + 0.5) * (10.0 / n)
    left = xc < 1.0
    rho = np.where(left, 3.857134, 1.0 + 0.2 * np.sin(5.0 * xc))
    u = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.33333, 1.0)
    return prim_to_cons(rho, u, None, p, gamma, dim=1)


def blast_wave_1d(n: int = 400, gamma=GAMMA):
    """Woodward-Colella interacting blast waves (Sec. 3.2(c)) on [0, 1]: rho = 1, U = 0 and p = 1000 for
    x < 0.1, 0.01 between, 100 for x > 0.9 (both jumps on faces for n divisible by 10)."""
    xc = (np.arange(n) + 0.5) / n
    p = np.where(xc < 0.1, 1000.0, np.where(xc < 0.9, 0.01, 100.0))
    return prim_to_cons(np.ones(n), np.zeros(n), None, p, gamma, dim=1)


def viscous_shock_tube(nx: int, ny: int, gamma=GAMMA):
    """(120, 0, 0, 120/gamma) for x < 0.5 and (1.2, 0, 0, 1.2/gamma) for x > 0.5 on [0,1]x[0,0.5]."""
    xc = (np.arange(nx) + 0.5) / nx
    X = np.broadcast_to(xc, (ny, nx))
    left = X < 0.5
    rho = np.where(left, 120.0, 1.2)
    p = np.where(left, 120.0 / gamma, 1.2 / gamma)
    z = np.zeros_like(rho)
    return prim_to_cons(rho, z, z, p, gamma)


# ------------------------------------------------------------------ double Mach reflection (Sec. 3.5)
DMR_POST = (8.0, 4.125 * math.sqrt(3.0), -4.125, 116.5)  # (rho, U, V, p) behind the Mach 10 shock
DMR_PRE = (1.4, 0.0, 0.0, 1.0)                            # (rho, U, V, p) ahead of it
DMR_X0 = 1.0 / 6.0                                        # the shock meets the wall at (1/6, 0) at t = 0
DMR_SHOCK_SPEED = 10.0                                    # Mach 10 into gas with sound speed 1


def _cons_tuple(state, gamma=GAMMA):
    rho, u, v, p = (float(x) for x in state)
    return (rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v))


def dmr_shock_x(y, t):
    """x where the 60-degree Mach 10 shock crosses height y at time t: the line through (1/6, 0) moving
    along its normal (cos 30, -sin 30) at speed 10, i.e. along x at 10 / cos 30 = 20 / sqrt 3."""
    return DMR_X0 + (np.asarray(y) + 2.0 * DMR_SHOCK_SPEED * np.asarray(t)) / math.sqrt(3.0)


def _shock_line_side(post, pre):
    """Prescribed-side data (plain dict) for a y-side that follows the exact moving shock: state `post`
    where x < 1/6 + y / sqrt 3 + (20 / sqrt 3) t, else `pre`."""
    r3 = math.sqrt(3.0)
    return dict(a=post, b=pre, s0=DMR_X0, sn=1.0 / r3, st=2.0 * DMR_SHOCK_SPEED / r3, rest=BC_PRESCRIBED)


def double_mach(nx: int = 960, ny: int = 240, walls: bool = True, cfl: float = 0.8):
    """Double Mach reflection on [0,4]x[0,1] (Sec. 3.5): cell centres behind the shock line take the
    post-shock state, the others the pre-shock state. Returns (W0, problem keywords). Boundaries: the
    post-shock state enters on the left, zero gradient on the right, the top follows the exact moving
    shock, and the bottom holds the post-shock state for x < 1/6 and is a slip wall beyond. With
    walls=False the bottom also follows the exact moving shock: the exact solution is then the
    translating oblique shock itself. The scheme as the paper states it produces a non-physical Gauss-point
    state at the wall corner in the first step, so the problem enables the first-order fallbacks. cfl: the
    paper's 0.8 by default; with these fallbacks the 960 x 240 run reaches t = 0.2 at 0.8 and at 0.5 (the
    value the paper gives for the classic WENO5 GKS in this case)."""
    post, pre = _cons_tuple(DMR_POST), _cons_tuple(DMR_PRE)
    xc = 4.0 * (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    behind = X < dmr_shock_x(Y, 0.0)
    W = np.stack([np.where(behind, post[c], pre[c]) for c in range(4)])
    bottom = (dict(a=post, b=post, s0=DMR_X0, sn=0.0, st=0.0, rest=BC_REFLECT) if walls
              else _shock_line_side(post, pre))
    kw = dict(dim=2, nx=nx, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0,
              bc=(BC_PRESCRIBED, BC_OUTFLOW, BC_PRESCRIBED, BC_PRESCRIBED),
              bcd=(dict(a=post, b=post, s0=math.inf, sn=0.0, st=0.0, rest=BC_PRESCRIBED), None, bottom,
                   _shock_line_side(post, pre)),
              cfl=cfl, c1=0.0, c2=1.0, positivity=1)
    return W, kw


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


def _shock_velocity_jump(p, rho_k, p_k, gamma=GAMMA):
    """Velocity change across a shock of pressure p > p_k running into the state (rho_k, p_k), and the
    post-shock density (Rankine-Hugoniot)."""
    A = 2.0 / ((gamma + 1.0) * rho_k)
    B = (gamma - 1.0) / (gamma + 1.0) * p_k
    f = (p - p_k) * math.sqrt(A / (p + B))
    r = p / p_k
    g = (gamma - 1.0) / (gamma + 1.0)
    return f, rho_k * (r + g) / (g * r + 1.0)


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


def _edges_nontrivial(states, min_ratio=1.25, min_dv=0.15):
    """Every edge (1-2, 2-3, 3-4, 4-1) carries a visible jump."""
    for a, b in ((0, 1), (1, 2), (2, 3), (3, 0)):
        ra, ua, va, pa = states[a]
        rb, ub, vb, pb = states[b]
        rr = max(ra, rb) / min(ra, rb)
        pr = max(pa, pb) / min(pa, pb)
        if rr < min_ratio and pr < min_ratio and abs(ua - ub) < min_dv and abs(va - vb) < min_dv:
            return False
    return True


def _symmetry(states, k):
    """Apply one of the dihedral symmetries of the square to a quadrant configuration (quadrants
    1 = upper right, 2 = upper left, 3 = lower left, 4 = lower right)."""
    s1, s2, s3, s4 = [list(x) for x in states]
    if k & 1:  # mirror x -> 1 - x: 1 <-> 2, 3 <-> 4, u -> -u
        s1, s2, s3, s4 = s2, s1, s4, s3
        for s in (s1, s2, s3, s4):
            s[1] = -s[1]
    if k & 2:  # mirror y -> 1 - y: 1 <-> 4, 2 <-> 3, v -> -v
        s1, s2, s3, s4 = s4, s3, s2, s1
        for s in (s1, s2, s3, s4):
            s[2] = -s[2]
    if k & 4:  # transpose x <-> y: 2 <-> 4, u <-> v
        s1, s2, s3, s4 = s1, s4, s3, s2
        for s in (s1, s2, s3, s4):
            s[1], s[2] = s[2], s[1]
    return [tuple(s) for s in (s1, s2, s3, s4)]


def random_quadrant_states(rng: np.random.Generator, max_tries: int = 1000):
    """Four quadrant states with exactly one elementary wave (shock, rarefaction or contact) on each
    edge, built exactly in one of four families and then turned by a random symmetry of the square:
      R4   four rarefactions: one isentrope, c3 = c2 + c4 - c1, velocities from the Riemann invariants
      J4   four contacts (slip lines): common pressure, u1 = u2, u3 = u4, v2 = v3, v4 = v1
      J2R2 contacts on the vertical edges, rarefactions on the horizontal ones
      J2S2 contacts on the vertical edges, shocks on the horizontal ones (Rankine-Hugoniot)
    Draws outside rho in [0.1, 1.5], p in [0.03, 1.5], |u|, |v| <= 1.2, or with a near-trivial edge, are
    rejected. Quadrants: 1 = (x>.5, y>.5), 2 = (x<.5, y>.5), 3 = (x<.5, y<.5), 4 = (x>.5, y<.5)."""
    g = GAMMA
    k2 = 2.0 / (g - 1.0)
    lo_r, hi_r = RANGES["rho"]
    lo_p, hi_p = RANGES["p"]
    vm = RANGES["vel"]
    for _ in range(max_tries):
        fam = int(rng.integers(4))
        if fam == 0:  # R4
            rho1, p1 = rng.uniform(0.5, hi_r), rng.uniform(0.4, hi_p)
            u1, v1 = rng.uniform(-0.6, 0.6, 2)
            c1 = math.sqrt(g * p1 / rho1)
            c2, c4 = c1 * rng.uniform(0.7, 0.95, 2)
            c3 = c2 + c4 - c1
            if c3 <= 0.3 * c1:
                continue
            ent = p1 / rho1 ** g

            def st(c, u, v):
                p = p1 * (c / c1) ** (2.0 * g / (g - 1.0))
                return ((p / ent) ** (1.0 / g), u, v, p)

            u2 = u1 + k2 * (c2 - c1)
            v4 = v1 + k2 * (c4 - c1)
            states = [(rho1, u1, v1, p1), st(c2, u2, v1), st(c3, u2, v4), st(c4, u1, v4)]
        elif fam == 1:  # J4
            p = rng.uniform(lo_p, hi_p)
            r = rng.uniform(lo_r, hi_r, 4)
            u12, u34, v14, v23 = rng.uniform(-vm, vm, 4)
            states = [(r[0], u12, v14, p), (r[1], u12, v23, p), (r[2], u34, v23, p), (r[3], u34, v14, p)]
        elif fam == 2:  # J2R2
            pa = rng.uniform(0.3, hi_p)
            pb = pa * rng.uniform(0.2, 0.7)
            r1, r2 = rng.uniform(0.3, hi_r, 2)
            u = rng.uniform(-vm, vm)
            v1, v2 = rng.uniform(-vm, vm, 2)
            f = (pb / pa) ** (1.0 / g)
            r4, r3 = r1 * f, r2 * f
            c = lambda r, p: math.sqrt(g * p / r)
            v4 = v1 + k2 * (c(r4, pb) - c(r1, pa))
            v3 = v2 + k2 * (c(r3, pb) - c(r2, pa))
            states = [(r1, u, v1, pa), (r2, u, v2, pa), (r3, u, v3, pb), (r4, u, v4, pb)]
        else:  # J2S2
            pa = rng.uniform(lo_p, 0.8)
            pb = pa * rng.uniform(1.5, 4.0)
            r1, r2 = rng.uniform(lo_r, 1.0, 2)
            u = rng.uniform(-vm, vm)
            v1, v2 = rng.uniform(-vm, vm, 2)
            f1, r4 = _shock_velocity_jump(pb, r1, pa)
            f2, r3 = _shock_velocity_jump(pb, r2, pa)
            states = [(r1, u, v1, pa), (r2, u, v2, pa), (r3, u, v2 + f2, pb), (r4, u, v1 + f1, pb)]
        states = _symmetry(states, int(rng.integers(8)))
        if _in_range(states) and _edges_nontrivial(states):
            return [tuple(float(a) for a in s) for s in states]
    raise RuntimeError("no admissible quadrant configuration drawn")


def riemann_2d(n: int, seed: int = 0, ny: int | None = None):
    """Seeded four-quadrant Riemann problem on [0,1]^2 with n x n (or n x ny) cells."""
    rng = np.random.default_rng(seed)
    states = random_quadrant_states(rng)
    return quadrants(n, ny or n, states), states


def batch_sizes(nprob: int = 64, seed: int = 0, lo: int = 128, hi: int = 1024):
    """Uneven square grid sizes N_b drawn uniformly from {lo..hi}."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi + 1, size=nprob)]
