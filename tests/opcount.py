"""Algorithmic operation count of the scheme's hot path, per Gauss point (test and measurement
infrastructure; no kernel code).

The formulas of the method evaluated once in plain Python on a counting scalar type: the normal
reconstruction of an interface row (Sec. 2.3.1 Step 5, linear, or WENO-AO in characteristic variables),
the tangential reconstruction at a Gauss point (Sec. 2.3.3), the equilibrium state of Eq. (equ46)-(equ47),
and the gas-kinetic flux of Eq. (equ10) with its time integrals over [0, dt] and [0, dt/2] turned into F
and dF/dt (Sec. 2.2). Every +, -, * and / on a value is one operation (a fused multiply-add is two);
sqrt, exp and erfc are counted apart (transcendental calls); comparisons and branches are not counted.
F and dF/dt are formed term by term from the five time-integral coefficients, the algebraically
identical form of (4 F(dt/2) - F(dt)) / dt and 4 (F(dt) - 2 F(dt/2)) / dt^2 that needs one flux assembly.

The same functions compute real values, which tests/test_opcount.py checks against the oracle's
interface fluxes (so the counted formulas are the scheme's), and bench.py's per-Gauss-point constants
are checked against the counts here.
"""
from collections import Counter
import math

COUNTS = Counter()


def _v(x):
    return x.v if isinstance(x, Num) else x


class Num:
    """A float that counts the arithmetic done on it."""
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v)

    def _op(self, kind, r):
        COUNTS[kind] += 1
        return Num(r)

    def __add__(self, o):
        return self._op("add", self.v + _v(o))

    __radd__ = __add__

    def __sub__(self, o):
        return self._op("add", self.v - _v(o))

    def __rsub__(self, o):
        return self._op("add", _v(o) - self.v)

    def __mul__(self, o):
        return self._op("mul", self.v * _v(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        return self._op("div", self.v / _v(o))

    def __rtruediv__(self, o):
        return self._op("div", _v(o) / self.v)

    def __neg__(self):
        return Num(-self.v)  # a sign change is not arithmetic

    def __abs__(self):
        return Num(abs(self.v))

    def __lt__(self, o):
        return self.v < _v(o)

    def __gt__(self, o):
        return self.v > _v(o)

    def __float__(self):
        return self.v


def sqrt(x):
    COUNTS["sqrt"] += 1
    return Num(math.sqrt(_v(x)))


def exp(x):
    COUNTS["exp"] += 1
    return Num(math.exp(_v(x)))


def erfc(x):
    COUNTS["erfc"] += 1
    return Num(math.erfc(_v(x)))


def flops():
    return COUNTS["add"] + COUNTS["mul"] + COUNTS["div"]


# ------------------------------------------------------------------ reconstruction (Sec. 2.3.1, 2.3.3)
S3 = math.sqrt(3.0)
ETA = 1.0 / (2.0 * S3)


def quartic_face(q, side):
    """Linear fifth-order value at the cell face xi = +1/2 (side 0) or -1/2 (side 1) of the middle cell of
    q[0..4] (the printed Step-5 coefficients), and its xi-derivative."""
    if side == 1:
        q = q[::-1]
    v = (2 * q[0] - 13 * q[1] + 47 * q[2] + 27 * q[3] - 3 * q[4]) / 60.0
    d = (q[1] - 15 * q[2] + 15 * q[3] - q[4]) / 12.0
    return v, (d if side == 0 else -d)


def quartic_gp(q, gp):
    """Value and xi-derivative of the cell-average quartic of q[0..4] at xi = -eta (gp 0) or +eta (gp 1)."""
    a = q if gp == 1 else q[::-1]
    c = (-1 / 4320 + 7 * S3 / 432, 1 / 1080 - 25 * S3 / 216, 719 / 720, 1 / 1080 + 25 * S3 / 216,
         -1 / 4320 - 7 * S3 / 432)
    e = (1 / 12 - S3 / 54, -2 / 3 + 13 * S3 / 54, -4 * S3 / 9, 2 / 3 + 13 * S3 / 54, -1 / 12 - S3 / 54)
    v = c[0] * a[0] + c[1] * a[1] + c[2] * a[2] + c[3] * a[3] + c[4] * a[4]
    d = e[0] * a[0] + e[1] * a[1] + e[2] * a[2] + e[3] * a[3] + e[4] * a[4]
    return v, (d if gp == 1 else -d)


def _subpolys(q, ev):
    """Values and derivatives of the three quadratics and the quartic at evaluation point ev (0/1: face
    +1/2 / -1/2; 2/3: Gauss point -eta / +eta)."""
    if ev in (0, 1):
        qq = q if ev == 0 else q[::-1]
        pv = [qq[0] / 3 - 7 * qq[1] / 6 + 11 * qq[2] / 6, -qq[1] / 6 + 5 * qq[2] / 6 + qq[3] / 3,
              qq[2] / 3 + 5 * qq[3] / 6 - qq[4] / 6]
        pd = [qq[0] - 3 * qq[1] + 2 * qq[2], qq[3] - qq[2], qq[3] - qq[2]]
        v3, d3 = quartic_face(q, ev)
        if ev == 1:
            pv = pv[::-1]
            pd = [-x for x in pd[::-1]]
        return pv + [v3], pd + [d3]
    gp = ev - 2
    a = q if gp == 1 else q[::-1]
    pv = [S3 / 12 * a[0] - S3 / 3 * a[1] + (1 + S3 / 4) * a[2], -S3 / 12 * a[1] + a[2] + S3 / 12 * a[3],
          (1 - S3 / 4) * a[2] + S3 / 3 * a[3] - S3 / 12 * a[4]]
    pd = [(0.5 + S3 / 6) * a[0] + (-2 - S3 / 3) * a[1] + (1.5 + S3 / 6) * a[2],
          (-0.5 + S3 / 6) * a[1] + (-S3 / 3) * a[2] + (0.5 + S3 / 6) * a[3],
          (-1.5 + S3 / 6) * a[2] + (2 - S3 / 3) * a[3] + (-0.5 + S3 / 6) * a[4]]
    v3, d3 = quartic_gp(q, gp)
    if gp == 0:
        pv = pv[::-1]
        pd = [-x for x in pd[::-1]]
    return pv + [v3], pd + [d3]


def _betas(q):
    b = []
    for s in range(3):
        x0, x1, x2 = q[s], q[s + 1], q[s + 2]
        d = x0 - 2 * x1 + x2
        e = (x0 - 4 * x1 + 3 * x2) if s == 0 else (x0 - x2) if s == 1 else (3 * x0 - 4 * x1 + x2)
        b.append(13 / 12 * d * d + 0.25 * e * e)
    u1 = (11 * (q[0] - q[4]) + 82 * (q[3] - q[1])) / 120
    u2 = (-3 * (q[0] + q[4]) + 40 * (q[1] + q[3]) - 74 * q[2]) / 56
    u3 = (-q[0] + 2 * q[1] - 2 * q[3] + q[4]) / 12
    u4 = (q[0] - 4 * q[1] + 6 * q[2] - 4 * q[3] + q[4]) / 24
    s1, s2 = u1 + 0.1 * u3, u2 + 123 / 455 * u4
    b.append(s1 * s1 + 13 / 3 * s2 * s2 + 781 / 20 * u3 * u3 + 1421461 / 2275 * u4 * u4)
    return b


def ao_scalar(q, ev, ghi=0.85, glo=0.85, eps=1e-8):
    """WENO-AO(5,3) value and derivative of one component (Sec. 2.3.1)."""
    beta = _betas(q)
    pv, pd = _subpolys(q, ev)
    g3, g0, g1 = ghi, (1 - ghi) * (1 - glo) / 2, (1 - ghi) * glo
    gam = (g0, g1, g0, g3)
    dl = (abs(beta[3] - beta[0]) + abs(beta[3] - beta[1]) + abs(beta[3] - beta[2])) / 3
    w = [gam[k] * (1 + dl / (beta[k] + eps)) for k in range(4)]
    tot = w[0] + w[1] + w[2] + w[3]
    wb = [x / tot for x in w]
    v = wb[3] / g3 * (pv[3] - g0 * pv[0] - g1 * pv[1] - g0 * pv[2]) + wb[0] * pv[0] + wb[1] * pv[1] + wb[2] * pv[2]
    d = wb[3] / g3 * (pd[3] - g0 * pd[0] - g1 * pd[1] - g0 * pd[2]) + wb[0] * pd[0] + wb[1] * pd[1] + wb[2] * pd[2]
    return v, d


def char_basis(w, gamma, slot):
    """Eigenvectors of the 2D Euler flux Jacobian along momentum slot `slot` (1 or 2) at state w: the
    right ones R (columns u_n - c, entropy, shear, u_n + c) and the left ones L = R^-1 in closed form."""
    t = 3 - slot
    u = [None, w[1] / w[0], w[2] / w[0]]
    q2 = u[1] * u[1] + u[2] * u[2]
    p = (gamma - 1) * (w[3] - 0.5 * w[0] * q2)
    c = sqrt(gamma * p / w[0])
    H = (w[3] + p) / w[0]
    b1 = (gamma - 1) / (c * c)
    b2 = 0.5 * q2 * b1
    un, ut = u[slot], u[t]
    R = [[1, 1, 0, 1], [0] * 4, [0] * 4, [H - un * c, 0.5 * q2, ut, H + un * c]]
    R[slot] = [un - c, un, 0, un + c]
    R[t] = [ut, ut, 1, ut]
    L = [[0] * 4 for _ in range(4)]
    L[0][0], L[0][slot], L[0][t], L[0][3] = 0.5 * (b2 + un / c), -0.5 * (b1 * un + 1 / c), -0.5 * b1 * ut, 0.5 * b1
    L[1][0], L[1][slot], L[1][t], L[1][3] = 1 - b2, b1 * un, b1 * ut, -b1
    L[2][0], L[2][slot], L[2][t], L[2][3] = -ut, 0, 1, 0
    L[3][0], L[3][slot], L[3][t], L[3][3] = 0.5 * (b2 - un / c), -0.5 * (b1 * un - 1 / c), -0.5 * b1 * ut, 0.5 * b1
    return R, L


def _dot4(row, x):
    acc = None
    for a, b in zip(row, x):
        if isinstance(a, (int, float)) and a == 0:
            continue
        term = b if (isinstance(a, (int, float)) and a == 1) else a * b
        acc = term if acc is None else acc + term
    return acc if acc is not None else 0.0


def ao_vector(rows, R, L, ev):
    """WENO-AO of four conserved components in characteristic variables: rows[r][c], r = 0..4."""
    ch = [[_dot4(L[k], rows[r]) for k in range(4)] for r in range(5)]
    cv, cd = [], []
    for k in range(4):
        v, d = ao_scalar([ch[r][k] for r in range(5)], ev)
        cv.append(v)
        cd.append(d)
    return [_dot4(R[c], cv) for c in range(4)], [_dot4(R[c], cd) for c in range(4)]


# ------------------------------------------------------------------ kinetic part (Sec. 2.1)
class Maxwellian:
    """Moments of the normalised Maxwellian with velocity (U, V) and lam = rho / (2 p): <u^n>, full line
    (half = 0) or half line (half = +1: u > 0, -1: u < 0), <v^n>, <xi^2>, <xi^4> (K internal dof)."""

    def __init__(self, w, gamma, K):
        self.rho = w[0]
        self.U = w[1] / w[0]
        self.V = w[2] / w[0]
        self.p = (gamma - 1) * (w[3] - 0.5 * w[0] * (self.U * self.U + self.V * self.V))
        self.lam = w[0] / (2 * self.p)
        self.K = K

    def moments(self, half):
        U, lam = self.U, self.lam
        s = 1 / (2 * lam)
        if half == 0:
            Mu = [1.0, U]
        else:
            sl = sqrt(lam)
            m0 = 0.5 * erfc(-half * sl * U)
            ex = exp(-lam * U * U) / (2 * math.sqrt(math.pi) * sl)
            Mu = [m0, U * m0 + half * ex]
        for n in range(5):
            Mu.append(U * Mu[n + 1] + (n + 1) * s * Mu[n])
        Mv = [1.0, self.V]
        for n in range(4):
            Mv.append(self.V * Mv[n + 1] + (n + 1) * s * Mv[n])
        self.Mu, self.Mv = Mu, Mv
        self.X1 = self.K * s
        self.X2 = self.K * (self.K + 2) * s * s

    def G(self, n, m):
        a, b = self.Mu[n], self.Mv[m]
        if isinstance(b, float) and b == 1.0:
            return a
        if isinstance(a, float) and a == 1.0:
            return b
        return a * b

    def mom_a(self, N, M, a):
        """<u^N v^M a psi> for a = a0 + a1 u + a2 v + a3 (u^2 + v^2 + xi^2) / 2."""
        G = self.G

        def SS(n, m):
            return 0.5 * (G(n + 2, m) + G(n, m + 2) + G(n, m) * self.X1)
        S00, S10, S01 = SS(N, M), SS(N + 1, M), SS(N, M + 1)
        TT = 0.25 * (G(N + 4, M) + G(N, M + 4) + G(N, M) * self.X2 +
                     2 * (G(N + 2, M + 2) + (G(N + 2, M) + G(N, M + 2)) * self.X1))
        return [a[0] * G(N, M) + a[1] * G(N + 1, M) + a[2] * G(N, M + 1) + a[3] * S00,
                a[0] * G(N + 1, M) + a[1] * G(N + 2, M) + a[2] * G(N + 1, M + 1) + a[3] * S10,
                a[0] * G(N, M + 1) + a[1] * G(N + 1, M + 1) + a[2] * G(N, M + 2) + a[3] * S01,
                a[0] * S00 + a[1] * S10 + a[2] * S01 + a[3] * TT]

    def mom_psi(self, N, M):
        G = self.G
        return [G(N, M), G(N + 1, M), G(N, M + 1), 0.5 * (G(N + 2, M) + G(N, M + 2) + G(N, M) * self.X1)]

    def solve(self, b):
        """a with <a psi> = b (closed form of the 4 x 4 moment system)."""
        U, V, l = self.U, self.V, self.lam
        q2 = U * U + V * V
        ni = (self.K + 2) / (2 * l)
        a3 = 4 * l * l / (self.K + 2) * (2 * b[3] - 2 * U * b[1] - 2 * V * b[2] + (q2 - ni) * b[0])
        a2 = 2 * l * (b[2] - V * b[0]) - V * a3
        a1 = 2 * l * (b[1] - U * b[0]) - U * a3
        a0 = b[0] - U * a1 - V * a2 - 0.5 * a3 * (q2 + ni)
        return [a0, a1, a2, a3]


def time_coeffs(d, tau):
    """Integrals over [0, d] of the five coefficient functions of Eq. (equ10) (closed forms, d/tau >= 1)."""
    e = exp(-(d / tau))
    return [d - tau * (1 - e), 2 * tau * tau - tau * d - tau * (d + 2 * tau) * e,
            0.5 * d * d - tau * d + tau * tau * (1 - e), tau * (1 - e), 2 * tau * tau - tau * (2 * tau + d) * e]


def gp_flux(Wl, Wxl, Wyl, Wr, Wxr, Wyr, gamma, c1, c2, dt, wgt):
    """wgt times F and dF/dt at one Gauss point (frame slot 1 normal), Euler collision time."""
    K = (4 - 2 * gamma) / (gamma - 1)
    acc = {k: [0.0] * 4 for k in ("Wc", "Wxc", "Wyc", "M4a", "M4b", "M5")}
    p = []
    for side, (W, Wx, Wy) in enumerate(((Wl, Wxl, Wyl), (Wr, Wxr, Wyr))):
        g = Maxwellian(W, gamma, K)
        p.append(g.p)
        g.moments(0)
        ax = g.solve([Wx[c] / g.rho for c in range(4)])
        ay = g.solve([Wy[c] / g.rho for c in range(4)])
        t1, t2 = g.mom_a(1, 0, ax), g.mom_a(0, 1, ay)
        A = g.solve([-(t1[c] + t2[c]) for c in range(4)])
        g.moments(1 if side == 0 else -1)
        parts = {"Wc": g.mom_psi(0, 0), "Wxc": g.mom_a(0, 0, ax), "Wyc": g.mom_a(0, 0, ay),
                 "M4a": g.mom_psi(1, 0), "M4b": g.mom_a(1, 0, A)}
        m5a, m5b = g.mom_a(2, 0, ax), g.mom_a(1, 1, ay)
        parts["M5"] = [m5a[c] + m5b[c] for c in range(4)]
        for k, x in parts.items():
            acc[k] = [g.rho * x[c] if side == 0 else acc[k][c] + g.rho * x[c] for c in range(4)]
    tau = c1 * dt + c2 * abs(p[0] - p[1]) / (p[0] + p[1]) * dt
    Cd, Ch = time_coeffs(dt, tau), time_coeffs(dt / 2, tau)
    cf = [wgt * (4 * Ch[m] - Cd[m]) / dt for m in range(5)]
    cdd = [wgt * 4 * (Cd[m] - 2 * Ch[m]) / (dt * dt) for m in range(5)]
    F, dF = [0.0] * 4, [0.0] * 4

    def fold(M, a, b):
        for c in range(4):
            F[c] = F[c] + a * M[c]
            dF[c] = dF[c] + b * M[c]
    fold(acc["M4a"], cf[3], cdd[3])
    fold(acc["M4b"], -tau * cf[3], -tau * cdd[3])
    fold(acc["M5"], -cf[4], -cdd[4])
    g0 = Maxwellian(acc["Wc"], gamma, K)
    g0.moments(0)
    r0 = g0.rho
    fold([r0 * x for x in g0.mom_psi(1, 0)], cf[0], cdd[0])
    a0 = g0.solve([acc["Wxc"][c] / r0 for c in range(4)])
    b0 = g0.solve([acc["Wyc"][c] / r0 for c in range(4)])
    m1, m2 = g0.mom_a(1, 0, a0), g0.mom_a(0, 1, b0)
    A0 = g0.solve([-(m1[c] + m2[c]) for c in range(4)])
    u2a, uvb = g0.mom_a(2, 0, a0), g0.mom_a(1, 1, b0)
    fold([r0 * (u2a[c] + uvb[c]) for c in range(4)], cf[1], cdd[1])
    fold([r0 * x for x in g0.mom_a(1, 0, A0)], cf[2], cdd[2])
    return F, dF


# ------------------------------------------------------------------ one x-interface segment
def normal_row(cells, flag_l, flag_r, ih, gamma=1.4):
    """(W^l, W^l_x, W^r, W^r_x) of one interface from its six cells (frame components): linear per
    component, or WENO-AO in the characteristic variables of the two cells' mean for a flagged side."""
    out = [None] * 4
    if flag_l or flag_r:
        R, L = char_basis([0.5 * (cells[2][c] + cells[3][c]) for c in range(4)], gamma, 1)
    for side, flag in ((0, flag_l), (1, flag_r)):
        rows = cells[side:side + 5]
        if flag:
            v, d = ao_vector(rows, R, L, side)
            out[2 * side + 1] = [x * ih for x in d]
        elif side == 1 and not flag_l:  # both linear: the two sides' quartic slopes are the same formula
            v = [quartic_face([r[c] for r in rows], side)[0] for c in range(4)]
            out[3] = out[1]
        else:
            vd = [quartic_face([r[c] for r in rows], side) for c in range(4)]
            v = [x[0] for x in vd]
            out[2 * side + 1] = [x[1] * ih for x in vd]
        out[2 * side] = v
    return out


def tangential_side(lines_v, lines_x, gp, flag, iht, gamma=1.4):
    """Gauss-point value, tangential slope and normal-slope value of one side from its five line values."""
    if flag:
        R, L = char_basis(lines_v[2], gamma, 2)
        v, d = ao_vector(lines_v, R, L, 2 + gp)
        wx, _ = ao_vector(lines_x, R, L, 2 + gp)
        return v, [x * iht for x in d], wx
    v, d, wx = [], [], []
    for c in range(4):
        a, b = quartic_gp([r[c] for r in lines_v], gp)
        v.append(a)
        d.append(b * iht)
        wx.append(quartic_gp([r[c] for r in lines_x], gp)[0])
    return v, d, wx


def interface_flux(stencil, hx, hy, dt, flags_n=None, flags_t=None, gamma=1.4, c1=0.01, c2=1.0):
    """F and dF/dt of one x-interface segment from its 5 x 6 cells stencil[r][m][c] (rows j-2..j+2, cells
    i-3..i+2 of the interface between cells i-1 and i). flags_n[r] = (left, right) normal flags per row,
    flags_t = (left, right) tangential flags."""
    flags_n = flags_n or [(0, 0)] * 5
    flags_t = flags_t or (0, 0)
    rows = [normal_row(stencil[r], *flags_n[r], 1 / hx, gamma) for r in range(5)]
    F, dF = [0.0] * 4, [0.0] * 4
    for gp in range(2):
        sides = []
        for s in range(2):
            sides.append(tangential_side([rw[2 * s] for rw in rows], [rw[2 * s + 1] for rw in rows], gp, flags_t[s],
                                         1 / hy, gamma))
        f, d = gp_flux(sides[0][0], sides[0][2], sides[0][1], sides[1][0], sides[1][2], sides[1][1], gamma, c1, c2,
                       dt, 0.5)
        F = [F[c] + f[c] for c in range(4)]
        dF = [dF[c] + d[c] for c in range(4)]
    return F, dF


# ------------------------------------------------------------------ counts per unit
def _count(fn):
    COUNTS.clear()
    fn()
    return flops(), dict(COUNTS)


def _state(seed):
    import random
    rnd = random.Random(seed)
    rho, u, v, p = 1 + 0.1 * rnd.random(), 0.3 * rnd.random(), 0.2 * rnd.random(), 1 + 0.1 * rnd.random()
    return [Num(rho), Num(rho * u), Num(rho * v), Num(p / 0.4 + 0.5 * rho * (u * u + v * v))]


def per_unit_counts():
    """Operation counts of the units the kernels are measured on:
    gp_flux: the gas-kinetic flux of one Gauss point from its two reconstructed sides;
    normal_row_linear: one interface row's normal reconstruction, both sides linear;
    tangential_linear: one side's tangential reconstruction at one Gauss point, linear;
    ao_normal_extra / ao_tangential_extra: what WENO-AO adds for one flagged side over the linear path;
    per_gp_linear: one Gauss point of the linear path = gp_flux + 2 tangential sides + half a normal row
    (each row serves the two Gauss points of its segment)."""
    cells = [_state(k) for k in range(6)]
    W, Wx, Wy = _state(10), _state(11), _state(12)
    W2, Wx2, Wy2 = _state(13), _state(14), _state(15)
    out = {}
    out["gp_flux"] = _count(lambda: gp_flux(W, Wx, Wy, W2, Wx2, Wy2, 1.4, 0.01, 1.0, 1e-3, 0.5))
    out["normal_row_linear"] = _count(lambda: normal_row(cells, 0, 0, 10.0))
    nl_ao = _count(lambda: normal_row(cells, 1, 0, 10.0))
    lines = [_state(20 + k) for k in range(5)]
    lines_x = [_state(30 + k) for k in range(5)]
    out["tangential_linear"] = _count(lambda: tangential_side(lines, lines_x, 1, 0, 10.0))
    t_ao = _count(lambda: tangential_side(lines, lines_x, 1, 1, 10.0))
    out["ao_normal_extra"] = (nl_ao[0] - out["normal_row_linear"][0], None)
    out["ao_tangential_extra"] = (t_ao[0] - out["tangential_linear"][0], None)
    out["per_gp_linear"] = (out["gp_flux"][0] + 2 * out["tangential_linear"][0] + out["normal_row_linear"][0] / 2,
                            None)
    return out


if __name__ == "__main__":
    for k, (n, detail) in per_unit_counts().items():
        print(f"{k:22s} {n:8.1f}  {detail or ''}")
