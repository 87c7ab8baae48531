"""Pins of the CPU oracle's building blocks against what the paper and the mathematics fix.

Each test compares the oracle with something other than itself: coefficients printed in the paper
(tests/golden/stencil_coeffs.txt), closed forms, brute-force quadrature (numpy Gauss-Hermite, mpmath),
finite-difference Jacobians, and textbook Chapman-Enskog results.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 1.4
K2 = (4 - 2 * G) / (G - 1)  # internal dof in 2D
K1 = (3 - G) / (G - 1)      # internal dof in 1D


# ------------------------------------------------------------------ reconstruction stencils
def _golden_stencils():
    rows = []
    with open(os.path.join(GOLDEN, "stencil_coeffs.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            parts = line.split()
            name, xi, kind = parts[0], parts[1], parts[2]
            coefs = [float(Fraction(c)) for c in parts[3:8]]
            rows.append((name, xi, kind, coefs))
    return rows


@pytest.mark.parametrize("row", _golden_stencils(), ids=lambda r: f"{r[0]}{r[1]}{r[2]}")
def test_stencil_coefficients_match_paper(row):
    """Printed interface values/slopes (Sec. 2.3.1 Step 5, WENO-AO sub-stencils) and the Step-1
    least-squares coefficients, recovered from the oracle by feeding unit cell averages."""
    name, xi, kind, coefs = row
    if name == "lsq":
        pytest.skip("least-squares coefficients are checked in test_least_squares_extreme_point")
    got = []
    for r in range(5):
        q = np.zeros(5)
        q[r] = 1.0
        v, d = O.stencil_eval(int(name[1]), q, float(xi))
        got.append(v if kind == "val" else d)
    np.testing.assert_allclose(got, coefs, rtol=0, atol=1e-14)


def test_least_squares_extreme_point():
    """Step 1-2: the indicator's extreme point is -a1/(2 a2) of the printed least-squares quadratic."""
    rows = {r[1]: np.array(r[3]) for r in _golden_stencils() if r[0] == "lsq"}
    rng = np.random.default_rng(5)
    for _ in range(50):
        q = rng.normal(size=5)
        a1, a2 = float(rows["a1"] @ q), float(rows["a2"] @ q)
        t, xbar, xhat, step = O.indicator(q, 1e-9)
        if step >= 2:
            assert xbar == pytest.approx(-a1 / (2 * a2), rel=1e-12)


def _cell_avg_poly(c, offs):
    """Exact cell averages of p(xi) = sum c_m xi^m over cells [o-1/2, o+1/2]."""
    out = []
    for o in offs:
        s = 0.0
        for m, cm in enumerate(c):
            s += cm * ((o + 0.5) ** (m + 1) - (o - 0.5) ** (m + 1)) / (m + 1)
        out.append(s)
    return np.array(out)


@pytest.mark.parametrize("xi", [0.5, -0.5, 1 / (2 * math.sqrt(3)), -1 / (2 * math.sqrt(3)), 0.17])
def test_stencils_exact_on_polynomials(xi):
    """The quartic reproduces any quartic and each quadratic any quadratic (cell-average matching)."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        c4 = rng.normal(size=5)
        q = _cell_avg_poly(c4, range(-2, 3))
        v, d = O.stencil_eval(3, q, xi)
        assert v == pytest.approx(np.polyval(c4[::-1], xi), abs=1e-12)
        assert d == pytest.approx(np.polyval(np.polyder(c4[::-1]), xi), abs=1e-12)
        c2 = rng.normal(size=3)
        q = _cell_avg_poly(c2, range(-2, 3))
        for k in range(3):
            v, d = O.stencil_eval(k, q, xi)
            assert v == pytest.approx(np.polyval(c2[::-1], xi), abs=1e-12)
            assert d == pytest.approx(np.polyval(np.polyder(c2[::-1]), xi), abs=1e-12)


def test_smoothness_indicators_closed_forms():
    """beta_k = sum_q int (d^q p / dxi^q)^2 over the cell: p = xi gives 1, p = xi^2 gives 1/3 + 4,
    p = xi^4 gives the quartic's 16/448 + 144/80 + 48 + 576."""
    q = _cell_avg_poly([0, 1], range(-2, 3))
    for k in range(4):
        assert O.beta(k, q) == pytest.approx(1.0, rel=1e-13)
    q = _cell_avg_poly([0, 0, 1], range(-2, 3))
    for k in range(4):
        assert O.beta(k, q) == pytest.approx(1 / 3 + 4, rel=1e-13)
    q = _cell_avg_poly([0, 0, 0, 0, 1], range(-2, 3))
    assert O.beta(3, q) == pytest.approx(16 / 448 + 144 / 80 + 48 + 576, rel=1e-13)


def test_weno_ao_reduces_to_linear_on_linear_data():
    """All beta equal -> delta = 0 -> omega = gamma -> p^AO = p3 exactly (identity of the AO form)."""
    q = _cell_avg_poly([0.3, -1.7], range(-2, 3))
    for xi in (0.5, -0.5, 0.2886751345948129):
        v, d = O.ao_eval(q, xi)
        vl, dl = O.stencil_eval(3, q, xi)
        assert v == pytest.approx(vl, abs=1e-14)
        assert d == pytest.approx(dl, abs=1e-14)


def test_weno_ao_converges_to_linear_on_smooth_data():
    for h in (0.2, 0.1, 0.05):
        offs = np.arange(-2, 3)
        q = np.array([(math.cos(h * (o - 0.5)) - math.cos(h * (o + 0.5))) / h for o in offs])  # avg of sin
        v, _ = O.ao_eval(q, 0.5)
        vl, _ = O.stencil_eval(3, q, 0.5)
        assert abs(v - vl) < 50 * h ** 5


def test_weno_ao_non_oscillatory_at_a_step():
    for q in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 1, 0, 0], [0, 0, 0, 0, 1]):
        q = np.array(q, float)
        for xi in (0.5, -0.5):
            v, _ = O.ao_eval(q, xi)
            assert -0.02 <= v <= 1.02, (q, xi, v)


# ------------------------------------------------------------------ troubled-cell indicator
def test_indicator_truth_tables():
    """Sec. 2.3.1 Steps 1-3: smooth data pass Step 1; unit steps are troubled with the extreme points
    computed by hand: (0,0,0,1,1): xbar=-1.02, xhat=-0.5; (0,0,1,1,1): xbar=1.02, xhat=0.5;
    (0,1,1,1,1): xbar=0.85, xhat=0 (the 1e-30 guard of the zero denominator)."""
    assert O.indicator([1, 1, 1, 1, 1], 0.1)[0] == 0
    assert O.indicator([1, 2, 3, 4, 5], 0.1)[0] == 0
    assert O.indicator([1, 2, 3, 4, 5], 0.1)[3] == 1
    for q, xb, xh in (([0, 0, 0, 1, 1], -1.02, -0.5), ([0, 0, 1, 1, 1], 1.02, 0.5), ([0, 1, 1, 1, 1], 0.85, 0.0)):
        t, xbar, xhat, step = O.indicator(q, 0.01)
        assert t == 1 and step == 3
        assert xbar == pytest.approx(xb, abs=1e-14)
        assert xhat == pytest.approx(xh, abs=1e-14)
    # a smooth extremum well resolved: Step 3 agrees (xbar ~ xhat)
    h = 0.01
    q = [(math.sin(h * (o + 0.5)) - math.sin(h * (o - 0.5))) / h for o in range(-2, 3)]  # avg of cos at 0
    t, xbar, xhat, step = O.indicator(q, 1e-9)
    assert t == 0 and step == 3 and abs(xbar) < 1e-6 and abs(xhat) < 1e-6


def test_indicator_mirror_symmetric_bitwise():
    rng = np.random.default_rng(7)
    for _ in range(4000):
        q = rng.normal(size=5) * rng.choice([1e-3, 1, 1e3])
        if rng.random() < 0.3:
            q = np.round(q, 1)
        a = O.indicator(q, 0.05)
        b = O.indicator(q[::-1].copy(), 0.05)
        assert a[0] == b[0]
        assert a[3] == b[3]
        if a[3] >= 2:
            assert a[1] == -b[1]


# ------------------------------------------------------------------ characteristic matrices
def _euler_flux(W, dim, direction):
    rho = W[0]
    if dim == 1:
        u = W[1] / rho
        p = (G - 1) * (W[2] - 0.5 * rho * u * u)
        return np.array([rho * u, rho * u * u + p, u * (W[2] + p)])
    u, v = W[1] / rho, W[2] / rho
    p = (G - 1) * (W[3] - 0.5 * rho * (u * u + v * v))
    un = u if direction == 1 else v
    return np.array([rho * un, W[1] * un + (p if direction == 1 else 0), W[2] * un + (p if direction == 2 else 0),
                     un * (W[3] + p)])


def _jacobian(W, dim, direction):
    n = len(W)
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1e-6 * max(1.0, abs(W[k]))
        J[:, k] = (_euler_flux(W + e, dim, direction) - _euler_flux(W - e, dim, direction)) / (2 * e[k])
    return J


@pytest.mark.parametrize("dim,direction", [(1, 1), (2, 1), (2, 2)])
def test_characteristic_matrices_diagonalise_the_jacobian(dim, direction):
    """R L = I and L A R = diag(u_n - c, u_n, (u_n,) u_n + c), A the finite-difference Jacobian."""
    rho, u, v, p = 0.8, 0.35, -0.6, 1.3
    if dim == 1:
        W = np.array([rho, rho * u, p / (G - 1) + 0.5 * rho * u * u])
    else:
        W = np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])
    R, L = O.char_matrices(dim, direction, W)
    np.testing.assert_allclose(R @ L, np.eye(dim + 2), atol=1e-13)
    D = L @ _jacobian(W, dim, direction) @ R
    c = math.sqrt(G * p / rho)
    un = u if direction == 1 else v
    lam = [un - c, un] + ([un] if dim == 2 else []) + [un + c]
    np.testing.assert_allclose(D, np.diag(lam), atol=1e-7)


# ------------------------------------------------------------------ Maxwellian moments
def test_moments_against_gauss_hermite_quadrature():
    from scipy import integrate
    U, V, lam, K = 0.37, -0.81, 1.9, K2
    Mu, Mv, Mx = O.maxwell_moments(U, V, lam, K, 0)
    x, w = np.polynomial.hermite.hermgauss(30)  # integrates exp(-x^2) poly exactly
    uu = U + x / math.sqrt(lam)
    for n in range(9):
        assert Mu[n] == pytest.approx((w * uu ** n).sum() / math.sqrt(math.pi), rel=1e-12, abs=1e-14)
    dens = lambda u: math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)
    for half, lo, hi in ((1, 0.0, np.inf), (-1, -np.inf, 0.0)):
        Mh, _, _ = O.maxwell_moments(U, V, lam, K, half)
        for n in range(9):
            ref = integrate.quad(lambda u: u ** n * dens(u), lo, hi, epsabs=1e-15, epsrel=1e-13)[0]
            assert Mh[n] == pytest.approx(ref, rel=1e-10, abs=1e-13)
    # xi^2 = sum of K squared N(0, 1/(2 lam)) variables, here K = 3 via a 3D Gauss-Hermite grid
    x3, w3 = np.polynomial.hermite.hermgauss(12)
    Xs = np.meshgrid(x3, x3, x3, indexing="ij")
    Ws = w3[:, None, None] * w3[None, :, None] * w3[None, None, :] / math.pi ** 1.5
    xi2 = sum(X ** 2 for X in Xs) / lam
    for k in range(4):
        assert Mx[k] == pytest.approx((Ws * xi2 ** k).sum(), rel=1e-12)


def _psi_matrix_quadrature(W, dim):
    """<psi_a psi_b> by tensor Gauss-Hermite quadrature over (u, v, xi_1..xi_K) for K = 3 (2D) / 4 (1D)."""
    rho = W[0]
    u0 = W[1] / rho
    v0 = W[2] / rho if dim == 2 else 0.0
    E = W[-1]
    p = (G - 1) * (E - 0.5 * rho * (u0 * u0 + v0 * v0))
    lam = rho / (2 * p)
    K = int(round(K2 if dim == 2 else K1))
    nvar = K + dim
    x, w = np.polynomial.hermite.hermgauss(6)
    grids = np.meshgrid(*([x] * nvar), indexing="ij")
    wts = np.ones(grids[0].shape)
    for k in range(nvar):
        shape = [1] * nvar
        shape[k] = len(w)
        wts = wts * w.reshape(shape)
    wts = wts / math.pi ** (nvar / 2)
    u = u0 + grids[0] / math.sqrt(lam)
    v = (v0 + grids[1] / math.sqrt(lam)) if dim == 2 else 0.0
    xi2 = sum(grids[k] ** 2 for k in range(dim, nvar)) / lam
    if dim == 2:
        psi = [np.ones_like(u), u, v, 0.5 * (u * u + v * v + xi2)]
    else:
        psi = [np.ones_like(u), u, 0.5 * (u * u + xi2)]
    n = len(psi)
    M = np.array([[(wts * psi[a] * psi[b]).sum() for b in range(n)] for a in range(n)])
    return M


@pytest.mark.parametrize("dim", [1, 2])
def test_slope_solver_roundtrip_by_quadrature(dim):
    """<a psi> = b with a = a.psi: check M a = b with M from brute-force quadrature over all K dof."""
    rho, u, v, p = 1.3, -0.4, 0.7, 0.8
    if dim == 2:
        W = np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])
    else:
        W = np.array([rho, rho * u, p / (G - 1) + 0.5 * rho * u * u])
    M = _psi_matrix_quadrature(W, dim)
    rng = np.random.default_rng(3)
    for _ in range(4):
        b = rng.normal(size=dim + 2)
        a = O.slope_solve(dim, W, b)
        np.testing.assert_allclose(M @ a, b, rtol=1e-11, atol=1e-11)


# ------------------------------------------------------------------ time integrals of Eq. (equ10)
def test_time_coefficients_against_mpmath():
    import mpmath as mp
    mp.mp.dps = 40
    funcs = [lambda t, T: 1 - mp.e ** (-t / T), lambda t, T: (t + T) * mp.e ** (-t / T) - T,
             lambda t, T: t - T + T * mp.e ** (-t / T), lambda t, T: mp.e ** (-t / T),
             lambda t, T: (t + T) * mp.e ** (-t / T)]
    for x in (1e-8, 1e-4, 0.03, 0.5, 0.99, 1.0, 1.7, 30.0, 1e4):
        tau = 0.37
        d = x * tau
        C = O.time_coeffs(d, tau)
        for k, f in enumerate(funcs):
            ref = mp.quad(lambda t: f(t, mp.mpf(tau)), [0, d])
            assert C[k] == pytest.approx(float(ref), rel=2e-14, abs=1e-300), (x, k)
    C = O.time_coeffs(0.3, 0.0)
    np.testing.assert_allclose(C, [0.3, 0, 0.045, 0, 0], atol=0)


# ------------------------------------------------------------------ gas-kinetic flux at a Gauss point
def _cons(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])


def _dcons(rho, u, v, p, dr, du, dv, dp):
    return np.array([dr, dr * u + rho * du, dr * v + rho * dv,
                     dp / (G - 1) + 0.5 * dr * (u * u + v * v) + rho * (u * du + v * dv)])


@pytest.mark.parametrize("tau_c", [0.0, 0.01, 1.0])
def test_uniform_state_gives_euler_flux(tau_c):
    W = _cons(0.9, 0.4, -0.3, 1.1)
    z = np.zeros(4)
    P = O.Problem(dim=2, c1=tau_c, c2=1.0)
    dt = 2e-3
    Fd, Fh, tau = O.gp_flux(P, W, z, z, W, z, z, dt)
    F = (4 * Fh - Fd) / dt
    dF = 4 * (Fd - 2 * Fh) / dt ** 2
    np.testing.assert_allclose(F, _euler_flux(W, 2, 1), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(dF, 0, atol=1e-9)


def test_inviscid_smooth_flux_time_derivative():
    """tau = 0 and continuous data: F = F_E(W) and dF/dt = A W_t, W_t = -(A W_x + B W_y)."""
    r, u, v, p = 1.1, 0.3, -0.2, 0.9
    W = _cons(r, u, v, p)
    Wx = _dcons(r, u, v, p, 0.2, -0.1, 0.3, 0.05)
    Wy = _dcons(r, u, v, p, -0.1, 0.25, 0.1, -0.2)
    P = O.Problem(dim=2, c1=0.0, c2=0.0)
    dt = 1e-3
    Fd, Fh, tau = O.gp_flux(P, W, Wx, Wy, W, Wx, Wy, dt)
    assert tau == 0.0
    F = (4 * Fh - Fd) / dt
    dF = 4 * (Fd - 2 * Fh) / dt ** 2
    A = _jacobian(W, 2, 1)
    B = _jacobian(W, 2, 2)
    np.testing.assert_allclose(F, _euler_flux(W, 2, 1), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dF, -A @ (A @ Wx + B @ Wy), rtol=1e-6, atol=1e-8)


def test_navier_stokes_shear_stress():
    """Continuous data, tau = mu/p: the x-flux of y-momentum carries -mu (U_y + V_x) and the energy
    flux the work -mu (U_y + V_x) V (Chapman-Enskog expansion of the BGK model)."""
    r, u, v, p, mu = 1.1, 0.3, -0.2, 0.9, 1e-3
    W = _cons(r, u, v, p)
    Wx = _dcons(r, u, v, p, 0, 0, 0.7, 0)
    Wy = _dcons(r, u, v, p, 0, 0.5, 0, 0)
    P = O.Problem(dim=2, eqn=O.NS, mu=mu, Pr=1.0, c1=0.0, c2=0.0)
    dt = 1e-3
    Fd, Fh, tau = O.gp_flux(P, W, Wx, Wy, W, Wx, Wy, dt)
    assert tau == pytest.approx(mu / p, rel=1e-14)
    F = (4 * Fh - Fd) / dt - _euler_flux(W, 2, 1)
    np.testing.assert_allclose(F, [0, 0, -mu * 1.2, -mu * 1.2 * v], atol=1e-14)


@pytest.mark.parametrize("Pr", [1.0, 0.73, 2.0])
def test_heat_flux_and_prandtl_correction(Pr):
    """Pure conduction (U = V = 0, uniform p): energy flux = -mu c_p T_x / Pr with c_p = (K+4)/2; the BGK
    model gives Pr = 1 and the correction (1/Pr - 1) q rescales the heat flux to the requested Pr."""
    r, p, mu, dr = 1.1, 0.9, 1e-3, -0.4
    W = _cons(r, 0, 0, p)
    Wx = _dcons(r, 0, 0, p, dr, 0, 0, 0)
    z = np.zeros(4)
    P = O.Problem(dim=2, eqn=O.NS, mu=mu, Pr=Pr, c1=0.0, c2=0.0)
    dt = 1e-3
    Fd, Fh, tau = O.gp_flux(P, W, Wx, z, W, Wx, z, dt)
    F = (4 * Fh - Fd) / dt - _euler_flux(W, 2, 1)
    dT = -p / r ** 2 * dr
    assert F[3] == pytest.approx(-mu * (K2 + 4) / 2 * dT / Pr, rel=1e-10)
    np.testing.assert_allclose(F[:3], 0, atol=1e-14)


def test_flux_mirror_symmetry():
    """Reflecting x -> -x (swap sides, negate normal momentum and x-slopes of the even variables) negates
    the mass, tangential-momentum and energy fluxes and keeps the normal-momentum flux."""
    rng = np.random.default_rng(11)
    P = O.Problem(dim=2, eqn=O.NS, mu=2e-3, Pr=0.73, c1=0.01, c2=1.0)
    for _ in range(3):
        Wl = _cons(rng.uniform(0.5, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 1.5))
        Wr = _cons(rng.uniform(0.5, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 1.5))
        Wxl, Wxr, Wyl, Wyr = (rng.normal(size=4) * 0.1 for _ in range(4))
        S = np.array([1, -1, 1, 1.0])
        Fd, Fh, _ = O.gp_flux(P, Wl, Wxl, Wyl, Wr, Wxr, Wyr, 1e-3)
        Gd, Gh, _ = O.gp_flux(P, S * Wr, -S * Wxr, S * Wyr, S * Wl, -S * Wxl, S * Wyl, 1e-3)
        np.testing.assert_allclose(Gd, -S * Fd, rtol=1e-11, atol=1e-15)


# ------------------------------------------------------------------ Step-4 widening of the indicator
def _isolated_pattern(n, c, s):
    """Zero data except (s, s, -s) on cells c, c+1, c+2 (s = 0.9 h). Steps 1-3 by hand, per cell window
    (cells i-2..i+2), with thr = 5h: i = c-2: D2 = 4s; c-1: D2 = 5s (both <= thr: smooth at Step 1);
    c: window (0,0,s,s,-s), D1 = -s, D2 = -13s, xbar = -17/130, 3-cell quadratic a1 = s/2, a2 = -s/2,
    xhat = 1/2, |xbar - xhat| = 0.631 > 1/4: TROUBLED; c+1: window (0,s,s,-s,0), D2 = -10s, D1 = -2s,
    xbar = -0.34, xhat = -0.5, |.| = 0.16 <= 1/4: smooth; c+2: window (s,s,-s,0,0), D2 = 15s, D1 = -3s,
    xbar = 0.34, xhat = 1/6, |.| = 0.173: smooth; c+3: D2 = 3s, c+4: D2 = -4s: smooth. So T = {c} only."""
    q = np.zeros(n)
    q[c:c + 3] = (s, s, -s)
    return q


def _widened(T):
    F = T.copy()
    F[1:] |= T[:-1]
    F[:-1] |= T[1:]
    return F


@pytest.mark.parametrize("comp", [0, -1])
def test_step4_widening_of_an_isolated_troubled_cell_1d(comp):
    """Sec. 2.3.1 Step 4 from the unwidened indicator: one troubled cell (c = 9) gives flags exactly at
    8, 9, 10; two troubled cells five apart give two separate triples (the widening is applied once, to
    the unwidened flags). The pattern sits in the density or in the energy of a state at rest."""
    n = 30
    h = 1.0 / n
    P = O.Problem(dim=1, nx=n, ny=1, bc=(0, 0, 0, 0))
    base = np.stack([np.ones(n), np.zeros(n), np.full(n, 2.5)])
    for cs in ([9], [9, 16]):
        W = base.copy()
        for c in cs:
            W[comp] += _isolated_pattern(n, c, 0.9 * h)
        fx, _ = O.flags(P, W)
        expect = np.zeros(n, np.uint8)
        for c in cs:
            expect[c - 1:c + 2] = 1
        assert np.array_equal(fx, expect), (cs, np.nonzero(fx))
        for c in cs:  # the unwidened indicator of the pattern's own window, by hand above
            assert O.indicator(W[comp][c - 2:c + 3], h)[0] == 1


@pytest.mark.parametrize("direction", [0, 1])
def test_step4_widening_per_direction_2d(direction):
    """2D: the pattern along x (the same in every row) flags columns c-1..c+1 in x and nothing in y; the
    transposed state flags rows c-1..c+1 in y and nothing in x (each direction widens its own flags)."""
    n = 24
    h = 1.0 / n
    P = O.Problem(dim=2, nx=n, ny=n, bc=(0, 0, 0, 0))
    line = _isolated_pattern(n, 11, 0.9 * h)
    rho = 1.0 + (line[None, :] if direction == 0 else line[:, None]) * np.ones((n, n))
    W = np.stack([rho, np.zeros((n, n)), np.zeros((n, n)), np.full((n, n), 2.5)])
    fx, fy = O.flags(P, W)
    band = np.zeros((n, n), np.uint8)
    if direction == 0:
        band[:, 10:13] = 1
        assert np.array_equal(fx, band) and not fy.any()
    else:
        band[10:13, :] = 1
        assert np.array_equal(fy, band) and not fx.any()
    # an isolated cell of the x-direction pattern in one row only: x flags in that row's three cells;
    # in y that cell's column sees a single cell of s and s, -s beside it: it decides its own y flags
    W1 = np.stack([np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n)), np.full((n, n), 2.5)])
    W1[0, 7] += line
    fx1, _ = O.flags(P, W1)
    exp = np.zeros((n, n), np.uint8)
    exp[7, 10:13] = 1
    assert np.array_equal(fx1, exp)
    assert np.array_equal(_widened(np.array([O.indicator(W1[0, 7, i - 2:i + 3], h)[0] if 2 <= i < n - 2 else 0
                                             for i in range(n)], np.uint8)), fx1[7])


# ------------------------------------------------------------------ smoothness indicators, exact arithmetic
def _frac_cell_avg_matrix(offs, deg):
    """Rows: exact cell averages of xi^m (m = 0..deg) over the cells [o - 1/2, o + 1/2]."""
    F = Fraction
    return [[(F(2 * o + 1, 2) ** (m + 1) - F(2 * o - 1, 2) ** (m + 1)) / (m + 1) for m in range(deg + 1)] for o in offs]


def _frac_solve(A, b):
    n = len(b)
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    for k in range(n):
        piv = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [x - f * y for x, y in zip(M[r], M[k])]
    return [M[k][n] / M[k][k] for k in range(n)]


def _frac_beta(q, offs):
    """sum over q = 1..deg of the integral over [-1/2, 1/2] of (d^q p / dxi^q)^2, p the polynomial of degree
    len(offs) - 1 with the given cell averages: polynomial algebra in exact fractions."""
    F = Fraction
    deg = len(offs) - 1
    c = _frac_solve(_frac_cell_avg_matrix(offs, deg), q)
    total = F(0)
    d = c[:]
    for _ in range(deg):
        d = [k * d[k] for k in range(1, len(d))]  # derivative
        sq = [F(0)] * (2 * len(d) - 1)
        for i, a in enumerate(d):
            for j, b in enumerate(d):
                sq[i + j] += a * b
        total += sum(a * (F(1, 2) ** (m + 1) - F(-1, 2) ** (m + 1)) / (m + 1) for m, a in enumerate(sq))
    return total


def test_smoothness_indicators_exact_on_random_data():
    """beta_k (Sec. 2.3.1, in normalised units) of generic data, every cross term of the squared
    derivatives included: random rational cell averages, the sub-stencil quadratics and the quartic
    fitted and integrated in exact fractions, against the oracle to 1e-12."""
    rng = np.random.default_rng(17)
    subs = {0: [-2, -1, 0], 1: [-1, 0, 1], 2: [0, 1, 2], 3: [-2, -1, 0, 1, 2]}
    for _ in range(30):
        q = [Fraction(int(rng.integers(-60, 61)), int(rng.integers(1, 13))) for _ in range(5)]
        for k, offs in subs.items():
            exact = _frac_beta([q[o + 2] for o in offs], offs)
            got = O.beta(k, np.array([float(x) for x in q]))
            assert got == pytest.approx(float(exact), rel=1e-12, abs=1e-12), (k, q)
