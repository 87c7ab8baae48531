"""The algorithmic operation count behind the bench's roofline (tests/opcount.py): its formulas are the
scheme's -- the interface flux it computes equals the oracle's, linear and WENO-AO paths -- and the
per-unit constants in bench.py are its counts."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import opcount as OC

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _smooth_state(n, jump=False):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = 1 + 0.1 * np.sin(2 * np.pi * (X + Y)) + 0.05 * np.cos(2 * np.pi * Y)
    u = 0.3 + 0.05 * np.sin(2 * np.pi * Y)
    v = -0.2 + 0.05 * np.cos(2 * np.pi * X)
    p = 1 + 0.03 * np.sin(2 * np.pi * (X - Y))
    if jump:
        rho = np.where(X + 0.3 * Y > 0.55, 0.4 * rho, rho)
        p = np.where(X + 0.3 * Y > 0.55, 0.3 * p, p)
    return np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])


def _stencil(W, j, i):
    ny, nx = W.shape[1:]
    return [[[OC.Num(W[c, (j + r - 2) % ny, (i - 3 + m) % nx]) for c in range(4)] for m in range(6)]
            for r in range(5)]


@pytest.mark.parametrize("jump", [False, True])
def test_counted_formulas_are_the_scheme(jump):
    """F and dF/dt of x-interfaces from the counted formulas against the oracle's stage fluxes (2D Euler,
    c1 = 0.01, c2 = 1, periodic), to 1e-11 relative: a smooth state (no troubled cell: the linear path)
    and one with an oblique jump, at interfaces whose normal or tangential flags are set (WENO-AO in
    characteristic variables), with the oracle's flags."""
    n = 32
    W = _smooth_state(n, jump)
    P = O.Problem(dim=2, nx=n, ny=n, bc=(0, 0, 0, 0), c1=0.01, c2=1.0)
    dt = 0.2 / n
    Fx, Gx, _, _ = O.stage_fluxes(P, W, dt)
    fx, fy = O.flags(P, W)
    if not jump:
        assert not fx.any() and not fy.any()
        picks = [(3, 5), (8, 0), (31, 11), (17, 30)]
    else:
        picks = [(j, i) for j in range(n) for i in range(n) if fx[j, i - 1] or fx[j, i] or fy[j, i - 1] or fy[j, i]][::7]
        assert len(picks) >= 5
    h = 1.0 / n
    for j, i in picks:
        fn = [(int(fx[(j + r - 2) % n, i - 1]), int(fx[(j + r - 2) % n, i % n])) for r in range(5)]
        ft = (int(fy[j, i - 1]), int(fy[j, i % n]))
        F, dF = OC.interface_flux(_stencil(W, j, i), h, h, dt, fn, ft)
        F = np.array([float(x) for x in F])
        dF = np.array([float(x) for x in dF])
        scale = np.abs(Fx[:, j, i]).max() + 1e-300
        np.testing.assert_allclose(F, Fx[:, j, i], rtol=0, atol=1e-11 * scale)
        np.testing.assert_allclose(dF, Gx[:, j, i], rtol=0, atol=1e-11 * (np.abs(Gx[:, j, i]).max() + 1e-300))


def test_bench_constants_are_the_counts():
    sys.path.insert(0, ROOT)
    import bench
    c = OC.per_unit_counts()
    assert bench.ALG_FLOPS_PER_GP_LINEAR == c["per_gp_linear"][0]
    assert bench.ALG_FLOPS_AO_NORMAL_SIDE == c["ao_normal_extra"][0]
    assert bench.ALG_FLOPS_AO_TANGENTIAL_SIDE == c["ao_tangential_extra"][0]
