"""The tangential flag read as the hybrid indicator on the line values along the interface (Sec. 2.3.3
Step 2 applies "the 1D hybrid method" to the line values; tangential_flag_mode = 1) against the default
reading (the side cell's flag along the interface, mode 0). On a state that varies along y only, the
line values at x-interfaces equal the cell averages and those at y-interfaces are constant along x, so
the two readings must flag the same sides and give the same fluxes: this pins the rows the line-value
indicator and its widening use. On general data the readings differ."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2304_05572_amd import workloads as wl

NT = min(8, os.cpu_count() or 1)


def _y_layered(nx, ny, seed):
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny
    rho = 1.0 + 0.5 * (y > 0.37) + 0.3 * np.sin(2 * np.pi * y) + 0.6 * (np.abs(y - 0.75) < 0.06)
    u = 0.2 + 0.1 * rng.standard_normal() + 0.0 * y
    v = 0.3 * np.cos(2 * np.pi * y)
    p = 1.0 + 0.4 * (y < 0.6)
    R, U, V, Pm = (np.broadcast_to(a[:, None], (ny, nx)) for a in (rho, u * np.ones(ny), v, p))
    return wl.prim_to_cons(R, U, V, Pm)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (0, 0, 2, 3)])
def test_line_value_indicator_equals_cell_flags_on_y_layered_state(bc):
    nx, ny = 12, 40
    W = _y_layered(nx, ny, 3)
    kw = dict(nx=nx, ny=ny, bc=bc, c1=0.01, c2=1.0)
    fx, fy = O.flags(O.Problem(**kw), W, 0.0)
    assert fy.any() and not fy.all()
    dt = O.cfl_dt(O.Problem(**kw), W)
    a = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
    b = O.stage_fluxes(O.Problem(**kw, tangential_flag_mode=1), W, dt, nthreads=NT)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_readings_agree_on_riemann_data_and_differ_on_noisy_data():
    """On a four-quadrant Riemann problem both readings flag the same sides: the widened cell flags cover
    the reach of the normal stencils, so a jump shows in the line values exactly where it shows in the
    cells. On a smooth field with small seeded noise (many marginal decisions) they differ."""
    W, _ = wl.riemann_2d(32, seed=9)
    kw = dict(nx=32, ny=32, bc=(1, 1, 1, 1), c1=0.01, c2=1.0)
    dt = O.cfl_dt(O.Problem(**kw), W)
    a = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
    b = O.stage_fluxes(O.Problem(**kw, tangential_flag_mode=1), W, dt, nthreads=NT)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    Wb, t, _, _ = O.run(O.Problem(**kw, tangential_flag_mode=1), W, 0.05, nthreads=NT)
    rho, _, _, p = wl.cons_to_prim(Wb)
    assert t == 0.05 and rho.min() > 0 and p.min() > 0
    n = 24
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc)
    rng = np.random.default_rng(1)
    rho = 1 + 0.3 * np.sin(2 * np.pi * (X + 0.3 * Y)) + 0.005 * rng.standard_normal((n, n))
    p = 1 + 0.2 * np.cos(2 * np.pi * (X - Y)) + 0.005 * rng.standard_normal((n, n))
    Ws = wl.prim_to_cons(rho, 0.1 + 0 * X, -0.1 + 0 * X, p)
    kw = dict(nx=n, ny=n, bc=(1, 1, 1, 1), c1=0.01, c2=1.0)
    dt = O.cfl_dt(O.Problem(**kw), Ws)
    a = O.stage_fluxes(O.Problem(**kw), Ws, dt, nthreads=NT)
    b = O.stage_fluxes(O.Problem(**kw, tangential_flag_mode=1), Ws, dt, nthreads=NT)
    assert any(not np.array_equal(x, y) for x, y in zip(a, b))


def test_forced_modes_ignore_the_reading():
    W, _ = wl.riemann_2d(16, seed=2)
    for recon in (1, 2):
        kw = dict(nx=16, ny=16, bc=(1, 1, 1, 1), recon=recon)
        dt = O.cfl_dt(O.Problem(**kw), W)
        a = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
        b = O.stage_fluxes(O.Problem(**kw, tangential_flag_mode=1), W, dt, nthreads=NT)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("bad", [dict(dim=1, nx=20, ny=1, tangential_flag_mode=1), dict(tangential_flag_mode=2)])
def test_invalid_modes_rejected(bad):
    p = O.Problem(**bad)
    W = np.ones(p.shape) * np.array([1.0, 0.0, 2.5] if p.dim == 1 else [1.0, 0.0, 0.0, 2.5]).reshape(-1, *([1] * (p.dim)))
    with pytest.raises(O.OracleError):
        O.step(p, W, 0.0)
