"""Two readings kept as switches beside the defaults, pinned in the oracle:

* char_state_mode = 1: the tangential WENO-AO of each side in the characteristic variables of the mean of
  both sides' centre line values (the normal step's "averaged conservative variables from both sides"
  carried over to the interface). Where the two sides' line values agree (a state layered along y) it
  gives the default's fluxes; on the viscous shock tube at 100 x 50 cells it produces a non-physical
  state in the first step (the no-slip wall's ghost negates the tangential velocity, and the mean state
  of the wall segment has none), which is why the default takes each side's own state.
* viscous_dt_mode = 1: the printed viscous limit nu = mu / p instead of mu / rho in the time step
  (Sec. 3): on a uniform state limited by viscosity the two steps differ by the factor p / rho, and agree
  where p = rho."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2304_05572_amd import workloads as wl

NT = min(8, os.cpu_count() or 1)


def test_mean_state_equals_own_state_where_the_sides_agree():
    ny, nx = 40, 12
    y = (np.arange(ny) + 0.5) / ny
    rho = 1.0 + 0.5 * (y > 0.37) + 0.3 * np.sin(2 * np.pi * y) + 0.6 * (np.abs(y - 0.75) < 0.06)
    v = 0.3 * np.cos(2 * np.pi * y)
    p = 1.0 + 0.4 * (y < 0.6)
    R, U, V, Pm = (np.broadcast_to(a[:, None], (ny, nx)) for a in (rho, 0.2 + 0 * y, v, p))
    W = wl.prim_to_cons(R, U, V, Pm)
    kw = dict(nx=nx, ny=ny, bc=(0, 0, 1, 1), c1=0.01, c2=1.0)
    dt = O.cfl_dt(O.Problem(**kw), W)
    a = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
    b = O.stage_fluxes(O.Problem(**kw, char_state_mode=1), W, dt, nthreads=NT)
    for x, y_ in zip(a, b):
        assert np.abs(x - y_).max() <= 1e-13 * np.abs(x).max()


def test_mean_state_fails_the_viscous_shock_tube_first_step():
    nx, ny = 100, 50
    W = wl.viscous_shock_tube(nx, ny)
    W = W[0] if isinstance(W, tuple) else W
    kw = dict(dim=2, nx=nx, ny=ny, y1=0.5, bc=(3, 3, 3, 2), eqn=1, mu=1 / 200, Pr=0.73, cfl=0.3, c1=0.01, c2=1.0)
    O.step(O.Problem(**kw), W, 0.0, nthreads=NT)
    with pytest.raises(O.OracleError) as e:
        O.step(O.Problem(**kw, char_state_mode=1), W, 0.0, nthreads=NT)
    assert e.value.code == O.ENONPHYS


def test_mean_state_differs_on_riemann_data():
    W, _ = wl.riemann_2d(24, seed=3)
    kw = dict(nx=24, ny=24, bc=(1, 1, 1, 1), c1=0.01, c2=1.0)
    dt = O.cfl_dt(O.Problem(**kw), W)
    a = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
    b = O.stage_fluxes(O.Problem(**kw, char_state_mode=1), W, dt, nthreads=NT)
    assert any(not np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_printed_viscous_limit_scales_by_p_over_rho(dim):
    n = 16
    shape = {1: (n,), 2: (n, n), 3: (n, n, n)}[dim]
    rho, p = 1.3, 0.65
    one = np.ones(shape)
    if dim == 3:
        W = wl.prim_to_cons3(rho * one, 0 * one, 0 * one, 0 * one, p * one)
        kw = dict(dim=3, nx=n, ny=n, nz=n, bc=(0, 0, 0, 0), bcz=(0, 0))
    elif dim == 2:
        W = wl.prim_to_cons(rho * one, 0 * one, 0 * one, p * one)
        kw = dict(nx=n, ny=n, bc=(0, 0, 0, 0))
    else:
        W = np.stack([rho * one, 0 * one, p / 0.4 * one])
        kw = dict(dim=1, nx=n, ny=1, bc=(0, 0, 0, 0))
    kw.update(eqn=O.NS, mu=0.5, Pr=1.0, cfl=0.5)  # strongly viscous: the viscous limit binds
    d0 = O.cfl_dt(O.Problem(**kw), W)
    d1 = O.cfl_dt(O.Problem(**kw, viscous_dt_mode=1), W)
    assert abs(d1 / d0 - p / rho) < 1e-14
    # equal (to the rounding of p from the energy) where p = rho
    W2 = W.copy()
    W2[-1] = W[-1] * (rho / p)  # energy of the state at rest with p = rho
    a, b = O.cfl_dt(O.Problem(**kw), W2), O.cfl_dt(O.Problem(**kw, viscous_dt_mode=1), W2)
    assert abs(a - b) <= 1e-15 * a


@pytest.mark.parametrize("bad", [dict(char_state_mode=2), dict(dim=1, nx=20, ny=1, char_state_mode=1),
                                 dict(viscous_dt_mode=2)])
def test_invalid_reading_modes_rejected(bad):
    p = O.Problem(**bad)
    W = np.ones(p.shape)
    W[1:-1] = 0.0
    W[-1] = 2.5
    with pytest.raises(O.OracleError):
        O.step(p, W, 0.0)
