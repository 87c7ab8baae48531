"""tangential_flag_mode = 1 (the hybrid indicator on the line values along the interface decides the
tangential reconstruction) through the C ABI against the oracle: stage fluxes of every launch
configuration (the tile then stages a third halo row), steps with bit-exact time steps, FP32-bulk, and on
a state layered along y the same fluxes as mode 0 to rounding (where the two readings agree)."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2304_05572_amd import hgks as H
from paper_2304_05572_amd import workloads as wl

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _noisy(n, m, seed):
    xc, yc = (np.arange(n) + 0.5) / n, (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(xc, yc)
    rng = np.random.default_rng(seed)
    rho = 1 + 0.3 * np.sin(2 * np.pi * (X + 0.3 * Y)) + 0.005 * rng.standard_normal((m, n)) + 0.5 * (X > 0.6)
    p = 1 + 0.2 * np.cos(2 * np.pi * (X - Y)) + 0.005 * rng.standard_normal((m, n))
    return wl.prim_to_cons(rho, 0.1 + 0 * X, -0.1 + 0 * X, p)


STATES = {
    "riemann": lambda: wl.riemann_2d(40, seed=11, ny=36)[0],
    "noisy": lambda: _noisy(40, 36, 5),
}


@pytest.fixture(scope="module", params=list(STATES))
def case(request):
    W = STATES[request.param]()
    kw = dict(nx=40, ny=36, bc=(1, 2, 0, 0), c1=0.01, c2=1.0, tangential_flag_mode=1)
    P = O.Problem(**kw)
    dt = O.cfl_dt(P, W)
    ref = O.stage_fluxes(P, W, dt, nthreads=NT)
    ref0 = O.stage_fluxes(O.Problem(**dict(kw, tangential_flag_mode=0)), W, dt, nthreads=NT)
    return request.param, kw, W, dt, ref, ref0


@pytest.mark.parametrize("config", range(H.NUM_LAUNCH_CONFIGS))
def test_stage_fluxes_every_config(case, config):
    name, kw, W, dt, ref, ref0 = case
    s = H.Solver(H.Problem(**kw), tile=config)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    worst = max(rel(a, b) for a, b in zip(g, ref))
    say(name, "config", config, "worst rel", worst)
    assert worst < 1e-12
    if name == "noisy" and config == 0:  # the readings differ on this state
        assert any(not np.allclose(a, b, rtol=0, atol=1e-10) for a, b in zip(ref, ref0))


def test_steps_match_oracle():
    """Six steps on a Riemann problem. (Unlike the cell flags, the line-value indicator decides on values
    that the two implementations compute with different rounding, so a value within rounding of a
    threshold can be decided differently: on the noisy state, which is full of marginal decisions, one
    such decision appeared within six steps and moved the state by 2e-5. Riemann data has none.)"""
    W = wl.riemann_2d(40, seed=12, ny=36)[0]
    kw = dict(nx=40, ny=36, bc=(1, 1, 1, 1), c1=0.01, c2=1.0, tangential_flag_mode=1)
    Po = O.Problem(**kw)
    s = H.Solver(H.Problem(**kw), use_graph=True)
    s.set_ic(0, W)
    Wg, tg, worst = W, 0.0, 0.0
    for k in range(6):
        Wo, to, dto = O.step(Po, Wg, tg, nthreads=NT)
        assert s.step()[0] == dto, k
        Wg, tg = s.get_state(0)
        assert tg == to
        worst = max(worst, rel(Wg, Wo))
    say("steps worst rel", worst)
    assert worst < 1e-12


def test_fp32_bulk_close_to_oracle():
    W = _noisy(40, 36, 7)
    kw = dict(nx=40, ny=36, bc=(1, 1, 1, 1), c1=0.01, c2=1.0, tangential_flag_mode=1)
    s = H.Solver(H.Problem(**kw), precision=H.FP32_BULK)
    s.set_ic(0, W)
    Wo, t = W.copy(), 0.0
    for _ in range(4):
        Wo, t, _ = O.step(O.Problem(**kw), Wo, t, nthreads=NT)
    s.run(np.inf, 4)
    Wg, _ = s.get_state(0)
    say("fp32 mode 1", rel(Wg, Wo))
    assert rel(Wg, Wo) < 1e-4


def test_y_layered_state_same_as_mode_0():
    ny, nx = 48, 20
    y = (np.arange(ny) + 0.5) / ny
    rho = 1.0 + 0.5 * (y > 0.37) + 0.3 * np.sin(2 * np.pi * y) + 0.6 * (np.abs(y - 0.75) < 0.06)
    v = 0.3 * np.cos(2 * np.pi * y)
    p = 1.0 + 0.4 * (y < 0.6)
    R, U, V, Pm = (np.broadcast_to(a[:, None], (ny, nx)) for a in (rho, 0.2 + 0 * y, v, p))
    W = wl.prim_to_cons(R, U, V, Pm)
    out = []
    for mode in (0, 1):
        s = H.Solver(H.Problem(nx=nx, ny=ny, bc=(0, 0, 1, 1), tangential_flag_mode=mode))
        s.set_ic(0, W)
        out.append(s.stage_fluxes(0, 1e-3))
    # the same decisions; the two modes are separate kernel instances, so only rounding may differ
    for a, b in zip(*out):
        assert rel(b, a) < 1e-12
