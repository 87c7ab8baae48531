"""The reading switches char_state_mode = 1 (tangential characteristic state: mean of both sides) and
viscous_dt_mode = 1 (printed viscous limit mu / p) through the C ABI against the oracle: stage fluxes,
steps with bit-exact time steps (2D Navier-Stokes and 3D), and FP32-bulk."""
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


@pytest.mark.parametrize("config", [0, 3, 4, 9])
def test_mean_char_state_stage_fluxes(config):
    W, _ = wl.riemann_2d(36, seed=14, ny=30)
    kw = dict(nx=36, ny=30, bc=(1, 1, 2, 3), c1=0.01, c2=1.0, char_state_mode=1)
    dt = O.cfl_dt(O.Problem(**kw), W)
    ref = O.stage_fluxes(O.Problem(**kw), W, dt, nthreads=NT)
    s = H.Solver(H.Problem(**kw), tile=config)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    worst = max(rel(a, b) for a, b in zip(g, ref))
    say("mean char state config", config, worst)
    assert worst < 1e-12


def test_mean_char_state_steps_and_fp32():
    W, _ = wl.riemann_2d(36, seed=15, ny=30)
    kw = dict(nx=36, ny=30, bc=(1, 1, 1, 1), c1=0.01, c2=1.0, char_state_mode=1, tangential_flag_mode=1)
    Po = O.Problem(**kw)
    s = H.Solver(H.Problem(**kw))
    s.set_ic(0, W)
    Wg, tg, worst = W, 0.0, 0.0
    for k in range(5):
        Wo, to, dto = O.step(Po, Wg, tg, nthreads=NT)
        assert s.step()[0] == dto, k
        Wg, tg = s.get_state(0)
        worst = max(worst, rel(Wg, Wo))
    say("mean char state steps", worst)
    assert worst < 1e-12
    f = H.Solver(H.Problem(**kw), precision=H.FP32_BULK)
    f.set_ic(0, W)
    f.run(np.inf, 5)
    Wf, _ = f.get_state(0)
    assert rel(Wf, Wg) < 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_printed_viscous_limit_steps(dim):
    if dim == 2:
        W, _ = wl.riemann_2d(30, seed=16, ny=24)
        kw = dict(nx=30, ny=24, bc=(3, 3, 2, 2))
    else:
        W = wl.octants_3d(10, 9, 8, seed=17)
        kw = dict(dim=3, nx=10, ny=9, nz=8, bc=(3, 3, 2, 2), bcz=(1, 1))
    kw.update(eqn=H.NS, mu=2e-2 if dim == 2 else 1e-1, Pr=1.0, cfl=0.4, c1=0.01, c2=1.0, viscous_dt_mode=1)
    Po = O.Problem(**kw)
    s = H.Solver(H.Problem(**kw))
    s.set_ic(0, W)
    Wg, tg, worst = W, 0.0, 0.0
    d0 = O.cfl_dt(O.Problem(**dict(kw, viscous_dt_mode=0)), W)
    for k in range(4):
        Wo, to, dto = O.step(Po, Wg, tg, nthreads=NT)
        assert s.step()[0] == dto, k
        Wg, tg = s.get_state(0)
        worst = max(worst, rel(Wg, Wo))
        if k == 0:
            say("dt printed / default", dto / d0)
            assert dto != d0  # the viscous limit binds and the readings differ
    assert worst < 1e-12
