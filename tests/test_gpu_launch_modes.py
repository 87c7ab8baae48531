"""Launch configurations of the flux kernel (six tile shapes, each launched with one block per tile or
as a persistent grid) and the compensated stage accumulation, through the C ABI, against the oracle and
against each other."""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2304_05572_amd import hgks as H
from paper_2304_05572_amd import workloads as wl

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
NCONF = H.NUM_LAUNCH_CONFIGS


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def noisy_state(nx, ny, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    u = amp * rng.uniform(-1, 1, (ny, nx))
    v = amp * rng.uniform(-1, 1, (ny, nx))
    p = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    return wl.prim_to_cons(rho, u, v, p)


RP = dict(nx=70, ny=45, bc=(1, 1, 1, 1))


@pytest.fixture(scope="module")
def rp_oracle():
    W0 = wl.riemann_2d(70, seed=3, ny=45)[0]
    Wo, t, dts = W0.copy(), 0.0, []
    for _ in range(2):
        Wo, t, dt = O.step(O.Problem(**RP), Wo, t, nthreads=NT)
        dts.append(dt)
    return W0, Wo, dts


@pytest.mark.parametrize("config", range(NCONF))
def test_every_launch_config_matches_oracle_2d(rp_oracle, config):
    W0, Wo, dts = rp_oracle
    say("2d config", config)
    s = H.Solver(H.Problem(**RP), tile=config)
    s.set_ic(0, W0)
    got = [s.step()[0] for _ in range(2)]
    tile = s.tile()
    assert tile[3] == config and (tile[4] > 0) == (config >= NCONF // 2)
    assert got == dts
    assert rel(s.get_state(0)[0], Wo) < 1e-12


@pytest.mark.parametrize("config", range(NCONF))
def test_every_launch_config_matches_oracle_1d(config):
    W0 = wl.sod_1d(200)
    kw = dict(dim=1, nx=200, ny=1, bc=(2, 2, 0, 0))
    Wo, t = W0.copy(), 0.0
    for _ in range(3):
        Wo, t, _ = O.step(O.Problem(**kw), Wo, t, nthreads=NT)
    say("1d config", config)
    s = H.Solver(H.Problem(**kw), tile=config)
    s.set_ic(0, W0)
    for _ in range(3):
        s.step()
    assert rel(s.get_state(0)[0], Wo) < 1e-12


@pytest.mark.parametrize("shape", range(NCONF // 2))
def test_persistent_equals_one_block_per_tile(shape):
    """Same tile shape, same per-tile code: the persistent walk over a batch of uneven problems gives the
    per-tile launch's states (rounding-order identical up to a few ulps) and the same time steps."""
    specs = [(dict(nx=37, ny=21, bc=(1, 1, 1, 1)), wl.riemann_2d(37, seed=1, ny=21)[0]),
             (dict(nx=130, ny=96, bc=(1, 1, 1, 1)), wl.riemann_2d(130, seed=2, ny=96)[0]),
             (dict(nx=64, ny=9, bc=(0, 0, 1, 1)), noisy_state(64, 9, 2))]
    say("persistent vs per-tile, shape", shape)
    out = []
    for config in (shape, shape + NCONF // 2):
        s = H.Solver([H.Problem(**kw) for kw, _ in specs], tile=config)
        for p, (_, W) in enumerate(specs):
            s.set_ic(p, W)
        dts = [tuple(s.step()) for _ in range(3)]
        out.append((dts, [s.get_state(p)[0] for p in range(len(specs))]))
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        assert rel(a, b) < 1e-14


def test_persistent_grid_larger_than_tile_count():
    """Problems with fewer tiles than the persistent grid has blocks (blocks with no tile exit at once)."""
    specs = [(dict(nx=5, ny=5, bc=(1, 1, 1, 1)), wl.quadrants(5, 5, wl.RP_CONFIG1)),
             (dict(nx=9, ny=6, bc=(0, 0, 0, 0)), noisy_state(9, 6, 4))]
    say("tiny persistent")
    s = H.Solver([H.Problem(**kw) for kw, _ in specs], tile=NCONF // 2 + 4)
    for p, (_, W) in enumerate(specs):
        s.set_ic(p, W)
    dts = s.step()
    for p, (kw, W) in enumerate(specs):
        Wo, _, dto = O.step(O.Problem(**kw), W, 0.0, nthreads=NT)
        assert dts[p] == dto
        assert rel(s.get_state(p)[0], Wo) < 1e-12


def test_autotuner_picks_a_valid_config_and_stays_exact(rp_oracle):
    W0, Wo, dts = rp_oracle
    say("autotune")
    s = H.Solver(H.Problem(**RP), autotune=True)
    s.set_ic(0, W0)
    got = [s.step()[0] for _ in range(2)]
    assert 0 <= s.tile()[3] < NCONF
    assert got == dts and rel(s.get_state(0)[0], Wo) < 1e-12


# ------------------------------------------------------------------ compensated stage accumulation
def test_compensated_fp64_matches_oracle_and_plain(rp_oracle):
    W0, Wo, dts = rp_oracle
    say("compensated fp64")
    res = {}
    for comp in (False, True):
        s = H.Solver(H.Problem(**RP), compensated=comp)
        s.set_ic(0, W0)
        got = [s.step()[0] for _ in range(2)]
        assert got[0] == dts[0]  # the first step starts from the same rounded state
        W, _ = s.get_state(0)
        E = s.get_state_lo(0)
        if not comp:
            assert not E.any()
        else:
            assert np.all(np.abs(E) <= np.spacing(np.abs(W)))  # E is below W's rounding
        res[comp] = W
    assert rel(res[True], Wo) < 1e-12
    assert rel(res[True], res[False]) < 1e-13


def test_compensated_fp32_bulk_close_to_oracle():
    W0 = wl.riemann_2d(70, seed=3, ny=45)[0]
    Wo, t = W0.copy(), 0.0
    s = H.Solver(H.Problem(**RP), precision=H.FP32_BULK, compensated=True, use_graph=True)
    s.set_ic(0, W0)
    say("compensated fp32")
    for _ in range(10):
        Wo, t, _ = O.step(O.Problem(**RP), Wo, t, nthreads=NT)
    s.run(np.inf, 10)
    Wg, _ = s.get_state(0)
    assert np.abs(Wg - Wo).mean() / np.abs(Wo).mean() < 1e-5 and rel(Wg, Wo) < 1e-3


def test_compensation_conserves_the_carried_state():
    """Periodic box: the conserved totals change only by rounding. With plain FP64 sums every cell's
    state rounding enters the totals each step; the compensated state W + E keeps it, so its totals drift
    far less over 400 steps. The change of each total is summed exactly on the host (the totals
    themselves are ~2e3, whose ulp would hide it)."""
    nx, ny = 48, 40
    W0 = noisy_state(nx, ny, 11, amp=0.2)
    kw = dict(nx=nx, ny=ny, bc=(0, 0, 0, 0), cfl=0.5)
    drift = {}
    for comp in (False, True):
        s = H.Solver(H.Problem(**kw), compensated=comp, use_graph=True)
        s.set_ic(0, W0)
        steps = s.run(np.inf, 400)[0]
        assert steps == 400
        W, _ = s.get_state(0)
        E = s.get_state_lo(0)
        assert np.abs(W - W0).max() > 0.1  # the state did evolve
        drift[comp] = max(abs(math.fsum(np.concatenate([W[c].ravel(), E[c].ravel(), -W0[c].ravel()])))
                          for c in range(4))
    say("largest absolute drift of a conserved total: plain", drift[False], "compensated", drift[True])
    assert drift[False] < 1e-11  # both conserve to rounding
    assert drift[True] < drift[False] / 4


# Every launch configuration in the kernel's other instances: the Prandtl correction (Navier-Stokes, Pr =
# 0.73), the line-value tangential flag, forced WENO5-AO (every side through the characteristic path) and
# FP32-bulk. Stage fluxes of a 37 x 29 state (ragged against every tile shape) against the oracle's.
MODES = {
    "ns_prandtl": dict(eqn=O.NS, mu=2e-3, Pr=0.73, bc=(3, 2, 3, 2)),
    "line_value_flag": dict(tangential_flag_mode=1, bc=(1, 1, 1, 1)),
    "forced_wenoao": dict(recon=1, bc=(1, 1, 1, 1)),
    "fp32_bulk": dict(bc=(1, 1, 1, 1)),
}
_MODE_ORACLE = {}


def _mode_case(mode):
    if mode not in _MODE_ORACLE:
        W = wl.quadrants(37, 29, wl.RP_CONFIG6)
        kw = dict(nx=37, ny=29, **MODES[mode])
        Po = O.Problem(**kw)
        dt = 0.4 * O.cfl_dt(Po, W) / Po.cfl
        _MODE_ORACLE[mode] = (kw, W, dt, O.stage_fluxes(Po, W, dt, nthreads=NT))
    return _MODE_ORACLE[mode]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("config", range(NCONF))
def test_every_launch_config_in_every_kernel_instance(config, mode):
    """FP64 instances: every interface's F and dF/dt within 1e-12 of the largest magnitude of its array.
    FP32-bulk: within 1e-4 of it (the reconstruction and the moments carry a few hundred units of the FP32
    roundoff, 6e-8, into F and dF/dt; the time coefficients stay FP64)."""
    kw, W, dt, o = _mode_case(mode)
    prec = H.FP32_BULK if mode == "fp32_bulk" else H.FP64
    s = H.Solver(H.Problem(**kw), precision=prec, tile=config)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    assert s.tile()[3] == config
    s.close()
    tol = 1e-4 if prec == H.FP32_BULK else 1e-12
    worst = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(g, o))
    say("config", config, mode, "worst", worst)
    assert worst <= tol


@pytest.mark.parametrize("precision", [H.FP64, H.FP32_BULK])
@pytest.mark.parametrize("config", range(NCONF))
def test_minimum_grid_every_launch_config(config, precision):
    """The smallest grid the library takes (5 x 5, a fraction of one tile, ghosts reaching across the
    whole grid: periodic sides on x, reflecting and no-slip walls on y), two steps against the oracle:
    the first time step bit-exact (identical input state); the states within 1e-12 (FP64) or 1e-5
    (FP32-bulk) of the largest magnitude, and the second time step, which follows from the state after the
    first step, relatively within the same bound."""
    kw = dict(nx=5, ny=5, bc=(0, 0, 2, 3))
    W = noisy_state(5, 5, 11)
    Wo, t, dts = W.copy(), 0.0, []
    for _ in range(2):
        Wo, t, dt = O.step(O.Problem(**kw), Wo, t, nthreads=1)
        dts.append(dt)
    s = H.Solver(H.Problem(**kw), precision=precision, tile=config)
    s.set_ic(0, W)
    got = [s.step()[0] for _ in range(2)]
    Wg, _ = s.get_state(0)
    s.close()
    say("5x5 config", config, precision, rel(Wg, Wo), got[1] / dts[1] - 1)
    tol = 1e-12 if precision == H.FP64 else 1e-5
    assert got[0] == dts[0] and abs(got[1] / dts[1] - 1) < tol
    assert rel(Wg, Wo) < tol


@pytest.mark.parametrize("precision", [H.FP64, H.FP32_BULK])
@pytest.mark.parametrize("nx,ny", [(2000, 5), (5, 2000)])
def test_strip_grids(nx, ny, precision):
    """Strips one way thin (five cells: every tile ragged across them, ghosts on both sides of every row)
    and long the other, outflow on the long sides, reflecting walls on the short: flags bit-exact, the first
    time step bit-exact, one step within 1e-12 (FP64) or 1e-5 (FP32-bulk) of the largest magnitude."""
    kw = dict(nx=nx, ny=ny, bc=(2, 1, 1, 2) if nx > ny else (1, 2, 2, 1))
    W = noisy_state(nx, ny, 12)
    Po = O.Problem(**kw)
    Wo, _, dto = O.step(Po, W, 0.0, nthreads=NT)
    s = H.Solver(H.Problem(**kw), precision=precision)
    s.set_ic(0, W)
    fx, fy = s.flags(0)
    ox, oy = O.flags(Po, W)
    dt = s.step()[0]
    Wg, _ = s.get_state(0)
    s.close()
    say("strip", nx, ny, precision, rel(Wg, Wo))
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)
    assert dt == dto
    assert rel(Wg, Wo) < (1e-12 if precision == H.FP64 else 1e-5)
