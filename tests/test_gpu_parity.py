"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on identical seeded inputs.

Bars: troubled-cell flags and the CFL time step bit-exact on an identical state; FP64 fluxes and states
to a relative 1e-12 (one stage) .. 1e-10 (tens of steps, rounding-order differences only); FP32-bulk
within the tolerance derived in the design notes. Grids are small enough for the oracle yet span several
tiles in both directions with ragged tails."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import parity_record as PR
from paper_2304_05572_amd import hgks as H
from paper_2304_05572_amd import workloads as wl

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def pair(**kw):
    return O.Problem(**kw), H.Problem(**kw)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _l1(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())


def noisy_state(nx, ny, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    u = amp * rng.uniform(-1, 1, (ny, nx))
    v = amp * rng.uniform(-1, 1, (ny, nx))
    p = 1.0 + amp * rng.uniform(-1, 1, (ny, nx))
    return wl.prim_to_cons(rho, u, v, p)


CASES_2D = {
    "rp_outflow": (dict(nx=70, ny=45, bc=(1, 1, 1, 1)), lambda: wl.riemann_2d(70, seed=3, ny=45)[0]),
    "rp_config1": (dict(nx=40, ny=36, bc=(1, 1, 1, 1)), lambda: wl.quadrants(40, 36, wl.RP_CONFIG1)),
    "noisy_reflect_periodic": (dict(nx=37, ny=29, bc=(2, 2, 0, 0)), lambda: noisy_state(37, 29, 5)),
    "noisy_noslip": (dict(nx=33, ny=40, bc=(3, 3, 3, 2)), lambda: noisy_state(33, 40, 6)),
}


def _flags_case(name):
    kw, ic = CASES_2D[name]
    return kw, ic()


@pytest.mark.parametrize("name", list(CASES_2D))
@pytest.mark.parametrize("zeta1_mode", [0, 1])
def test_flags_bit_exact(name, zeta1_mode):
    kw, W = _flags_case(name)
    Po, Ph = pair(zeta1_mode=zeta1_mode, **kw)
    say("flags", name, zeta1_mode)
    s = H.Solver(Ph)
    s.set_ic(0, W)
    fx, fy = s.flags(0)
    ox, oy = O.flags(Po, W)
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)
    assert ox.sum() + oy.sum() > 0 or name == "rp_config1"
    s.close()


def test_flags_bit_exact_1d():
    Po, Ph = pair(dim=1, nx=200, ny=1, bc=(2, 2, 0, 0))
    W = wl.sod_1d(200)
    say("flags 1d sod")
    s = H.Solver(Ph)
    s.set_ic(0, W)
    fx, _ = s.flags(0)
    ox, _ = O.flags(Po, W)
    assert np.array_equal(fx, ox) and ox.sum() > 0


@pytest.mark.parametrize("name", list(CASES_2D))
def test_stage_fluxes_fp64(name):
    kw, W = _flags_case(name)
    Po, Ph = pair(**kw)
    dt = 0.4 * O.cfl_dt(Po, W) / Po.cfl
    say("stage fluxes", name, dt)
    s = H.Solver(Ph)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    o = O.stage_fluxes(Po, W, dt, nthreads=NT)
    for a, b in zip(g, o):
        for c in range(4):
            assert rel(a[c], b[c]) < 1e-12 or np.abs(a[c] - b[c]).max() < 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("eqn,Pr,recon", [(O.NS, 0.73, 0), (O.NS, 1.0, 1), (O.EULER, 1.0, 1), (O.EULER, 1.0, 2)])
def test_stage_fluxes_fp64_modes(eqn, Pr, recon):
    """Navier-Stokes with and without the Prandtl correction, forced WENO-AO everywhere, forced linear."""
    nx, ny = 41, 23
    W = wl.quadrants(nx, ny, wl.RP_CONFIG6)
    Po, Ph = pair(nx=nx, ny=ny, bc=(3, 2, 3, 2), eqn=eqn, mu=2e-3, Pr=Pr, recon=recon)
    dt = 0.4 * O.cfl_dt(Po, W) / Po.cfl
    say("stage fluxes modes", eqn, Pr, recon)
    s = H.Solver(Ph)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    o = O.stage_fluxes(Po, W, dt, nthreads=NT)
    for a, b in zip(g, o):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_stage_fluxes_1d():
    Po, Ph = pair(dim=1, nx=200, ny=1, bc=(2, 2, 0, 0))
    W = wl.sod_1d(200)
    dt = O.cfl_dt(Po, W)
    say("stage fluxes 1d")
    s = H.Solver(Ph)
    s.set_ic(0, W)
    g = s.stage_fluxes(0, dt)
    o = O.stage_fluxes(Po, W, dt)
    for a, b in zip(g[:2], o[:2]):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("name", ["rp_outflow", "noisy_noslip"])
def test_steps_fp64(name):
    kw, W = _flags_case(name)
    Po, Ph = pair(**kw)
    say("steps fp64", name)
    s = H.Solver(Ph)
    s.set_ic(0, W)
    Wo, t = W.copy(), 0.0
    for k in range(6):
        dt_g = s.step()[0]
        Wg, tg = s.get_state(0)
        if k == 0:
            assert dt_g == O.cfl_dt(Po, W) * 1.0  # the CFL minimum is reproduced bit for bit
        Wo, t, dt_o = O.step(Po, Wo, t, nthreads=NT)
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o
        assert rel(Wg, Wo) < (1e-12 if k == 0 else 1e-11)
    # flags of the advanced state, evaluated on identical input, are still bit-exact
    fx, fy = s.flags(0)
    ox, oy = O.flags(Po, Wg)
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)


@pytest.mark.parametrize("precision", [H.FP64, H.FP32_BULK])
def test_sod_1d_full_run(precision):
    """Shock tube, 200 cells, reflective ends, CFL 0.5, t_end 0.2: FP64 within 1e-10 of the oracle's whole
    run (Linf relative); FP32-bulk within 1e-5 (L1) and 1e-3 (Linf), its step count within one of the
    oracle's (its time steps come from a state that differs by FP32 rounding)."""
    Po, Ph = pair(dim=1, nx=200, ny=1, bc=(2, 2, 0, 0), cfl=0.5)
    W = wl.sod_1d(200)
    say("sod 1d full run", precision)
    s = H.Solver(Ph, precision=precision)
    s.set_ic(0, W)
    steps = s.run(0.2)[0]
    Wg, tg = s.get_state(0)
    Wo, to, no, _ = O.run(Po, W, 0.2)
    if precision == H.FP64:
        PR.record("0 Sod tube 1D, 200 cells", "fp64", f"whole run to t = 0.2 ({no} steps)", _l1(Wg, Wo),
                  rel(Wg, Wo), 1e-10, 1e-10)
        assert tg == 0.2 and to == 0.2 and steps == no
        assert rel(Wg, Wo) < 1e-10
    else:
        PR.record("0 Sod tube 1D, 200 cells", "fp32_bulk", f"whole run to t = 0.2 ({no} oracle steps, {int(steps)} "
                  "GPU steps)", _l1(Wg, Wo), rel(Wg, Wo), 1e-5, 1e-3)
        assert tg == 0.2 and abs(int(steps) - no) <= 1
        assert _l1(Wg, Wo) < 1e-5 and rel(Wg, Wo) < 1e-3


def test_navier_stokes_steps():
    nx, ny = 48, 24
    W = wl.viscous_shock_tube(nx, ny)
    Po, Ph = pair(nx=nx, ny=ny, y1=0.5, bc=(3, 3, 3, 2), eqn=O.NS, mu=1 / 200, Pr=0.73, cfl=0.3)
    say("ns vst steps")
    s = H.Solver(Ph)
    s.set_ic(0, W)
    Wo, t = W.copy(), 0.0
    for k in range(4):
        s.step()
        Wo, t, _ = O.step(Po, Wo, t, nthreads=NT)
    Wg, _ = s.get_state(0)
    assert rel(Wg, Wo) < 1e-11


def test_batch_equals_single_problems():
    """Uneven problems in one handle advance exactly as when run alone (each has its own dt)."""
    specs = [(dict(nx=37, ny=21, bc=(1, 1, 1, 1)), wl.riemann_2d(37, seed=1, ny=21)[0]),
             (dict(nx=18, ny=40, bc=(2, 2, 2, 2)), wl.quadrants(18, 40, wl.RP_CONFIG6)),
             (dict(nx=64, ny=9, bc=(0, 0, 1, 1)), noisy_state(64, 9, 2))]
    say("batch")
    probs = [H.Problem(**kw) for kw, _ in specs]
    sb = H.Solver(probs)
    for p, (_, W) in enumerate(specs):
        sb.set_ic(p, W)
    for _ in range(3):
        dts = sb.step()
    for p, (kw, W) in enumerate(specs):
        s1 = H.Solver(H.Problem(**kw))
        s1.set_ic(0, W)
        for _ in range(3):
            dt1 = s1.step()[0]
        assert dt1 == dts[p]
        a, _ = sb.get_state(p)
        b, _ = s1.get_state(0)
        assert np.array_equal(a, b)
        Wo, t = W.copy(), 0.0
        Po = O.Problem(**kw)
        for _ in range(3):
            Wo, t, _ = O.step(Po, Wo, t, nthreads=NT)
        PR.record("4 batch (uneven problems in one handle)", "fp64",
                  f"problem {p} ({kw['nx']} x {kw['ny']}) after 3 steps; equal to its single run bitwise",
                  _l1(a, Wo), rel(a, Wo), 1e-11, 1e-11)
        assert rel(a, Wo) < 1e-11


def test_graph_replay_matches_direct_launches():
    kw, W = _flags_case("rp_outflow")
    say("graph replay")
    out = []
    for g in (0, 1):
        s = H.Solver(H.Problem(**kw), use_graph=g)
        s.set_ic(0, W)
        s.run(1.0, max_steps=5)
        out.append(s.get_state(0)[0])
        s.close()
    assert np.array_equal(out[0], out[1])


def test_free_stream_bitwise():
    one = np.ones((24, 40))
    W = wl.prim_to_cons(0.7 * one, 0.3 * one, -0.45 * one, 1.2 * one)
    say("free stream")
    s = H.Solver(H.Problem(nx=40, ny=24, bc=(1, 1, 0, 0)))
    s.set_ic(0, W)
    for _ in range(3):
        s.step()
    assert np.array_equal(s.get_state(0)[0], W)


def test_nonphysical_state_reported():
    W = wl.quadrants(20, 20, wl.RP_CONFIG1)
    W[3, 10, 10] = -1.0
    say("nonphysical")
    s = H.Solver(H.Problem(nx=20, ny=20))
    s.set_ic(0, W)
    with pytest.raises(H.HgksError) as e:
        s.step()
    assert e.value.code in (H.ENONPHYS, H.EDT)


def test_fp32_bulk_close_to_oracle():
    kw, W = _flags_case("rp_outflow")
    Po, Ph = pair(**kw)
    say("fp32 bulk")
    s = H.Solver(Ph, precision=H.FP32_BULK)
    s.set_ic(0, W)
    fx, fy = s.flags(0)
    ox, oy = O.flags(Po, W)
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)  # flags stay FP64
    Wo, t = W.copy(), 0.0
    for _ in range(10):
        s.step()
        Wo, t, _ = O.step(Po, Wo, t, nthreads=NT)
    Wg, _ = s.get_state(0)
    l1 = np.abs(Wg - Wo).mean() / np.abs(Wo).mean()
    say("fp32 L1_rel", l1, "Linf_rel", rel(Wg, Wo))
    PR.record("2 four-quadrant Riemann problem", "fp32_bulk", "70 x 45 (outflow), 10 steps", l1, rel(Wg, Wo), 1e-5,
              1e-3)
    assert l1 < 1e-5 and rel(Wg, Wo) < 1e-3


def test_batch_1d_uneven_with_minimum_size():
    """1D problems of uneven sizes down to the minimum of 5 cells in one handle: each advances exactly as
    when run alone (own dt) and matches the oracle."""
    specs = [(dict(dim=1, nx=200, ny=1, bc=(2, 2, 0, 0)), wl.sod_1d(200)),
             (dict(dim=1, nx=400, ny=1, x0=0.0, x1=10.0, bc=(1, 1, 0, 0)), wl.shu_osher_1d(400)),
             (dict(dim=1, nx=5, ny=1, x1=2.0, bc=(0, 0, 0, 0)), wl.advection_1d(5)),
             (dict(dim=1, nx=37, ny=1, bc=(3, 1, 0, 0)), wl.sod_1d(37))]
    say("batch 1d")
    sb = H.Solver([H.Problem(**kw) for kw, _ in specs])
    for p, (_, W) in enumerate(specs):
        sb.set_ic(p, W)
    for _ in range(4):
        dts = sb.step()
    for p, (kw, W) in enumerate(specs):
        s1 = H.Solver(H.Problem(**kw))
        s1.set_ic(0, W)
        for _ in range(4):
            dt1 = s1.step()[0]
        assert dt1 == dts[p]
        a, _ = sb.get_state(p)
        assert np.array_equal(a, s1.get_state(0)[0])
        Wo, t = W.copy(), 0.0
        for _ in range(4):
            Wo, t, _ = O.step(O.Problem(**kw), Wo, t, nthreads=NT)
        assert rel(a, Wo) < 1e-11
