"""Long runs against the CPU oracle: whole runs to the end time where the oracle finishes in seconds
(Shu-Osher, a 256^2 four-quadrant Riemann problem), windows of the 100th step of the viscous shock tube,
and the blast wave's failure reported the same way by both. After many steps the two states differ by
rounding order, so the bars are looser than one step's; troubled-cell flags stay bit-exact on an
identical state."""
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


def l1(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())


def linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


SHU = dict(dim=1, nx=400, ny=1, x0=0.0, x1=10.0, bc=(1, 1, 0, 0), cfl=0.5)


@pytest.fixture(scope="module")
def shu_oracle():
    W, t, n, _ = O.run(O.Problem(**SHU), wl.shu_osher_1d(400), 1.8, nthreads=NT)
    return W, n


@pytest.mark.parametrize("precision,tol1,tolinf", [(H.FP64, 1e-9, 1e-6), (H.FP32_BULK, 1e-4, 1e-2)])
def test_shu_osher_to_end_time(shu_oracle, precision, tol1, tolinf):
    """Sec. 3.2(b), 400 cells to t = 1.8 (689 steps), the whole run on the GPU against the oracle's."""
    Wo, no = shu_oracle
    say("shu-osher", precision)
    s = H.Solver(H.Problem(**SHU), precision=precision, use_graph=True)
    s.set_ic(0, wl.shu_osher_1d(400))
    steps = s.run(1.8)[0]
    Wg, t = s.get_state(0)
    say("steps", steps, "oracle", no, "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    PR.record("Shu-Osher 1D, 400 cells", PR.prec_name(precision), f"whole run to t = 1.8 ({no} oracle steps)",
              l1(Wg, Wo), linf(Wg, Wo), tol1, tolinf)
    assert t == 1.8 and abs(int(steps) - no) <= 1
    assert l1(Wg, Wo) < tol1 and linf(Wg, Wo) < tolinf
    fx, _ = s.flags(0)
    ox, _ = O.flags(O.Problem(**SHU), Wg)
    assert np.array_equal(fx, ox)


def test_blast_wave_reported_nonphysical_like_the_oracle():
    """Sec. 3.2(c) read as stated has no positivity treatment: the first step drives a cell's pressure
    negative next to the 1e5 pressure jump. Both paths report it as a non-physical state."""
    kw = dict(dim=1, nx=400, ny=1, bc=(2, 2, 0, 0), cfl=0.5)
    W0 = wl.blast_wave_1d(400)
    with pytest.raises(O.OracleError) as eo:
        O.step(O.Problem(**kw), W0, 0.0)
    assert eo.value.code == O.ENONPHYS
    say("blast wave")
    s = H.Solver(H.Problem(**kw))
    s.set_ic(0, W0)
    with pytest.raises(H.HgksError) as eg:
        s.step()
    assert eg.value.code == H.ENONPHYS


@pytest.mark.parametrize("precision,tol1", [(H.FP64, 1e-10), (H.FP32_BULK, 1e-4)])
def test_blast_wave_with_fallbacks_to_end_time(precision, tol1):
    """Sec. 3.2(c) with positivity = 1 (first-order fallbacks, among them the conservative one-stage flux
    on the faces of a cell the S2O4 update would leave non-physical): the whole run to t = 0.038 on the
    GPU against the oracle's, mass and energy conserved between the walls."""
    kw = dict(dim=1, nx=400, ny=1, bc=(2, 2, 0, 0), cfl=0.5, positivity=1)
    W0 = wl.blast_wave_1d(400)
    say("blast wave with fallbacks, oracle")
    Wo, to, no, _ = O.run(O.Problem(**kw), W0, 0.038, nthreads=NT)
    say("blast wave with fallbacks, gpu", precision)
    s = H.Solver(H.Problem(**kw), precision=precision, use_graph=True)
    s.set_ic(0, W0)
    steps = s.run(0.038)[0]
    Wg, t = s.get_state(0)
    say("steps", steps, "oracle", no, "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    PR.record("blast wave 1D with the first-order fallbacks", PR.prec_name(precision),
              f"whole run to t = 0.038 ({no} oracle steps)", l1(Wg, Wo), linf(Wg, Wo), tol1)
    assert t == 0.038 and abs(int(steps) - no) <= 2
    assert l1(Wg, Wo) < tol1
    for c in (0, 2):
        assert abs(Wg[c].sum() - W0[c].sum()) < (1e-12 if precision == H.FP64 else 1e-6) * W0[c].sum()


def test_riemann_256_to_end_time():
    """The seed-0 four-quadrant problem at 256^2 to t = 0.25 in FP64, GPU against oracle over the whole run
    (about 300 steps, each with its own bit-exact CFL step while the states agree to rounding)."""
    n = 256
    kw = dict(dim=2, nx=n, ny=n, bc=(1, 1, 1, 1), cfl=0.5, c1=0.01, c2=1.0)
    W0, _ = wl.riemann_2d(n, seed=0)
    say("rp256 to t_end: oracle")
    Wo, to, no, _ = O.run(O.Problem(**kw), W0, 0.25, nthreads=NT)
    say("rp256 to t_end: gpu")
    s = H.Solver(H.Problem(**kw), use_graph=True, autotune=True)
    s.set_ic(0, W0)
    steps = s.run(0.25)[0]
    Wg, t = s.get_state(0)
    say("steps", steps, "oracle", no, "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    fx, fy = s.flags(0)
    ox, oy = O.flags(O.Problem(**kw), Wg)
    PR.record("2 four-quadrant Riemann problem", "fp64", f"256^2 seed 0, whole run to t = 0.25 ({no} steps)",
              l1(Wg, Wo), linf(Wg, Wo), 1e-9, 1e-6,
              flag_mismatches_final_state=int((fx != ox).sum() + (fy != oy).sum()))
    assert t == 0.25 and steps == no
    assert l1(Wg, Wo) < 1e-9 and linf(Wg, Wo) < 1e-6
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)


def test_riemann_256_fp32_bulk_to_end_time():
    """The same problem in FP32-bulk (FP32 reconstruction and flux, FP64 state, flags and time step) to
    t = 0.25 against the FP64 oracle's whole run: the step count within one of the oracle's (the time step
    comes from a state that differs by FP32 rounding), L1 within 1e-5 and Linf within 1e-3 relative, and
    the flags of the final state, evaluated in FP64, bit-exact with the oracle's on that state."""
    n = 256
    kw = dict(dim=2, nx=n, ny=n, bc=(1, 1, 1, 1), cfl=0.5, c1=0.01, c2=1.0)
    W0, _ = wl.riemann_2d(n, seed=0)
    say("rp256 fp32-bulk to t_end: oracle")
    Wo, to, no, _ = O.run(O.Problem(**kw), W0, 0.25, nthreads=NT)
    say("rp256 fp32-bulk to t_end: gpu")
    s = H.Solver(H.Problem(**kw), precision=H.FP32_BULK, use_graph=True, autotune=True)
    s.set_ic(0, W0)
    steps = s.run(0.25)[0]
    Wg, t = s.get_state(0)
    say("steps", steps, "oracle", no, "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    fx, fy = s.flags(0)
    ox, oy = O.flags(O.Problem(**kw), Wg)
    PR.record("2 four-quadrant Riemann problem", "fp32_bulk", f"256^2 seed 0, whole run to t = 0.25 ({no} oracle "
              f"steps, {int(steps)} GPU steps)", l1(Wg, Wo), linf(Wg, Wo), 1e-5, 1e-3,
              flag_mismatches_final_state=int((fx != ox).sum() + (fy != oy).sum()))
    assert t == 0.25 and abs(int(steps) - no) <= 1
    assert l1(Wg, Wo) < 1e-5 and linf(Wg, Wo) < 1e-3
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)


@pytest.mark.parametrize("name,states,cfl,t_end", [("configuration 1", wl.RP_CONFIG1, 0.5, 0.2),
                                                   ("configuration 6", wl.RP_CONFIG6, 0.95, 0.6)])
def test_paper_riemann_configurations_to_end_time(name, states, cfl, t_end):
    """Sec. 3.4's configurations with their CFL numbers and end times, on a 128^2 grid: the whole FP64 run
    on the GPU against the oracle's (same step count; states to rounding-order differences), and the flags
    of the final state bit-exact."""
    n = 128
    kw = dict(dim=2, nx=n, ny=n, bc=(1, 1, 1, 1), cfl=cfl, c1=0.01, c2=1.0)
    W0 = wl.quadrants(n, n, states)
    say(name, "oracle")
    Wo, to, no, _ = O.run(O.Problem(**kw), W0, t_end, nthreads=NT)
    say(name, "gpu")
    s = H.Solver(H.Problem(**kw), use_graph=True, autotune=True)
    s.set_ic(0, W0)
    steps = s.run(t_end)[0]
    Wg, t = s.get_state(0)
    say("steps", steps, "oracle", no, "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    fx, fy = s.flags(0)
    ox, oy = O.flags(O.Problem(**kw), Wg)
    PR.record("2 four-quadrant Riemann problem", "fp64", f"Sec. 3.4 {name}, 128^2, whole run to t = {t_end} "
              f"({no} steps)", l1(Wg, Wo), linf(Wg, Wo), 1e-9, 1e-6,
              flag_mismatches_final_state=int((fx != ox).sum() + (fy != oy).sum()))
    assert t == t_end and steps == no
    assert l1(Wg, Wo) < 1e-9 and linf(Wg, Wo) < 1e-6
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)


def test_viscous_shock_tube_hundredth_step():
    """Navier-Stokes, 1000 x 500, Re = 200, Pr = 0.73: the 100th FP64 step on windows over the shock, the
    contact, the wall corners and the symmetry line against the oracle (each window one oracle step with
    the GPU's dt, margins beyond the dependency radius); FP32-bulk after 100 steps against FP64."""
    nx, ny = 1000, 500
    kw = dict(dim=2, nx=nx, ny=ny, y1=0.5, bc=(3, 3, 3, 2), eqn=1, mu=1 / 200, Pr=0.73, cfl=0.3, c1=0.01, c2=1.0)
    W0 = wl.viscous_shock_tube(nx, ny)
    say("vst 100 steps fp64")
    s = H.Solver(H.Problem(**kw), autotune=True, use_graph=True)
    s.set_ic(0, W0)
    s.run(np.inf, 99)
    W99, t99 = s.get_state(0)
    dt = s.step()[0]
    W100, _ = s.get_state(0)
    h = 1.0 / nx
    worst = 0.0
    A_all, B_all = [], []
    for (ci, cj) in [(500, 250), (520, 30), (560, 480), (30, 20), (970, 490), (700, 300)]:
        half, margin = 24, 10
        i0, i1 = max(ci - half - margin, 0), min(ci + half + margin, nx)
        j0, j1 = max(cj - half - margin, 0), min(cj + half + margin, ny)
        sub = np.ascontiguousarray(W99[:, j0:j1, i0:i1])
        wbc = (3 if i0 == 0 else 1, 3 if i1 == nx else 1, 3 if j0 == 0 else 1, 2 if j1 == ny else 1)
        P = O.Problem(dim=2, nx=i1 - i0, ny=j1 - j0, x0=i0 * h, x1=i1 * h, y0=j0 * h, y1=j1 * h, bc=wbc, eqn=1,
                      mu=1 / 200, Pr=0.73, fixed_dt=dt, c1=0.01, c2=1.0)
        Wo, _, _ = O.step(P, sub, t99, nthreads=NT)
        a0 = 0 if i0 == 0 else margin
        a1 = (i1 - i0) if i1 == nx else (i1 - i0 - margin)
        b0 = 0 if j0 == 0 else margin
        b1 = (j1 - j0) if j1 == ny else (j1 - j0 - margin)
        worst = max(worst, linf(W100[:, j0 + b0:j0 + b1, i0 + a0:i0 + a1], Wo[:, b0:b1, a0:a1]))
        A_all.append(W100[:, j0 + b0:j0 + b1, i0 + a0:i0 + a1].reshape(4, -1))
        B_all.append(Wo[:, b0:b1, a0:a1].reshape(4, -1))
    say("vst window Linf", worst)
    PR.record("3 viscous shock tube, NS 1000 x 500, Pr = 0.73", "fp64", "the 100th step on 6 windows of 48^2 cells "
              "(one oracle step from the GPU's 99th state); Linf: worst window",
              l1(np.concatenate(A_all, 1), np.concatenate(B_all, 1)), worst, 1e-12, 1e-12)
    assert worst < 1e-12
    say("vst 100 steps fp32-bulk")
    s32 = H.Solver(H.Problem(**kw), precision=H.FP32_BULK, autotune=True, use_graph=True)
    s32.set_ic(0, W0)
    s32.run(np.inf, 100)
    W32, _ = s32.get_state(0)
    say("fp32 vs fp64 after 100 steps L1", l1(W32, W100), "Linf", linf(W32, W100))
    PR.record("3 viscous shock tube, NS 1000 x 500, Pr = 0.73", "fp32_bulk", "after 100 steps against the FP64 GPU "
              "run (whose 100th step matches the oracle above)", l1(W32, W100), linf(W32, W100), 1e-6)
    assert l1(W32, W100) < 1e-6
