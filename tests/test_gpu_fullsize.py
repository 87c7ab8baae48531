"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark uses (autotuned),
against the CPU oracle: whole grids for one step where the oracle finishes in seconds, windows the oracle
can reproduce exactly (margin beyond the two-stage dependency radius of 8 cells) for later steps, sampled
problems of the 64-problem batch, and the 2D advection convergence study."""
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


def rp(n, **kw):
    return dict(dim=2, nx=n, ny=n, bc=(1, 1, 1, 1), cfl=0.5, c1=0.01, c2=1.0, **kw)


def l1(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())


def linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def rp1024():
    W0, _ = wl.riemann_2d(1024, seed=0)
    Wo, _, dto = O.step(O.Problem(**rp(1024)), W0, 0.0, nthreads=NT)
    return W0, Wo, dto


@pytest.mark.parametrize("precision,tol1,tolinf", [(H.FP64, 1e-14, 1e-12), (H.FP32_BULK, 1e-8, 1e-5)])
def test_riemann_1024_first_step_full_grid(rp1024, precision, tol1, tolinf):
    W0, Wo, dto = rp1024
    say("rp1024 first step", precision)
    s = H.Solver(H.Problem(**rp(1024)), precision=precision, autotune=True)
    s.set_ic(0, W0)
    fx, fy = s.flags(0)
    ox, oy = O.flags(O.Problem(**rp(1024)), W0)
    assert np.array_equal(fx, ox) and np.array_equal(fy, oy)
    dt = s.step()[0]
    assert dt == dto
    Wg, _ = s.get_state(0)
    say("L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
    PR.record("2 four-quadrant Riemann problem", PR.prec_name(precision), "1024^2 seed 0, first step, full grid",
              l1(Wg, Wo), linf(Wg, Wo), tol1, tolinf, dt_bit_exact=(dt == dto), flags_bit_exact=True)
    assert l1(Wg, Wo) < tol1 and linf(Wg, Wo) < tolinf


def _window_check(Wprev, Wnext, dt, n, centres, half=24, margin=10, bc=(1, 1, 1, 1), **kw):
    """Oracle one step on windows of Wprev (margin cells beyond the dependency radius, real boundary
    conditions where a window touches the domain edge) with the GPU's dt; compare window interiors."""
    h = 1.0 / n
    worst = 0.0
    A_all, B_all = [], []
    for (ci, cj) in centres:
        i0, i1 = max(ci - half - margin, 0), min(ci + half + margin, n)
        j0, j1 = max(cj - half - margin, 0), min(cj + half + margin, n)
        sub = np.ascontiguousarray(Wprev[:, j0:j1, i0:i1])
        wbc = (bc[0] if i0 == 0 else 1, bc[1] if i1 == n else 1, bc[2] if j0 == 0 else 1, bc[3] if j1 == n else 1)
        P = O.Problem(dim=2, nx=i1 - i0, ny=j1 - j0, x0=i0 * h, x1=i1 * h, y0=j0 * h, y1=j1 * h, bc=wbc,
                      fixed_dt=dt, **kw)
        Wo, _, _ = O.step(P, sub, 0.0, nthreads=NT)
        a0 = 0 if i0 == 0 else margin
        a1 = (i1 - i0) if i1 == n else (i1 - i0 - margin)
        b0 = 0 if j0 == 0 else margin
        b1 = (j1 - j0) if j1 == n else (j1 - j0 - margin)
        A = Wnext[:, j0 + b0:j0 + b1, i0 + a0:i0 + a1]
        B = Wo[:, b0:b1, a0:a1]
        worst = max(worst, linf(A, B))
        A_all.append(A.reshape(A.shape[0], -1))
        B_all.append(B.reshape(B.shape[0], -1))
    return worst, l1(np.concatenate(A_all, 1), np.concatenate(B_all, 1))


def test_riemann_1024_after_twelve_steps_windows():
    """After the waves have developed: the 12th step on windows over the shocks, the centre, a corner."""
    n = 1024
    W0, _ = wl.riemann_2d(n, seed=0)
    say("rp1024 windows after 12 steps")
    s = H.Solver(H.Problem(**rp(n)), precision=H.FP64, autotune=True)
    s.set_ic(0, W0)
    for _ in range(11):
        s.step()
    W11, _ = s.get_state(0)
    dt = s.step()[0]
    W12, _ = s.get_state(0)
    fx, _ = s.flags(0)
    centres = [(512, 512), (512, 300), (700, 512), (40, 30), (1000, 1010)]
    worst, wl1 = _window_check(W11, W12, dt, n, centres, cfl=0.5, c1=0.01, c2=1.0)
    say("worst window Linf", worst, "flagged", fx.mean())
    PR.record("2 four-quadrant Riemann problem", "fp64", "1024^2 seed 0, the 12th step on 5 windows of 48^2 cells "
              "(one oracle step from the GPU's 11th state); Linf: worst window", wl1, worst, 1e-12, 1e-12)
    assert worst < 1e-12


def test_riemann_1024_hundredth_step_windows():
    """The 100th step of the 1024^2 problem (seed 0) in the benchmark's launch configuration (autotuned), on
    windows over the developed shocks and contacts, the centre, the corners (one oracle step from the
    GPU's 99th state with its dt)."""
    n = 1024
    W0, _ = wl.riemann_2d(n, seed=0)
    say("rp1024 windows of the 100th step")
    s = H.Solver(H.Problem(**rp(n)), precision=H.FP64, autotune=True)
    s.set_ic(0, W0)
    s.run(np.inf, 99)
    W99, _ = s.get_state(0)
    dt = s.step()[0]
    W100, _ = s.get_state(0)
    centres = [(512, 512), (512, 300), (700, 512), (300, 700), (40, 30), (1000, 1010), (30, 1000)]
    worst, wl1 = _window_check(W99, W100, dt, n, centres, cfl=0.5, c1=0.01, c2=1.0)
    say("worst window Linf", worst)
    PR.record("2 four-quadrant Riemann problem", "fp64", "1024^2 seed 0, the 100th step on 7 windows of 48^2 cells "
              "(one oracle step from the GPU's 99th state); Linf: worst window", wl1, worst, 1e-12, 1e-12)
    assert worst < 1e-12


def test_viscous_shock_tube_1000x500():
    """Navier-Stokes, Re = 200, Pr = 0.73, no-slip walls, symmetry top: two steps of the full grid in FP64
    and in FP32-bulk against the oracle."""
    nx, ny = 1000, 500
    kw = dict(dim=2, nx=nx, ny=ny, y1=0.5, bc=(3, 3, 3, 2), eqn=1, mu=1 / 200, Pr=0.73, cfl=0.3, c1=0.01, c2=1.0)
    W0 = wl.viscous_shock_tube(nx, ny)
    Wo, t = W0, 0.0
    for _ in range(2):
        Wo, t, dto = O.step(O.Problem(**kw), Wo, t, nthreads=NT)
    for precision, tol in ((H.FP64, 1e-12), (H.FP32_BULK, 1e-6)):
        say("vst 1000x500", precision)
        s = H.Solver(H.Problem(**kw), precision=precision, autotune=True)
        s.set_ic(0, W0)
        s.step()
        s.step()
        Wg, tg = s.get_state(0)
        say("L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
        PR.record("3 viscous shock tube, NS 1000 x 500, Pr = 0.73", PR.prec_name(precision), "two steps, full grid",
                  l1(Wg, Wo), linf(Wg, Wo), tol)
        assert tg == pytest.approx(t, rel=1e-14)
        assert l1(Wg, Wo) < tol


@pytest.mark.parametrize("precision,tol1,tolinf", [(H.FP32_BULK, 1e-8, 1e-5), (H.FP64, 1e-14, 1e-12)])
def test_batch_of_64_sampled_problems(precision, tol1, tolinf):
    """64 uneven Riemann problems in one handle, one step; the smallest, the largest and two others are
    checked against the oracle (each has its own dt, bit-exact)."""
    sizes = wl.batch_sizes(64, seed=0)
    states = [wl.riemann_2d(m, seed=k + 1)[0] for k, m in enumerate(sizes)]
    say("batch 64", sum(m * m for m in sizes), "cells", precision)
    s = H.Solver([H.Problem(**rp(m)) for m in sizes], precision=precision, autotune=True)
    for p, W in enumerate(states):
        s.set_ic(p, W)
    dts = s.step()
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 41})
    for p in picks:
        Po = O.Problem(**rp(sizes[p]))
        Wo, _, dto = O.step(Po, states[p], 0.0, nthreads=NT)
        assert dts[p] == dto
        Wg, _ = s.get_state(p)
        say("problem", p, sizes[p], "L1", l1(Wg, Wo), "Linf", linf(Wg, Wo))
        PR.record("4 batch of 64 uneven problems", PR.prec_name(precision), f"problem {p} ({sizes[p]}^2), first step",
                  l1(Wg, Wo), linf(Wg, Wo), tol1, tolinf, dt_bit_exact=(dts[p] == dto))
        assert l1(Wg, Wo) < tol1 and linf(Wg, Wo) < tolinf


def _adv_points(n, t):
    xc = (np.arange(n) + 0.5) * (2.0 / n)
    X, Y = np.meshgrid(xc, xc)
    one = np.ones_like(X)
    return wl.prim_to_cons(1 + 0.2 * np.sin(np.pi * (X + Y - t)), one, one, one)


def test_advection_convergence_fp64_and_fp32():
    """2D density-wave advection, periodic [0,2]^2, CFL 0.5, tau = 0, t = 2, N = 20 .. 320: FP64 converges
    at fifth order on coarse grids and tends to the fourth order of the S2O4 time error on fine ones (the
    paper's WENO-AO table drops to 4.8 as well); FP32-bulk follows FP64 until its rounding floor (~1e-6
    after ~1e3 steps); both match the oracle at N = 20, 40."""
    errs = {H.FP64: [], H.FP32_BULK: []}
    ns = (20, 40, 80, 160, 320)
    for precision in (H.FP64, H.FP32_BULK):
        for n in ns:
            kw = dict(dim=2, nx=n, ny=n, x1=2.0, y1=2.0, bc=(0, 0, 0, 0), cfl=0.5, c1=0.0, c2=0.0)
            s = H.Solver(H.Problem(**kw), precision=precision)
            s.set_ic(0, _adv_points(n, 0.0))
            steps = s.run(2.0)[0]
            Wg, t = s.get_state(0)
            assert t == 2.0
            e = float(np.abs(Wg[0] - _adv_points(n, 2.0)[0]).mean())
            errs[precision].append(e)
            say("advection", precision, n, steps, "L1", e)
            if n <= 40:
                Wo, to, no, _ = O.run(O.Problem(**kw), _adv_points(n, 0.0), 2.0, nthreads=NT)
                tol = 1e-12 if precision == H.FP64 else 1e-6
                PR.record("1 density-wave advection 2D", PR.prec_name(precision), f"{n}^2, whole run to t = 2 ({no} steps)",
                          l1(Wg, Wo), linf(Wg, Wo), tol, exact_l1=e)
                assert no == steps
                assert l1(Wg, Wo) < tol
    e64 = np.array(errs[H.FP64])
    orders = np.log2(e64[:-1] / e64[1:])
    say("fp64 orders", orders)
    assert np.all(orders[:2] > 4.75) and np.all(orders > 4.0)
    e32 = np.array(errs[H.FP32_BULK])
    assert abs(e32[0] - e64[0]) / e64[0] < 0.02 and abs(e32[1] - e64[1]) / e64[1] < 0.15
    assert np.all(e32 < 2e-6 + e64)


def test_graph_replays_with_eager_work_between():
    """The captured step graph replayed many times, with eager torch work and synchronisations in
    between, gives the same states as eager launches after every replay."""
    import torch
    W0, _ = wl.riemann_2d(96, seed=5)
    a = H.Solver(H.Problem(**rp(96)), use_graph=True)
    b = H.Solver(H.Problem(**rp(96)), use_graph=False)
    a.set_ic(0, W0)
    b.set_ic(0, W0)
    x = torch.randn(1 << 20, device="cuda")
    for k in range(5):
        a.run(np.inf, 3)
        y = (x * 2.0).sum()  # unrelated eager work on the GPU
        torch.cuda.synchronize()
        b.run(np.inf, 3)
        assert np.array_equal(a.get_state(0)[0], b.get_state(0)[0]), k
        assert float(y) == float(y)


def test_workspace_bound_from_torch_matches_library_allocation():
    import torch
    W0, _ = wl.riemann_2d(64, seed=9)
    a = H.Solver(H.Problem(**rp(64)))
    ws = torch.empty(a.workspace_bytes(), dtype=torch.uint8, device="cuda")
    a.bind_workspace(ws)
    b = H.Solver(H.Problem(**rp(64)))
    for s in (a, b):
        s.set_ic(0, torch.from_numpy(W0).cuda())
        s.run(np.inf, 4)
    out = torch.empty(W0.shape, dtype=torch.float64, device="cuda")
    a.get_state(0, out)
    assert np.array_equal(out.cpu().numpy(), b.get_state(0)[0])


def test_largest_grid_64bit_offsets():
    """8192^2 cells (state arrays of 2.1 GB, flux arrays beyond 2^31 bytes): one FP64 step, windows at the
    origin, the centre and the far corner (whose byte offsets need 64 bits) against the oracle."""
    n = 8192
    W0, _ = wl.riemann_2d(n, seed=4)
    say("8192^2 one step")
    s = H.Solver(H.Problem(**rp(n)), precision=H.FP64)
    s.set_ic(0, W0)
    dt = s.step()[0]
    W1, _ = s.get_state(0)
    worst, wl1 = _window_check(W0, W1, dt, n, [(20, 20), (4096, 4096), (8170, 8175), (4096, 8180)], cfl=0.5,
                               c1=0.01, c2=1.0)
    say("worst window Linf", worst)
    PR.record("2 four-quadrant Riemann problem", "fp64", "8192^2 seed 4, first step on 4 windows (64-bit offsets); "
              "Linf: worst window", wl1, worst, 1e-12, 1e-12)
    assert worst < 1e-12
    del W1


def dyadic_cells(shape, nc, seed, block=64):
    """Cell averages on small dyadic alphabets (k/4 and 3k/8 for k = 0..3, k/2 for k = 1..16) with a cell
    size of 1, so that the indicator's sums are exact and many decisions fall exactly on a threshold
    (|D2| = 5 dx, |xbar| = 5/2, |xbar - xhat| = 1/4): there only a correctly rounded FP64 division in the
    canonical operation order gives the oracle's answer. Each block of cells draws one component from one
    alphabet (the other components stay constant, hence smooth), so that the OR over components and the
    widening mask few decisions in the blocks of the first two alphabets, whose flagged fraction is low."""
    table = np.concatenate([np.tile(np.arange(4) / 4, 4), np.tile(np.arange(4) * 3 / 8, 4),
                            np.arange(1, 17) / 2])
    rng = np.random.default_rng(seed)
    code = rng.integers(0, 16, shape, dtype=np.int16)
    axes = [(np.arange(m) // block).reshape([-1 if a == d else 1 for a in range(len(shape))])
            for d, m in enumerate(shape)]
    b = sum(ax * (1 + 6 * d) for d, ax in enumerate(reversed(axes)))
    comp, alph = b % nc, (b // nc) % 3
    code += (alph * 16).astype(np.int16)
    q = table[code]
    del code
    W = np.empty((nc,) + tuple(shape))
    for c, const in enumerate([1.0] + [0.0] * (nc - 2) + [2.5]):
        W[c] = np.where(comp == c, q, const)
    return W


@pytest.mark.parametrize("dim", [1, 2])
def test_flags_bit_exact_on_1e8_cells_at_exact_thresholds(dim):
    """The indicator's divisions and comparisons on 10^8 cells built to land exactly on its thresholds:
    the widened flags of every cell equal the oracle's."""
    if dim == 1:
        n = 10 ** 8
        kw = dict(dim=1, nx=n, ny=1, x0=0.0, x1=float(n), bc=(0, 0, 0, 0))
        W = dyadic_cells((n,), 3, seed=21, block=500)
    else:
        n = 10 ** 4
        kw = dict(dim=2, nx=n, ny=n, x0=0.0, x1=float(n), y0=0.0, y1=float(n), bc=(0, 0, 0, 0))
        W = dyadic_cells((n, n), 4, seed=22)
    say("flags at exact thresholds, dim", dim)
    s = H.Solver(H.Problem(**kw))
    s.set_ic(0, W)
    got = s.flags(0)
    s.close()
    ref = O.flags(O.Problem(**kw), W)
    del W
    for d in range(dim):
        say("direction", d, "flagged fraction", float(ref[d].mean()))
        assert 0.05 < ref[d].mean() < 0.7
        assert np.array_equal(got[d], ref[d])
