"""Two-derivative multistage steps (hgks_stepper) through the C ABI against the oracle: one-, two- and
three-stage tableaux in 1D, 2D and 3D, each step checked by an oracle step from the GPU's state (time
steps bit-exact, states to 1e-12); S2O4 written as a tableau against the library's own S2O4 path; the
FP32-bulk mode and HIP-graph replay."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2304_05572_amd import hgks as H
from paper_2304_05572_amd import workloads as wl

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)

# tableaux as plain data (Sec. 2.2's S2O4; the one-stage scheme; a three-stage tableau with every
# coefficient slot non-zero and distinct)
TABLEAUX = {
    "one": dict(stages=1, b=(1, 0, 0), bh=(0.5, 0, 0)),
    "s2o4": dict(stages=2, a=((0, 0, 0), (0.5, 0, 0), (0, 0, 0)), ah=((0, 0, 0), (0.125, 0, 0), (0, 0, 0)),
                 b=(1, 0, 0), bh=(1 / 6, 1 / 3, 0)),
    "three": dict(stages=3, a=((0, 0, 0), (0.4, 0, 0), (0.25, 0.35, 0)),
                  ah=((0, 0, 0), (0.08, 0, 0), (0.03, 0.05, 0)),
                  b=(0.3, 0.45, 0.25), bh=(0.07, 0.2, 0.05)),
}


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _case(dim):
    if dim == 1:
        return dict(dim=1, nx=70, ny=1, bc=(2, 1, 0, 0), cfl=0.4), wl.sod_1d(70)
    if dim == 2:
        W, _ = wl.riemann_2d(28, seed=6, ny=21)
        return dict(nx=28, ny=21, bc=(1, 1, 3, 2), cfl=0.4), W
    return dict(dim=3, nx=11, ny=9, nz=10, bc=(1, 1, 2, 2), bcz=(0, 0), cfl=0.4), wl.octants_3d(11, 9, 10, seed=7)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("name", list(TABLEAUX))
def test_tableau_steps_match_oracle(name, dim):
    kw, W = _case(dim)
    kw = dict(kw, c1=0.01, c2=1.0)
    Po = O.Problem(**kw, stepper=O.Stepper(**TABLEAUX[name]))
    s = H.Solver(H.Problem(**kw, stepper=H.Stepper(**TABLEAUX[name])))
    s.set_ic(0, W)
    say("tableau", name, "dim", dim)
    Wg, tg, worst = W, 0.0, 0.0
    for k in range(5):
        Wo, to, dto = O.step(Po, Wg, tg, nthreads=NT)
        assert s.step()[0] == dto, k
        Wg, tg = s.get_state(0)
        assert tg == to, k
        worst = max(worst, rel(Wg, Wo))
    say("worst step rel", worst)
    assert worst < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_s2o4_tableau_equals_the_s2o4_path(dim):
    kw, W = _case(dim)
    a = H.Solver(H.Problem(**kw))
    b = H.Solver(H.Problem(**kw, stepper=H.Stepper(**TABLEAUX["s2o4"])))
    a.set_ic(0, W)
    b.set_ic(0, W)
    a.run(np.inf, 6)
    b.run(np.inf, 6)
    Wa, ta = a.get_state(0)
    Wb, tb = b.get_state(0)
    say("s2o4 tableau vs path", rel(Wb, Wa), ta, tb)
    assert abs(ta - tb) <= 1e-14 * ta and rel(Wb, Wa) < 1e-12


def test_three_stage_fp32_and_graph_replay():
    kw, W = _case(2)
    st = H.Stepper(**TABLEAUX["three"])
    ref = H.Solver(H.Problem(**kw, stepper=st))
    ref.set_ic(0, W)
    ref.run(np.inf, 6)
    Wr, tr = ref.get_state(0)
    g = H.Solver(H.Problem(**kw, stepper=st), use_graph=True)
    g.set_ic(0, W)
    g.run(np.inf, 6)
    Wg, tg = g.get_state(0)
    assert tg == tr and np.array_equal(Wg, Wr)
    f = H.Solver(H.Problem(**kw, stepper=st), precision=H.FP32_BULK)
    f.set_ic(0, W)
    f.run(np.inf, 6)
    Wf, tf = f.get_state(0)
    say("fp32 three-stage", rel(Wf, Wr), abs(tf - tr) / tr)
    assert rel(Wf, Wr) < 1e-4 and abs(tf - tr) < 1e-5 * tr
