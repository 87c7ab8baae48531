"""The entry point that allocates nothing (hgks_step_noalloc) against hgks_step on a handle, through the C
ABI on the GPU: the same kernels and launch configuration, so the state and the time step agree bit for
bit. Two calls in a row on the shared scratch array, the second with a smaller problem, in both
precisions and in 1D; a problem beyond the array's capacity is rejected before any device work; a step
that produces a non-physical state leaves the caller's state untouched."""
import sys

import numpy as np
import pytest
import torch

from paper_2304_05572_amd import hgks as H
from paper_2304_05572_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _handle_step(P, W0, precision):
    s = H.Solver(P, precision=precision)
    s.set_ic(0, W0)
    dt = s.step()[0]
    W, _ = s.get_state(0)
    s.close()
    return W, dt


def _noalloc_step(P, W0, precision, stream):
    Wd = torch.from_numpy(np.ascontiguousarray(W0)).to("cuda")
    torch.cuda.synchronize()
    dt = H.hgks_step_noalloc(P, precision, Wd, 0.0, stream)
    return Wd.cpu().numpy(), dt


@pytest.mark.parametrize("precision", [H.FP64, H.FP32_BULK])
def test_noalloc_step_equals_handle_step(precision):
    stream = torch.cuda.Stream()
    cases = [  # the second call of each pair smaller than the first
        (H.Problem(nx=560, ny=520), wl.riemann_2d(560, seed=4, ny=520)[0]),
        (H.Problem(nx=150, ny=90), wl.riemann_2d(150, seed=5, ny=90)[0]),
        (H.Problem(dim=1, nx=400, ny=1, bc=(H.BC_REFLECT,) * 2 + (0, 0)), wl.sod_1d(400)),
        (H.Problem(dim=1, nx=37, ny=1), wl.sod_1d(37)),
    ]
    for P, W0 in cases:
        say("noalloc", precision, P.dim, P.nx, P.ny)
        Wref, dtref = _handle_step(P, W0, precision)
        W, dt = _noalloc_step(P, W0, precision, stream)
        assert dt == dtref
        assert np.array_equal(W, Wref)
    # a second step of a double Mach reflection window (prescribed sides, positivity fallbacks), then a
    # fresh handle's two steps: the call takes the time t of its state
    W0, kw = wl.double_mach(120, 30)
    P = H.Problem(**kw)
    s = H.Solver(P, precision=precision)
    s.set_ic(0, W0)
    dts = [s.step()[0] for _ in range(2)]
    Wref, _ = s.get_state(0)
    Wd = torch.from_numpy(W0).to("cuda")
    torch.cuda.synchronize()
    d0 = H.hgks_step_noalloc(P, precision, Wd, 0.0, stream)
    d1 = H.hgks_step_noalloc(P, precision, Wd, d0, stream)
    assert [d0, d1] == dts and np.array_equal(Wd.cpu().numpy(), Wref)


def test_noalloc_rejects_and_keeps_state():
    # beyond the scratch array: rejected on the host, the caller's state untouched
    n = 700
    W0, _ = wl.riemann_2d(n, seed=1)
    Wd = torch.from_numpy(W0).to("cuda")
    with pytest.raises(H.HgksError) as e:
        H.hgks_step_noalloc(H.Problem(nx=n, ny=n), H.FP64, Wd, 0.0)
    assert e.value.code == H.ENOMEM
    assert np.array_equal(Wd.cpu().numpy(), W0)
    # a 3D problem is not taken
    W3 = torch.zeros((5, 6, 6, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HgksError) as e:
        H.hgks_step_noalloc(H.Problem(dim=3, nx=6, ny=6, nz=6), H.FP64, W3, 0.0)
    assert e.value.code == H.EINVAL
    # the blast wave as the paper states it fails in its first step: W stays the initial state
    Wb = wl.blast_wave_1d(400)
    P = H.Problem(dim=1, nx=400, ny=1, bc=(H.BC_REFLECT,) * 2 + (0, 0))
    Wd = torch.from_numpy(Wb).to("cuda")
    torch.cuda.synchronize()
    with pytest.raises(H.HgksError) as e:
        H.hgks_step_noalloc(P, H.FP64, Wd, 0.0)
    assert e.value.code == H.ENONPHYS
    assert np.array_equal(Wd.cpu().numpy(), Wb)
    # and the scratch array serves the next call normally
    W0, _ = wl.riemann_2d(64, seed=2)
    Wref, dtref = _handle_step(H.Problem(nx=64, ny=64), W0, H.FP64)
    Wd = torch.from_numpy(W0).to("cuda")
    torch.cuda.synchronize()
    assert H.hgks_step_noalloc(H.Problem(nx=64, ny=64), H.FP64, Wd, 0.0) == dtref
    assert np.array_equal(Wd.cpu().numpy(), Wref)
