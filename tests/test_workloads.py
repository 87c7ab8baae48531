"""The seeded four-quadrant generator: every edge carries exactly one elementary wave, checked with the
exact 1D Riemann solver across each edge, and states stay within the stated ranges."""
import numpy as np
import pytest

import exact_riemann as ER
from paper_2304_05572_amd import workloads as wl


def _one_wave(L, R, tol=1e-7):
    """L, R = (rho, u_normal, p): exactly one of the three waves of their Riemann problem is present."""
    ps, us = ER.star_state(L, R)
    left_trivial = abs(ps - L[2]) < tol * ps and abs(us - L[1]) < tol * (1 + abs(us))
    right_trivial = abs(ps - R[2]) < tol * ps and abs(us - R[1]) < tol * (1 + abs(us))
    return left_trivial or right_trivial


@pytest.mark.parametrize("seed", range(40))
def test_quadrant_edges_are_elementary_waves(seed):
    st = wl.random_quadrant_states(np.random.default_rng(seed))
    assert wl._in_range(st)
    for a, b, normal in ((1, 0, 1), (2, 3, 1), (2, 1, 2), (3, 0, 2)):
        # vertical edges 2|1 and 3|4 (x-waves, normal velocity u); horizontal edges 3/2 and 4/1 (y-waves)
        A, B = st[a], st[b]
        L = (A[0], A[normal], A[3])
        R = (B[0], B[normal], B[3])
        assert _one_wave(L, R), (seed, a, b)
        tang = 3 - normal
        ps, us = ER.star_state(L, R)
        contact_only = abs(L[2] - R[2]) < 1e-9 and abs(L[1] - R[1]) < 1e-9
        if not contact_only:  # an acoustic wave keeps the tangential velocity and the entropy on one side
            assert abs(A[tang] - B[tang]) < 1e-12


def test_batch_sizes_range():
    s = wl.batch_sizes(64, seed=0)
    assert len(s) == 64 and min(s) >= 128 and max(s) <= 1024
