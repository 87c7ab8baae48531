"""A seeded 2D state whose first-stage intermediate state goes non-physical in the first step (strong
jumps along x at CFL 0.8, c1 = 0): the case that exercises the first-stage first-order fallback. Input
generation only."""
import numpy as np

from paper_2304_05572_amd import workloads as wl


def stage1_case(seed: int = 89):
    rng = np.random.default_rng(seed)
    n, ny = 40, 12
    k = rng.integers(3, 8)
    edges = np.sort(rng.choice(np.arange(5, n - 5), k, replace=False))
    seg = np.searchsorted(edges, np.arange(n))
    rho = 10 ** rng.uniform(-2, 1, k + 1)[seg]
    p = 10 ** rng.uniform(-3, 2, k + 1)[seg]
    u = rng.uniform(-6, 6, k + 1)[seg]
    R = np.broadcast_to(rho, (ny, n))
    Pm = np.broadcast_to(p, (ny, n))
    U = np.broadcast_to(u, (ny, n))
    V = 0.5 * np.sin(2 * np.pi * (np.arange(ny) + 0.5) / ny)[:, None] * np.ones((1, n))
    W = wl.prim_to_cons(R, U, V, Pm)
    kw = dict(nx=n, ny=ny, bc=(1, 1, 0, 0), cfl=0.8, c1=0.0, c2=1.0, positivity=1)
    return W, kw
