"""A seeded state whose first-stage intermediate state goes non-physical in the first step (strong
jumps along x at CFL 0.8, c1 = 0): the case that exercises the first-stage first-order fallback. Input
generation only."""
import numpy as np

from paper_2304_05572_amd import workloads as wl


def _profile(seed: int, n: int):
    rng = np.random.default_rng(seed)
    k = rng.integers(3, 8)
    edges = np.sort(rng.choice(np.arange(5, n - 5), k, replace=False))
    seg = np.searchsorted(edges, np.arange(n))
    rho = 10 ** rng.uniform(-2, 1, k + 1)[seg]
    p = 10 ** rng.uniform(-3, 2, k + 1)[seg]
    u = rng.uniform(-6, 6, k + 1)[seg]
    return rho, u, p


def stage1_case(seed: int = 89):
    """2D, 40 x 12 cells: the x-profile on every row and a y-velocity varying along y."""
    n, ny = 40, 12
    rho, u, p = _profile(seed, n)
    R = np.broadcast_to(rho, (ny, n))
    Pm = np.broadcast_to(p, (ny, n))
    U = np.broadcast_to(u, (ny, n))
    V = 0.5 * np.sin(2 * np.pi * (np.arange(ny) + 0.5) / ny)[:, None] * np.ones((1, n))
    W = wl.prim_to_cons(R, U, V, Pm)
    kw = dict(nx=n, ny=ny, bc=(1, 1, 0, 0), cfl=0.8, c1=0.0, c2=1.0, positivity=1)
    return W, kw


def stage1_case_1d(seed: int = 89):
    """1D, 40 cells: the same x-profile (one first-stage cell goes non-physical for seed 89)."""
    n = 40
    rho, u, p = _profile(seed, n)
    W = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
    kw = dict(dim=1, nx=n, ny=1, bc=(1, 1, 0, 0), cfl=0.8, c1=0.0, c2=1.0, positivity=1)
    return W, kw
