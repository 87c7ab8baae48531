"""FP64 CPU oracle of the hybrid WENO5-AO gas-kinetic scheme -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. It loads ``oracle/liboracle.so`` (built from ``hgks_oracle.c`` by
``oracle/build.py``) and shares no code with the HIP library in ``paper_2304_05572_amd``.

Every function follows a passage of Mu et al., arXiv 2304.05572; see ``hgks_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_NOSLIP, BC_PRESCRIBED = 0, 1, 2, 3, 4
RECON_HYBRID, RECON_WENOAO, RECON_LINEAR = 0, 1, 2
EULER, NS = 0, 1
OK, EINVAL, ENONPHYS, EDT = 0, -1, -4, -5  # status codes of the C oracle


class _BcData(C.Structure):
    _fields_ = [("a", C.c_double * 4), ("b", C.c_double * 4), ("s0", C.c_double), ("sn", C.c_double),
                ("st", C.c_double), ("rest", C.c_int32), ("pad", C.c_int32)]


@dataclasses.dataclass
class BcData:
    """A prescribed-state side (boundary kind 4): a ghost cell takes the conserved state ``a`` where its
    tangential coordinate is below s0 + sn * (its normal coordinate) + st * t, else state ``b``
    (rest = 4) or the ghost of boundary kind ``rest`` (1 outflow, 2 reflect, 3 no-slip)."""
    a: tuple = (1.0, 0.0, 0.0, 2.5)
    b: tuple = (1.0, 0.0, 0.0, 2.5)
    s0: float = float("inf")
    sn: float = 0.0
    st: float = 0.0
    rest: int = BC_PRESCRIBED


class _Stepper(C.Structure):
    _fields_ = [("stages", C.c_int32), ("pad", C.c_int32), ("a", (C.c_double * 3) * 3), ("ah", (C.c_double * 3) * 3),
                ("b", C.c_double * 3), ("bh", C.c_double * 3)]


@dataclasses.dataclass
class Stepper:
    """Two-derivative multistage tableau (Sec. 2.2's family): W^(i) = W^n + sum_{j<i} (dt a[i][j] L_j +
    dt^2 ah[i][j] L_t,j), W^{n+1} = W^n + sum_i (dt b[i] L_i + dt^2 bh[i] L_t,i); stages 0 is the built-in
    S2O4."""
    stages: int = 0
    a: tuple = ((0.0,) * 3,) * 3
    ah: tuple = ((0.0,) * 3,) * 3
    b: tuple = (0.0,) * 3
    bh: tuple = (0.0,) * 3

    def c_struct(self) -> _Stepper:
        m = _Stepper()
        m.stages = int(self.stages)
        for i in range(3):
            m.b[i] = float((list(self.b) + [0.0] * 3)[i])
            m.bh[i] = float((list(self.bh) + [0.0] * 3)[i])
            for j in range(3):
                m.a[i][j] = float(self.a[i][j]) if i < len(self.a) and j < len(self.a[i]) else 0.0
                m.ah[i][j] = float(self.ah[i][j]) if i < len(self.ah) and j < len(self.ah[i]) else 0.0
        return m


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("eqn", C.c_int32), ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
        ("cfl", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("fixed_dt", C.c_double),
        ("bc", C.c_int32 * 4), ("recon", C.c_int32),
        ("gamma_hi", C.c_double), ("gamma_lo", C.c_double), ("weno_eps", C.c_double),
        ("zeta1_mode", C.c_int32), ("tangential_flag_mode", C.c_int32), ("positivity", C.c_int32),
        ("bcd", _BcData * 4), ("nz", C.c_int32), ("z0", C.c_double), ("z1", C.c_double), ("bcz", C.c_int32 * 2),
        ("stepper", _Stepper), ("char_state_mode", C.c_int32), ("viscous_dt_mode", C.c_int32),
    ]


@dataclasses.dataclass
class Problem:
    """Problem statement (paper Sec. 2 and Sec. 3); defaults are the paper's usual parameters."""
    dim: int = 2
    nx: int = 64
    ny: int = 64
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    eqn: int = EULER
    gamma: float = 1.4
    mu: float = 0.0
    Pr: float = 1.0
    cfl: float = 0.5
    c1: float = 0.01
    c2: float = 1.0
    fixed_dt: float = 0.0
    bc: tuple = (BC_OUTFLOW,) * 4
    recon: int = RECON_HYBRID
    gamma_hi: float = 0.85
    gamma_lo: float = 0.85
    weno_eps: float = 1e-8
    zeta1_mode: int = 0
    tangential_flag_mode: int = 0
    positivity: int = 0  # 1: first-order fallback for non-physical reconstructed states
    bcd: tuple = ()  # BcData per side (x-low, x-high, y-low, y-high), read where bc is BC_PRESCRIBED
    nz: int = 1      # 3D (dim = 3): cells along z on [z0, z1] and the kinds of the z sides
    z0: float = 0.0
    z1: float = 1.0
    bcz: tuple = (BC_OUTFLOW, BC_OUTFLOW)
    stepper: object = None  # Stepper (or its fields as a dict); None: the built-in S2O4
    char_state_mode: int = 0  # 2D: tangential characteristic state, 0 own side, 1 mean of both sides
    viscous_dt_mode: int = 0  # NS time step: 0 nu = mu / rho, 1 nu = mu / p

    @property
    def nc(self) -> int:
        return self.dim + 2

    @property
    def shape(self):
        if self.dim == 3:
            return (self.nc, self.nz, self.ny, self.nx)
        return (self.nc, self.nx) if self.dim == 1 else (self.nc, self.ny, self.nx)

    def c_struct(self) -> _Problem:
        s = _Problem()
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if f.name == "bc":
                arr = (C.c_int32 * 4)(*[int(b) for b in (list(v) + [0] * 4)[:4]])
                s.bc = arr
            elif f.name == "bcz":
                s.bcz = (C.c_int32 * 2)(*[int(b) for b in v])
            elif f.name == "stepper":
                if v is not None:
                    s.stepper = (Stepper(**v) if isinstance(v, dict) else v).c_struct()
            elif f.name == "bcd":
                for k, d in enumerate(list(v)[:4]):
                    if d is None:
                        continue
                    if isinstance(d, dict):
                        d = BcData(**d)
                    s.bcd[k].a = (C.c_double * 4)(*d.a)
                    s.bcd[k].b = (C.c_double * 4)(*d.b)
                    s.bcd[k].s0, s.bcd[k].sn, s.bcd[k].st, s.bcd[k].rest = d.s0, d.sn, d.st, int(d.rest)
            else:
                setattr(s, f.name, v)
        return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        d, i32, vp = C.c_double, C.c_int32, C.c_void_p
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        sig = {
            "oracle_flags": (i32, [P, vp, d, vp, vp]),
            "oracle_cfl_dt": (d, [P, vp]),
            "oracle_step": (i32, [P, vp, dp, d, dp, i32]),
            "oracle_stage_fluxes": (i32, [P, vp, d, d, vp, vp, vp, vp, i32]),
            "oracle_stencil_eval": (None, [i32, vp, d, dp, dp]),
            "oracle_beta": (d, [i32, vp]),
            "oracle_ao_eval": (None, [vp, d, d, d, d, dp, dp]),
            "oracle_indicator": (i32, [vp, d, i32, dp, dp, C.POINTER(i32)]),
            "oracle_char_matrices": (None, [i32, i32, vp, d, vp, vp]),
            "oracle_maxwell_moments": (None, [d, d, d, d, d, i32, vp, vp, vp]),
            "oracle_slope_solve": (None, [i32, vp, d, vp, vp]),
            "oracle_time_coeffs": (None, [d, d, vp]),
            "oracle_gp_flux": (None, [P, vp, vp, vp, vp, vp, vp, d, vp, vp, dp]),
            "oracle_cfl_dt3": (d, [P, vp]),
            "oracle_flags3": (i32, [P, vp, C.POINTER(vp)]),
            "oracle_stage_fluxes3": (i32, [P, vp, d, C.POINTER(vp), C.POINTER(vp), i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned status {code}")
        self.code = code


# ---------------------------------------------------------------- whole scheme
def flags(prob: Problem, W, t: float = 0.0):
    """Widened troubled-cell flags (Sec. 2.3.1 Steps 1-4) of every interior cell: (fx, fy); t is the time
    at which prescribed-state sides are evaluated."""
    W = _f64(W)
    ps = prob.c_struct()
    cells = prob.nx * (prob.ny if prob.dim == 2 else 1)
    fx = np.zeros(cells, np.uint8)
    fy = np.zeros(cells, np.uint8)
    rc = lib().oracle_flags(C.byref(ps), _ptr(W), float(t), _ptr(fx), _ptr(fy))
    if rc:
        raise OracleError(rc)
    shp = (prob.nx,) if prob.dim == 1 else (prob.ny, prob.nx)
    return fx.reshape(shp), (fy.reshape(shp) if prob.dim == 2 else None)


def flags3(prob: Problem, W):
    """Widened troubled-cell flags of every cell of a 3D problem, per direction: (fx, fy, fz), [nz][ny][nx]."""
    W = _f64(W)
    ps = prob.c_struct()
    f = [np.zeros((prob.nz, prob.ny, prob.nx), np.uint8) for _ in range(3)]
    arr = (C.c_void_p * 3)(*[x.ctypes.data for x in f])
    rc = lib().oracle_flags3(C.byref(ps), _ptr(W), arr)
    if rc:
        raise OracleError(rc)
    return tuple(f)


def stage_fluxes3(prob: Problem, W, dt: float, nthreads: int = 1):
    """F and dF/dt of a 3D state at every face: ((Fx, Gx), (Fy, Gy), (Fz, Gz)); Fx [5][nz][ny][nx+1], ..."""
    W = _f64(W)
    ps = prob.c_struct()
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    shapes = [(5, nz, ny, nx + 1), (5, nz, ny + 1, nx), (5, nz + 1, ny, nx)]
    F = [np.zeros(sh) for sh in shapes]
    G = [np.zeros(sh) for sh in shapes]
    fa = (C.c_void_p * 3)(*[x.ctypes.data for x in F])
    ga = (C.c_void_p * 3)(*[x.ctypes.data for x in G])
    rc = lib().oracle_stage_fluxes3(C.byref(ps), _ptr(W), float(dt), fa, ga, int(nthreads))
    if rc:
        raise OracleError(rc)
    return tuple(zip(F, G))


def cfl_dt(prob: Problem, W) -> float:
    """CFL time step (Sec. 3) before clipping to the end time."""
    W = _f64(W)
    ps = prob.c_struct()
    return lib().oracle_cfl_dt(C.byref(ps), _ptr(W))


def step(prob: Problem, W, t: float, t_end: float = float("inf"), nthreads: int = 1):
    """One S2O4 step (Sec. 2.2). Returns (W_new, t_new, dt_taken)."""
    W = _f64(W).copy()
    ps = prob.c_struct()
    tt = C.c_double(t)
    dtk = C.c_double(0.0)
    rc = lib().oracle_step(C.byref(ps), _ptr(W), C.byref(tt), float(t_end), C.byref(dtk), int(nthreads))
    if rc:
        raise OracleError(rc)
    return W, tt.value, dtk.value


def run(prob: Problem, W, t_end: float, max_steps: int = 10**9, t0: float = 0.0, nthreads: int = 1):
    """Advance to t_end (or max_steps). Returns (W, t, steps, dts)."""
    W = _f64(W).copy()
    t = t0
    dts = []
    while t < t_end and len(dts) < max_steps:
        W, t, dt = step(prob, W, t, t_end, nthreads)
        dts.append(dt)
    return W, t, len(dts), dts


def stage_fluxes(prob: Problem, W, dt: float, nthreads: int = 1, t: float = 0.0):
    """F and dF/dt at every interface of state W at time t for time step dt (paper eqs. for F and its
    time derivative)."""
    W = _f64(W)
    ps = prob.c_struct()
    nc, nx, ny = prob.nc, prob.nx, (prob.ny if prob.dim == 2 else 1)
    Fx = np.zeros((nc, ny, nx + 1))
    Gx = np.zeros_like(Fx)
    Fy = np.zeros((nc, ny + 1, nx)) if prob.dim == 2 else np.zeros(1)
    Gy = np.zeros_like(Fy)
    rc = lib().oracle_stage_fluxes(C.byref(ps), _ptr(W), float(t), float(dt), _ptr(Fx), _ptr(Gx), _ptr(Fy),
                                   _ptr(Gy), int(nthreads))
    if rc:
        raise OracleError(rc)
    if prob.dim == 1:
        return Fx[:, 0, :], Gx[:, 0, :], None, None
    return Fx, Gx, Fy, Gy


# ---------------------------------------------------------------- unit level
def stencil_eval(k: int, q, xi: float):
    q = _f64(q)
    v, d = C.c_double(), C.c_double()
    lib().oracle_stencil_eval(int(k), _ptr(q), float(xi), C.byref(v), C.byref(d))
    return v.value, d.value


def beta(k: int, q) -> float:
    q = _f64(q)
    return lib().oracle_beta(int(k), _ptr(q))


def ao_eval(q, xi: float, gamma_hi=0.85, gamma_lo=0.85, eps=1e-8):
    q = _f64(q)
    v, d = C.c_double(), C.c_double()
    lib().oracle_ao_eval(_ptr(q), float(xi), gamma_hi, gamma_lo, eps, C.byref(v), C.byref(d))
    return v.value, d.value


def indicator(q, h: float, zeta1_mode: int = 0):
    """Troubled-cell test of one component: (troubled, xbar, xhat, deciding step)."""
    q = _f64(q)
    xb, xh = C.c_double(), C.c_double()
    st = C.c_int32()
    t = lib().oracle_indicator(_ptr(q), float(h), int(zeta1_mode), C.byref(xb), C.byref(xh), C.byref(st))
    return int(t), xb.value, xh.value, st.value


def char_matrices(dim: int, direction: int, W, gamma=1.4):
    W = _f64(W)
    n = dim + 2
    R = np.zeros((n, n))
    L = np.zeros((n, n))
    lib().oracle_char_matrices(int(dim), int(direction), _ptr(W), float(gamma), _ptr(R), _ptr(L))
    return R, L


def maxwell_moments(U, V, lam, K, half=0):
    Mu = np.zeros(9)
    Mv = np.zeros(9)
    Mx = np.zeros(4)
    lib().oracle_maxwell_moments(1.0, float(U), float(V), float(lam), float(K), int(half), _ptr(Mu),
                                 _ptr(Mv), _ptr(Mx))
    return Mu, Mv, Mx


def slope_solve(dim: int, W, b, gamma=1.4):
    W = _f64(W)
    b = _f64(b)
    a = np.zeros(dim + 2)
    lib().oracle_slope_solve(int(dim), _ptr(W), float(gamma), _ptr(b), _ptr(a))
    return a


def time_coeffs(delta: float, tau: float):
    Cc = np.zeros(5)
    lib().oracle_time_coeffs(float(delta), float(tau), _ptr(Cc))
    return Cc


def gp_flux(prob: Problem, Wl, Wxl, Wyl, Wr, Wxr, Wyr, dt: float):
    """Time-integrated flux at one Gauss point for delta = dt and dt/2, and the collision time."""
    arrs = [_f64(a) for a in (Wl, Wxl, Wyl, Wr, Wxr, Wyr)]
    n = prob.nc
    Fd = np.zeros(n)
    Fh = np.zeros(n)
    tau = C.c_double()
    ps = prob.c_struct()
    lib().oracle_gp_flux(C.byref(ps), *[_ptr(a) for a in arrs], float(dt), _ptr(Fd), _ptr(Fh), C.byref(tau))
    return Fd, Fh, tau.value
