"""Python binding of the HIP library libhgks.so (C ABI in include/hgks.h).

Argument marshalling only: every step of the scheme runs in the library's HIP kernels. The functions
``hgks_create`` ... ``hgks_status_str`` mirror the C entry points one to one; ``Solver`` is a small
convenience wrapper over them. Device buffers may be torch tensors on the GPU (passed by address with
``on_device=1``); host buffers are numpy arrays.

Importing this module does not touch the GPU. Loading the library fails loudly (``HgksLibraryMissing``)
if ``libhgks.so`` has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgks.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYS, EDT = 0, -1, -2, -3, -4, -5
EULER, NS = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_NOSLIP, BC_PRESCRIBED = 0, 1, 2, 3, 4
RECON_HYBRID, RECON_WENOAO, RECON_LINEAR = 0, 1, 2
FP64, FP32_BULK = 0, 1
NUM_LAUNCH_CONFIGS = 12  # flux launch configurations: 6 tile shapes x (one block per tile, persistent)

ENTRY_POINTS = ("hgks_create", "hgks_workspace_bytes", "hgks_bind_workspace", "hgks_set_ic", "hgks_step",
                "hgks_run", "hgks_get_state", "hgks_get_state_lo", "hgks_debug_flags", "hgks_debug_stage_fluxes",
                "hgks_debug_flags3", "hgks_debug_stage_fluxes3", "hgks_get_stats", "hgks_get_tile", "hgks_get_profile", "hgks_destroy", "hgks_status_str",
                "hgks_step_noalloc")
NOALLOC_SCRATCH_BYTES = 64 << 20  # HGKS_NOALLOC_SCRATCH_BYTES


class HgksLibraryMissing(ImportError):
    pass


class HgksError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {hgks_status_str(code)} ({code})")
        self.code = code


class hgks_bc_data(C.Structure):
    _fields_ = [("a", C.c_double * 4), ("b", C.c_double * 4), ("s0", C.c_double), ("sn", C.c_double),
                ("st", C.c_double), ("rest", C.c_int32), ("reserved", C.c_int32)]


@dataclasses.dataclass
class BcData:
    """A prescribed-state side (BC_PRESCRIBED): ghost cells take the conserved state ``a`` where their
    tangential coordinate is below s0 + sn * (normal coordinate) + st * t, else the state ``b``
    (rest = BC_PRESCRIBED) or the ghost of boundary kind ``rest``."""
    a: tuple = (1.0, 0.0, 0.0, 2.5)
    b: tuple = (1.0, 0.0, 0.0, 2.5)
    s0: float = float("inf")
    sn: float = 0.0
    st: float = 0.0
    rest: int = BC_PRESCRIBED


class hgks_stepper(C.Structure):
    _fields_ = [("stages", C.c_int32), ("reserved", C.c_int32), ("a", (C.c_double * 3) * 3),
                ("ah", (C.c_double * 3) * 3), ("b", C.c_double * 3), ("bh", C.c_double * 3)]


@dataclasses.dataclass
class Stepper:
    """Two-derivative multistage tableau (hgks_stepper): W^(i) = W^n + sum_{j<i} (dt a[i][j] L_j + dt^2
    ah[i][j] L_t,j), W^{n+1} = W^n + sum_i (dt b[i] L_i + dt^2 bh[i] L_t,i); stages 0 is S2O4."""
    stages: int = 0
    a: tuple = ((0.0,) * 3,) * 3
    ah: tuple = ((0.0,) * 3,) * 3
    b: tuple = (0.0,) * 3
    bh: tuple = (0.0,) * 3

    def c_struct(self) -> hgks_stepper:
        m = hgks_stepper()
        m.stages = int(self.stages)
        for i in range(3):
            m.b[i] = float((list(self.b) + [0.0] * 3)[i])
            m.bh[i] = float((list(self.bh) + [0.0] * 3)[i])
            for j in range(3):
                m.a[i][j] = float(self.a[i][j]) if i < len(self.a) and j < len(self.a[i]) else 0.0
                m.ah[i][j] = float(self.ah[i][j]) if i < len(self.ah) and j < len(self.ah[i]) else 0.0
        return m


class hgks_problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("eqn", C.c_int32), ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
        ("cfl", C.c_double), ("c1", C.c_double), ("c2", C.c_double), ("fixed_dt", C.c_double),
        ("bc", C.c_int32 * 4), ("recon", C.c_int32),
        ("gamma_hi", C.c_double), ("gamma_lo", C.c_double), ("weno_eps", C.c_double),
        ("zeta1_mode", C.c_int32), ("tangential_flag_mode", C.c_int32), ("positivity", C.c_int32),
        ("bcd", hgks_bc_data * 4),
        ("nz", C.c_int32), ("z0", C.c_double), ("z1", C.c_double), ("bcz", C.c_int32 * 2),
        ("stepper", hgks_stepper), ("char_state_mode", C.c_int32), ("viscous_dt_mode", C.c_int32),
    ]


class hgks_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("autotune", C.c_int32), ("use_graph", C.c_int32),
                ("tile", C.c_int32), ("profile", C.c_int32), ("compensated", C.c_int32),
                ("hip_stream", C.c_void_p)]


@dataclasses.dataclass
class Problem:
    """Problem statement (paper Sec. 2; parameters of Sec. 3). dim 1, 2 or 3; for dim 3 the grid is
    nx x ny x nz on [x0, x1] x [y0, y1] x [z0, z1], bc holds the x and y sides and bcz the z sides."""
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
    nz: int = 1
    z0: float = 0.0
    z1: float = 1.0
    bcz: tuple = (BC_OUTFLOW,) * 2
    stepper: object = None  # Stepper (or its fields as a dict); None: S2O4
    char_state_mode: int = 0  # 2D: tangential characteristic state, 0 own side, 1 mean of both sides
    viscous_dt_mode: int = 0  # NS time step: 0 nu = mu / rho, 1 the printed nu = mu / p

    @property
    def nc(self):
        return self.dim + 2

    @property
    def shape(self):
        if self.dim == 1:
            return (self.nc, self.nx)
        return (self.nc, self.ny, self.nx) if self.dim == 2 else (self.nc, self.nz, self.ny, self.nx)

    @property
    def cells(self):
        return self.nx * (self.ny if self.dim >= 2 else 1) * (self.nz if self.dim == 3 else 1)

    def c_struct(self) -> hgks_problem:
        s = hgks_problem()
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if f.name == "bc":
                s.bc = (C.c_int32 * 4)(*[int(b) for b in (list(v) + [0] * 4)[:4]])
            elif f.name == "bcz":
                s.bcz = (C.c_int32 * 2)(*[int(b) for b in (list(v) + [0] * 2)[:2]])
            elif f.name == "stepper":
                if v is not None:
                    s.stepper = (Stepper(**v) if isinstance(v, dict) else v).c_struct()
            elif f.name == "bcd":
                for k, d in enumerate(list(v)[:4]):
                    if isinstance(d, dict):
                        d = BcData(**d)
                    if d is not None:
                        s.bcd[k] = hgks_bc_data((C.c_double * 4)(*d.a), (C.c_double * 4)(*d.b), d.s0, d.sn,
                                                d.st, int(d.rest), 0)
            else:
                setattr(s, f.name, v)
        return s


_lib = None


def lib():
    """The loaded libhgks.so; raises HgksLibraryMissing if it was never built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; load it first so that the process holds
        # one runtime, which libhgks.so then binds to (device memory and streams are torch's)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise HgksLibraryMissing(f"{LIB_PATH} is missing: build it with paper_2304_05572_amd/build.py "
                                     "(hipcc, gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "hgks_create": (i32, [C.POINTER(hgks_problem), i32, C.POINTER(hgks_opts), C.POINTER(vp)]),
            "hgks_workspace_bytes": (C.c_size_t, [vp]),
            "hgks_bind_workspace": (i32, [vp, vp, C.c_size_t]),
            "hgks_set_ic": (i32, [vp, i32, vp, i32, d]),
            "hgks_step": (i32, [vp, vp]),
            "hgks_run": (i32, [vp, vp, i64, vp]),
            "hgks_get_state": (i32, [vp, i32, vp, i32, vp]),
            "hgks_get_state_lo": (i32, [vp, i32, vp, i32]),
            "hgks_debug_flags": (i32, [vp, i32, vp, vp]),
            "hgks_debug_stage_fluxes": (i32, [vp, i32, d, vp, vp, vp, vp]),
            "hgks_debug_flags3": (i32, [vp, i32, vp, vp, vp]),
            "hgks_debug_stage_fluxes3": (i32, [vp, i32, d, vp, vp, vp, vp, vp, vp]),
            "hgks_get_stats": (i32, [vp, i32, vp]),
            "hgks_get_tile": (i32, [vp, vp]),
            "hgks_get_profile": (i32, [vp, vp]),
            "hgks_destroy": (None, [vp]),
            "hgks_status_str": (C.c_char_p, [i32]),
            "hgks_step_noalloc": (i32, [C.POINTER(hgks_problem), i32, vp, d, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ------------------------------------------------------------------ one-to-one wrappers of the C ABI
def _addr(buf):
    """(address, on_device) of a numpy array or a torch tensor."""
    if hasattr(buf, "data_ptr"):
        return C.c_void_p(buf.data_ptr()), int(buf.is_cuda)
    return buf.ctypes.data_as(C.c_void_p), 0


def _check(code: int, where: str):
    if code != OK:
        raise HgksError(code, where)


def hgks_status_str(code: int) -> str:
    return lib().hgks_status_str(int(code)).decode()


def hgks_create(problems: Sequence[Problem], precision=FP64, autotune=0, use_graph=0, tile=-1, hip_stream=None,
                profile=0, compensated=0):
    arr = (hgks_problem * len(problems))(*[p.c_struct() for p in problems])
    opts = hgks_opts(int(precision), int(autotune), int(use_graph), int(tile), int(profile), int(compensated),
                     C.c_void_p(hip_stream) if hip_stream else None)
    h = C.c_void_p()
    _check(lib().hgks_create(arr, len(problems), C.byref(opts), C.byref(h)), "hgks_create")
    return h


def hgks_workspace_bytes(h) -> int:
    return int(lib().hgks_workspace_bytes(h))


def hgks_bind_workspace(h, buf, nbytes: int):
    if hasattr(buf, "is_cuda") and buf.is_cuda:
        # torch's allocator may hand out memory that earlier work on torch's stream still uses
        import torch
        torch.cuda.current_stream(buf.device).synchronize()
    ptr, _ = _addr(buf)
    _check(lib().hgks_bind_workspace(h, ptr, int(nbytes)), "hgks_bind_workspace")


def hgks_set_ic(h, prob: int, W, t0: float = 0.0):
    if not hasattr(W, "data_ptr"):
        W = np.ascontiguousarray(W, dtype=np.float64)
    elif W.is_cuda:
        # the library's stream does not wait for torch's: make the tensor's producer finish first
        import torch
        torch.cuda.current_stream(W.device).synchronize()
    ptr, dev = _addr(W)
    _check(lib().hgks_set_ic(h, int(prob), ptr, dev, float(t0)), "hgks_set_ic")


def hgks_step(h, nprob: int):
    dt = np.zeros(nprob)
    _check(lib().hgks_step(h, dt.ctypes.data_as(C.c_void_p)), "hgks_step")
    return dt


def hgks_run(h, t_end, max_steps: int):
    t_end = np.ascontiguousarray(t_end, dtype=np.float64)
    steps = np.zeros(len(t_end), np.int64)
    _check(lib().hgks_run(h, t_end.ctypes.data_as(C.c_void_p), int(max_steps), steps.ctypes.data_as(C.c_void_p)),
           "hgks_run")
    return steps


def hgks_get_state(h, prob: int, out):
    t = C.c_double()
    ptr, dev = _addr(out)
    _check(lib().hgks_get_state(h, int(prob), ptr, dev, C.byref(t)), "hgks_get_state")
    return t.value


def hgks_get_state_lo(h, prob: int, out):
    ptr, dev = _addr(out)
    _check(lib().hgks_get_state_lo(h, int(prob), ptr, dev), "hgks_get_state_lo")


def hgks_debug_flags(h, prob: int, fx: np.ndarray, fy: np.ndarray | None):
    _check(lib().hgks_debug_flags(h, int(prob), fx.ctypes.data_as(C.c_void_p),
                                  fy.ctypes.data_as(C.c_void_p) if fy is not None else None), "hgks_debug_flags")


def hgks_debug_stage_fluxes(h, prob: int, dt: float, Fx, Gx, Fy, Gy):
    ptrs = [a.ctypes.data_as(C.c_void_p) if a is not None else None for a in (Fx, Gx, Fy, Gy)]
    _check(lib().hgks_debug_stage_fluxes(h, int(prob), float(dt), *ptrs), "hgks_debug_stage_fluxes")


def hgks_debug_flags3(h, prob: int, fx: np.ndarray, fy: np.ndarray, fz: np.ndarray):
    _check(lib().hgks_debug_flags3(h, int(prob), *[a.ctypes.data_as(C.c_void_p) for a in (fx, fy, fz)]),
           "hgks_debug_flags3")


def hgks_debug_stage_fluxes3(h, prob: int, dt: float, Fx, Gx, Fy, Gy, Fz, Gz):
    ptrs = [a.ctypes.data_as(C.c_void_p) for a in (Fx, Gx, Fy, Gy, Fz, Gz)]
    _check(lib().hgks_debug_stage_fluxes3(h, int(prob), float(dt), *ptrs), "hgks_debug_stage_fluxes3")


STATS_ENTRIES = 10


def hgks_get_stats(h, prob: int):
    out = np.zeros(STATS_ENTRIES)
    _check(lib().hgks_get_stats(h, int(prob), out.ctypes.data_as(C.c_void_p)), "hgks_get_stats")
    return out


def hgks_step_noalloc(problem: Problem, precision, W, t: float, hip_stream=None) -> float:
    """One step of a single problem without a handle or any allocation (hgks_step_noalloc): W is a device
    tensor of the problem's cell averages, advanced in place; returns the step's dt."""
    if not (hasattr(W, "is_cuda") and W.is_cuda):
        raise ValueError("hgks_step_noalloc takes a device tensor")
    ps = problem.c_struct()
    dt = C.c_double()
    sp = None
    if hip_stream is not None:
        sp = C.c_void_p(hip_stream.cuda_stream if hasattr(hip_stream, "cuda_stream") else int(hip_stream))
    _check(lib().hgks_step_noalloc(C.byref(ps), int(precision), C.c_void_p(W.data_ptr()), float(t), C.byref(dt), sp),
           "hgks_step_noalloc")
    return dt.value


def hgks_get_tile(h):
    """(interfaces along the normal, rows along the tangential direction, waves-per-SIMD target,
    configuration index, persistent grid blocks or 0)."""
    out = np.zeros(5, np.int32)
    _check(lib().hgks_get_tile(h, out.ctypes.data_as(C.c_void_p)), "hgks_get_tile")
    return tuple(int(x) for x in out)


def hgks_get_profile(h):
    out = np.zeros(8)
    _check(lib().hgks_get_profile(h, out.ctypes.data_as(C.c_void_p)), "hgks_get_profile")
    return out


def hgks_destroy(h):
    lib().hgks_destroy(h)


# ------------------------------------------------------------------ convenience wrapper
class Solver:
    """Owns one library handle for a list of problems advanced together."""

    def __init__(self, problems: Sequence[Problem] | Problem, precision=FP64, autotune=False, use_graph=False,
                 tile=-1, stream=None, workspace=None, profile=False, compensated=False):
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems = list(problems)
        sp = None
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.h = hgks_create(self.problems, precision, int(autotune), int(use_graph), tile, sp, int(profile),
                             int(compensated))
        self.workspace = None
        if workspace is not None:
            self.bind_workspace(workspace)

    @property
    def nprob(self):
        return len(self.problems)

    def workspace_bytes(self):
        return hgks_workspace_bytes(self.h)

    def bind_workspace(self, buf):
        """Use caller-owned device memory, e.g. torch.empty(n, dtype=torch.uint8, device='cuda')."""
        hgks_bind_workspace(self.h, buf, buf.numel() * buf.element_size())
        self.workspace = buf  # keep the owner alive

    def set_ic(self, prob: int, W, t0: float = 0.0):
        hgks_set_ic(self.h, prob, W, t0)

    def step(self):
        return hgks_step(self.h, self.nprob)

    def run(self, t_end, max_steps: int = 2 ** 62):
        if np.isscalar(t_end):
            t_end = [t_end] * self.nprob
        return hgks_run(self.h, t_end, max_steps)

    def get_state(self, prob: int = 0, out=None):
        if out is None:
            out = np.zeros(self.problems[prob].shape)
        t = hgks_get_state(self.h, prob, out)
        return out, t

    def get_state_lo(self, prob: int = 0, out=None):
        """Low-order part E of the carried state W + E (zeros unless compensated)."""
        if out is None:
            out = np.zeros(self.problems[prob].shape)
        hgks_get_state_lo(self.h, prob, out)
        return out

    def flags(self, prob: int = 0):
        P = self.problems[prob]
        if P.dim == 3:
            fx, fy, fz = (np.zeros((P.nz, P.ny, P.nx), np.uint8) for _ in range(3))
            hgks_debug_flags3(self.h, prob, fx, fy, fz)
            return fx, fy, fz
        shp = (P.nx,) if P.dim == 1 else (P.ny, P.nx)
        fx = np.zeros(shp, np.uint8)
        fy = np.zeros(shp, np.uint8) if P.dim == 2 else None
        hgks_debug_flags(self.h, prob, fx, fy)
        return fx, fy

    def stage_fluxes(self, prob: int, dt: float):
        """(F, G) per direction at the interfaces: F the time-averaged flux and G its time derivative."""
        P = self.problems[prob]
        if P.dim == 3:
            nx, ny, nz = P.nx, P.ny, P.nz
            Fx, Gx = np.zeros((5, nz, ny, nx + 1)), np.zeros((5, nz, ny, nx + 1))
            Fy, Gy = np.zeros((5, nz, ny + 1, nx)), np.zeros((5, nz, ny + 1, nx))
            Fz, Gz = np.zeros((5, nz + 1, ny, nx)), np.zeros((5, nz + 1, ny, nx))
            hgks_debug_stage_fluxes3(self.h, prob, dt, Fx, Gx, Fy, Gy, Fz, Gz)
            return (Fx, Gx), (Fy, Gy), (Fz, Gz)
        nc, nx, ny = P.nc, P.nx, (P.ny if P.dim == 2 else 1)
        Fx = np.zeros((nc, ny, nx + 1))
        Gx = np.zeros_like(Fx)
        Fy = np.zeros((nc, ny + 1, nx)) if P.dim == 2 else None
        Gy = np.zeros_like(Fy) if P.dim == 2 else None
        hgks_debug_stage_fluxes(self.h, prob, dt, Fx, Gx, Fy, Gy)
        if P.dim == 1:
            return Fx[:, 0, :], Gx[:, 0, :], None, None
        return Fx, Gx, Fy, Gy

    def stats(self, prob: int = 0):
        """Counters of problem `prob`; bad_stage / bad_cell name the first non-physical state (stage 0 and
        cell -1 while there is none); seconds is the handle's wall time in step / run."""
        s = hgks_get_stats(self.h, prob)
        return dict(steps=int(s[0]), cells=int(s[1]), t=s[2], dt=s[3], flagged_x=s[4], flagged_y=s[5],
                    flagged_z=s[6], bad_stage=int(s[7]), bad_cell=int(s[8]), seconds=s[9])

    def tile(self):
        return hgks_get_tile(self.h)

    def profile(self):
        """Per kernel group: (total ms, launches) for flux, update, flags, scalar kernels (profile=1 times
        the flux launches only, profile=2 every launch)."""
        o = hgks_get_profile(self.h)
        names = ("flux", "update", "flags", "scalar")
        return {n: (o[2 * k], int(o[2 * k + 1])) for k, n in enumerate(names)}

    def close(self):
        if self.h:
            hgks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
