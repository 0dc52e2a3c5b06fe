"""Python binding of libhydro.so: argument marshalling only.

Every function takes torch tensors that live on the current HIP device and
passes their pointers, plus torch's current stream, to the C ABI declared in
include/hydro.h.  All arithmetic happens in the HIP kernels; if the library is
not built, every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhydro.so")

HYDRO_OK = 0
HYDRO_EINVAL = -1
HYDRO_EDEVICE = -2
F64, F32 = 0, 1
SCHEME_MHM_PLM_HLLC = 1
WAVESPEED_ROE = 0 << 8
WAVESPEED_DAVIS = 1 << 8
FIRST_ORDER = 1 << 10
BC_PERIODIC, BC_OUTFLOW = 0, 1

_lib = None


class HydroError(RuntimeError):
    def __init__(self, fn: str, status: int):
        lib = load()
        msg = lib.hydro_strerror(status).decode()
        if status == HYDRO_EDEVICE:
            msg += " (hipError_t %d)" % lib.hydro_last_hip_error()
        super().__init__("%s: %s" % (fn, msg))
        self.status = status


def load():
    """Load libhydro.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhydro.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "hydro_advance": (i32, [P, P, i64, i32, i32, f64, f64, f64, i32, f64, P, P, P]),
        "hydro_advance_level": (i32, [P, P, i32, i32, i32, P, i32, f64, f64, f64, i32, f64, P, P, f64, P, P, P,
                                      P]),
        "hydro_dt": (i32, [P, i64, i32, i32, f64, f64, f64, P, P, P]),
        "hydro_fill_ghosts": (i32, [P, P, i32, i32, i32, i32, i32, P, P]),
        "hydro_num_variants": (i32, []),
        "hydro_set_variant": (i32, [i32, i32]),
        "hydro_get_variant": (i32, [i32]),
        "hydro_variant_name": (i32, [i32, ctypes.c_char_p, i32]),
        "hydro_autotune": (i32, [P, P, i32, i32, i32, P, i32, f64, f64, i32, P, P]),
        "hydro_strerror": (ctypes.c_char_p, [i32]),
        "hydro_last_hip_error": (i32, []),
        "hydro_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("state tensors must be float64 or float32, got %s" % t.dtype)


def _dev(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _opt(t: Optional[torch.Tensor], name: str, dtype) -> Optional[int]:
    if t is None:
        return None
    if t.dtype != dtype or t.numel() < 1:
        raise ValueError("%s must be a %s tensor with at least one element" % (name, dtype))
    return _dev(t, name)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check(status: int, fn: str):
    if status != HYDRO_OK:
        raise HydroError(fn, status)


def ghost_of(U_pad: torch.Tensor) -> int:
    P = U_pad.shape[-1]
    if U_pad.dim() != 5 or U_pad.shape[1] != 5 or tuple(U_pad.shape[2:]) != (P, P, P) or (P - 16) % 2:
        raise ValueError("padded groups must have shape [G, 5, P, P, P] with P = 16 + 2*ghost")
    return (P - 16) // 2


# --------------------------------------------------------------- entry points --

def advance(U_pad: torch.Tensor, dt: float, dx: float, gamma: float, theta: float = 1.5,
            scheme: int = SCHEME_MHM_PLM_HLLC, out: Optional[torch.Tensor] = None,
            n_bad: Optional[torch.Tensor] = None, dt_dev: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One MHM step: U_pad[G,5,P,P,P] -> U_out[G,5,16,16,16] (hydro_advance)."""
    gh = ghost_of(U_pad)
    G = U_pad.shape[0]
    if out is None:
        out = torch.empty((G, 5, 16, 16, 16), dtype=U_pad.dtype, device=U_pad.device)
    if out.dtype != U_pad.dtype or tuple(out.shape) != (G, 5, 16, 16, 16):
        raise ValueError("out must be [G,5,16,16,16] of the input dtype")
    st = load().hydro_advance(_dev(U_pad, "U_pad"), _dev(out, "out"), G, gh, _dtype_code(U_pad), float(dt),
                              float(dx), float(gamma), int(scheme), float(theta),
                              _opt(dt_dev, "dt_dev", torch.float64), _opt(n_bad, "n_bad", torch.int32), _stream())
    _check(st, "hydro_advance")
    return out


def advance_level(level: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dt: float, dx: float, gamma: float,
                  theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC, out: Optional[torch.Tensor] = None,
                  n_bad: Optional[torch.Tensor] = None, dt_dev: Optional[torch.Tensor] = None, c_cfl: float = 0.5,
                  dt_next: Optional[torch.Tensor] = None, dt_patch_next: Optional[torch.Tensor] = None,
                  dt_reset: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One MHM step of a whole level read from level storage (hydro_advance_level)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level.shape) != (G, 5, 16, 16, 16):
        raise ValueError("level must be [G,5,16,16,16] with G = ngx*ngy*ngz")
    if out is None:
        out = torch.empty_like(level)
    if out.dtype != level.dtype or out.shape != level.shape:
        raise ValueError("out must match the level")
    if dt_patch_next is not None and (dt_patch_next.dtype != torch.float64 or dt_patch_next.numel() != 8 * G):
        raise ValueError("dt_patch_next must hold G*8 float64")
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_advance_level(_dev(level, "level"), _dev(out, "out"), ngx, ngy, ngz, b, _dtype_code(level),
                                    float(dt), float(dx), float(gamma), int(scheme), float(theta),
                                    _opt(dt_dev, "dt_dev", torch.float64), _opt(n_bad, "n_bad", torch.int32),
                                    float(c_cfl), _opt(dt_next, "dt_next", torch.float64),
                                    _opt(dt_patch_next, "dt_patch_next", torch.float64),
                                    _opt(dt_reset, "dt_reset", torch.float64), _stream())
    _check(st, "hydro_advance_level")
    return out


def cfl_dt(U_pad: torch.Tensor, dx: float, gamma: float, c_cfl: float = 0.5, out: Optional[torch.Tensor] = None,
           dt_min: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-patch CFL time-step (hydro_dt): returns dt_patch[G, 8] (float64)."""
    gh = ghost_of(U_pad)
    G = U_pad.shape[0]
    if out is None:
        out = torch.empty((G, 8), dtype=torch.float64, device=U_pad.device)
    if out.dtype != torch.float64 or out.numel() != 8 * G:
        raise ValueError("out must hold G*8 float64")
    st = load().hydro_dt(_dev(U_pad, "U_pad"), G, gh, _dtype_code(U_pad), float(dx), float(gamma), float(c_cfl),
                         _dev(out, "out"), _opt(dt_min, "dt_min", torch.float64), _stream())
    _check(st, "hydro_dt")
    return out


def fill_ghosts(level: torch.Tensor, ng: Sequence[int], ghost: int, bc: Sequence[int],
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Level storage [G,5,16,16,16] -> padded groups [G,5,P,P,P] (hydro_fill_ghosts)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level.shape) != (G, 5, 16, 16, 16):
        raise ValueError("level must be [G,5,16,16,16] with G = ngx*ngy*ngz")
    P = 16 + 2 * int(ghost)
    if out is None:
        out = torch.empty((G, 5, P, P, P), dtype=level.dtype, device=level.device)
    if out.dtype != level.dtype or tuple(out.shape) != (G, 5, P, P, P):
        raise ValueError("out must be [G,5,P,P,P] of the level dtype")
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_fill_ghosts(_dev(level, "level"), _dev(out, "out"), ngx, ngy, ngz, int(ghost),
                                  _dtype_code(level), b, _stream())
    _check(st, "hydro_fill_ghosts")
    return out


# ------------------------------------------------------------- launch shapes --

def num_variants() -> int:
    return int(load().hydro_num_variants())


def variant_name(v: int) -> str:
    buf = ctypes.create_string_buffer(128)
    _check(load().hydro_variant_name(int(v), buf, 128), "hydro_variant_name")
    return buf.value.decode()


def set_variant(dtype, v: int) -> None:
    _check(load().hydro_set_variant(F64 if dtype == torch.float64 else F32, int(v)), "hydro_set_variant")


def get_variant(dtype) -> int:
    return int(load().hydro_get_variant(F64 if dtype == torch.float64 else F32))


def autotune(level: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dx: float, gamma: float,
             reps: int = 5) -> Tuple[int, list]:
    """Time every launch shape on this level, select the fastest (hydro_autotune).

    Returns (chosen variant, mean ms per variant)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    scratch = torch.empty_like(level)
    n = num_variants()
    times = (ctypes.c_float * n)()
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_autotune(_dev(level, "level"), _dev(scratch, "scratch"), ngx, ngy, ngz, b, _dtype_code(level),
                               float(dx), float(gamma), int(reps), times, _stream())
    if st < 0:
        raise HydroError("hydro_autotune", st)
    return int(st), list(times)


# -------------------------------------------------------------- level driver --

class LevelSolver:
    """Device-resident driver for one level: buffers are allocated once and
    every step stays on the device, the time-step travelling between kernels
    in device memory.

    fused=True (default): one hydro_advance_level launch per step; it reads
    neighbour groups directly and reduces the CFL time-step of its output for
    the next step (three rotating device scalars: read, reduce, reset).
    fused=False: hydro_fill_ghosts + hydro_dt + hydro_advance per step."""

    def __init__(self, ng: Sequence[int], dx: float, gamma: float, bc: Sequence[int] = (0,) * 6,
                 ghost: int = 3, dtype=torch.float64, theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC,
                 c_cfl: float = 0.5, device=None, fused: bool = True):
        self.ng = tuple(int(v) for v in ng)
        self.G = self.ng[0] * self.ng[1] * self.ng[2]
        self.dx, self.gamma, self.bc, self.ghost = float(dx), float(gamma), tuple(bc), int(ghost)
        self.theta, self.scheme, self.c_cfl = float(theta), int(scheme), float(c_cfl)
        self.fused = bool(fused)
        dev = torch.device("cuda") if device is None else torch.device(device)
        P = 16 + 2 * self.ghost
        self.pad = None if self.fused else torch.empty((self.G, 5, P, P, P), dtype=dtype, device=dev)
        self.bufs = [torch.empty((self.G, 5, 16, 16, 16), dtype=dtype, device=dev) for _ in range(2)]
        self.dt_patch = torch.empty((self.G, 8), dtype=torch.float64, device=dev)
        self.dts = torch.full((3,), float("inf"), dtype=torch.float64, device=dev)  # rotating dt scalars
        self.dt_min = self.dts[0:1]
        self.n_bad = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cur = 0
        self.turn = 0
        self.primed = False

    def load_state(self, level: torch.Tensor):
        self.bufs[self.cur].copy_(level)
        self.primed = False

    @property
    def state(self) -> torch.Tensor:
        return self.bufs[self.cur]

    def _prime(self):
        """CFL time-step of the loaded state into the current dt scalar."""
        a = self.dts[self.turn:self.turn + 1]
        # level storage is the padded layout with zero ghost zones
        cfl_dt(self.bufs[self.cur], self.dx, self.gamma, self.c_cfl, out=self.dt_patch, dt_min=a)
        self.dts[(self.turn + 1) % 3:(self.turn + 1) % 3 + 1].fill_(float("inf"))
        self.primed = True

    def step(self, dt: Optional[float] = None, events=None) -> None:
        """One step: fixed dt if given, else the CFL time-step of the current state.

        events: optional (start, end) torch.cuda.Event pair recorded on the
        current stream around the MHM update.  After a CFL step, dt_min views
        the time-step that step used."""
        nxt = self.bufs[1 - self.cur]
        stream = torch.cuda.current_stream()
        if self.fused:
            if dt is None and not self.primed:
                self._prime()
            a = self.dts[self.turn:self.turn + 1]
            b = self.dts[(self.turn + 1) % 3:(self.turn + 1) % 3 + 1]
            c = self.dts[(self.turn + 2) % 3:(self.turn + 2) % 3 + 1]
            if events is not None:
                events[0].record(stream)
            if dt is None:
                advance_level(self.bufs[self.cur], self.ng, self.bc, 1.0, self.dx, self.gamma, self.theta,
                              self.scheme, out=nxt, n_bad=self.n_bad, dt_dev=a, c_cfl=self.c_cfl, dt_next=b,
                              dt_reset=c)
                self.dt_min = a
                self.turn = (self.turn + 1) % 3
            else:
                advance_level(self.bufs[self.cur], self.ng, self.bc, dt, self.dx, self.gamma, self.theta,
                              self.scheme, out=nxt, n_bad=self.n_bad)
                self.primed = False
            if events is not None:
                events[1].record(stream)
        else:
            fill_ghosts(self.bufs[self.cur], self.ng, self.ghost, self.bc, out=self.pad)
            dt_dev = None
            if dt is None:
                self.dt_min = self.dts[0:1]
                cfl_dt(self.pad, self.dx, self.gamma, self.c_cfl, out=self.dt_patch, dt_min=self.dt_min)
                dt, dt_dev = 1.0, self.dt_min
            if events is not None:
                events[0].record(stream)
            advance(self.pad, dt, self.dx, self.gamma, self.theta, self.scheme, out=nxt, n_bad=self.n_bad,
                    dt_dev=dt_dev)
            if events is not None:
                events[1].record(stream)
        self.cur = 1 - self.cur
