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
HYDRO_UNPHYSICAL = 1
HYDRO_EINVAL = -1
HYDRO_EDEVICE = -2
HYDRO_ENOTUNED = -3
HYDRO_EIO = -4
F64, F32 = 0, 1
SCHEME_MHM_PLM_HLLC = 1
WAVESPEED_ROE = 0 << 8
WAVESPEED_DAVIS = 1 << 8
FIRST_ORDER = 1 << 10
BC_PERIODIC, BC_OUTFLOW = 0, 1
# scheme-word fields of hydro_advance_ext (include/hydro.h)
SCHEME_MHM, SCHEME_CTU = 1, 2
LIMITER_GMINMOD, LIMITER_VANLEER, LIMITER_VANALBADA, LIMITER_HYBRID = 0 << 11, 1 << 11, 2 << 11, 3 << 11
CHARACTERISTIC = 1 << 13
PPM = 1 << 14
RIEMANN_HLLC, RIEMANN_ROE, RIEMANN_HLLE = 0 << 16, 1 << 16, 2 << 16
DUAL_ENERGY = 1 << 18
BATCH_WORK_WORDS = 16       # uint32 words of the batched kernel's work buffer
BATCHED_VARIANTS = 16       # launch shapes of the batched kernel

_lib = None


class HydroLevel(ctypes.Structure):
    """hydro_level_t of include/hydro.h."""
    _fields_ = [("level_dev", ctypes.c_void_p), ("level_out_dev", ctypes.c_void_p), ("ngx", ctypes.c_int32),
                ("ngy", ctypes.c_int32), ("ngz", ctypes.c_int32), ("bc", ctypes.c_int32 * 6), ("dt", ctypes.c_double),
                ("dx", ctypes.c_double), ("dt_dev", ctypes.c_void_p), ("dt_dev_scale", ctypes.c_double),
                ("c_cfl", ctypes.c_double), ("dt_next_scale", ctypes.c_double), ("dt_next_dev", ctypes.c_void_p),
                ("dt_patch_next_dev", ctypes.c_void_p), ("dt_reset_dev", ctypes.c_void_p)]


class HydroAmrLevel(ctypes.Structure):
    """hydro_amr_level_t of include/hydro.h."""
    _fields_ = [("U_dev", ctypes.c_void_p), ("pos_dev", ctypes.c_void_p), ("map_dev", ctypes.c_void_p),
                ("n_groups", ctypes.c_int64), ("n", ctypes.c_int32 * 3)]


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
        "hydro_ctx_create": (i32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_char_p]),
        "hydro_ctx_destroy": (i32, [P]),
        "hydro_ctx_save": (i32, [P]),
        "hydro_ctx_set_require_tuned": (i32, [P, i32]),
        "hydro_ctx_num_tuned": (i32, [P]),
        "hydro_check_unphysical": (i32, [P, P, P]),
        "hydro_advance": (i32, [P, P, i64, i32, i32, f64, f64, f64, i32, f64, P, P, P]),
        "hydro_branch_record": (i32, [P, P, i64, i32, i32, f64, f64, f64, i32, f64, P, P]),
        "hydro_ext_workspace_bytes": (i64, [i64, i32, i32, i32]),
        "hydro_advance_ext": (i32, [P, P, i64, i32, i32, f64, f64, f64, i32, f64, f64, P, P, P, i64, P, P]),
        "hydro_repair_unphysical": (i32, [P, P, i32, i32, i32, P, i32, f64, f64, f64, i32, P, P, P]),
        "hydro_fallback_workspace_bytes": (i64, [i32, i32, i32, i32, i32]),
        "hydro_advance_level_fallback": (i32, [P, P, P, i32, i32, i32, P, i32, f64, f64, f64, f64, f64, i32, f64,
                                               P, i64, P, P]),
        "hydro_amr_fill_ghosts": (i32, [P, P, P, P, f64, P, i32, i32, P, P]),
        "hydro_amr_flux_accumulate": (i32, [P, P, f64, P, i32, P, P]),
        "hydro_amr_restrict": (i32, [P, P, i32, P]),
        "hydro_amr_fixup": (i32, [P, P, P, P, f64, P, i32, P]),
        "hydro_advance_level": (i32, [P, P, P, i32, i32, i32, P, i32, f64, f64, f64, i32, f64, P, P, f64, P, P, P,
                                      P]),
        "hydro_dt": (i32, [P, i64, i32, i32, f64, f64, f64, P, P, P]),
        "hydro_fill_ghosts": (i32, [P, P, i32, i32, i32, i32, i32, P, P]),
        "hydro_gather_ghost_adjoint": (i32, [P, P, i32, i32, i32, i32, i32, P, P]),
        "hydro_num_variants": (i32, []),
        "hydro_set_variant": (i32, [P, i32, i32]),
        "hydro_set_level_variant": (i32, [P, i32, i32, i32]),
        "hydro_get_level_variant": (i32, [P, i32, i32]),
        "hydro_set_adjoint_variant": (i32, [P, i32, i32]),
        "hydro_get_adjoint_variant": (i32, [P, i32]),
        "hydro_get_variant": (i32, [P, i32]),
        "hydro_variant_name": (i32, [i32, ctypes.c_char_p, i32]),
        "hydro_autotune": (i32, [P, P, P, i32, i32, i32, P, i32, f64, f64, P, i64, i32, P, P]),
        "hydro_advance_batched": (i32, [P, P, i32, i32, f64, i32, f64, P, P, i32, P]),
        "hydro_advance_batched_noalloc": (i32, [P, P, i32, i32, f64, i32, f64, P, i32, P]),
        "hydro_set_batched_variant": (i32, [P, i32, i32]),
        "hydro_get_batched_variant": (i32, [P, i32]),
        "hydro_autotune_batched": (i32, [P, P, i32, i32, f64, P, i32, P, P]),
        "hydro_autotune_adjoint": (i32, [P, P, P, P, i32, i32, i32, P, i32, f64, f64, P, i64, i32, P, P]),
        "hydro_graph_begin": (i32, [P]),
        "hydro_graph_end": (i32, [P, P, ctypes.POINTER(ctypes.c_void_p)]),
        "hydro_graph_launch": (i32, [P, P]),
        "hydro_graph_destroy": (i32, [P, P]),
        "hydro_adjoint_workspace_bytes": (i64, [i64, i32, i32]),
        "hydro_advance_adjoint": (i32, [P, P, P, P, i64, i32, i32, f64, f64, f64, i32, f64, P, i64, P]),
        "hydro_advance_level_adjoint": (i32, [P, P, P, P, i32, i32, i32, P, i32, f64, f64, f64, i32, f64, P, P, i64,
                                              P]),
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


class Context:
    """A solver context (hydro_ctx): launch-shape selections, explicit or
    autotuned per dtype and lattice, optionally persisted in a tuning-cache
    JSON file, and the graphs captured through it."""

    def __init__(self, tune_cache: Optional[str] = None, require_tuned: bool = False):
        lib = load()
        h = ctypes.c_void_p()
        st = lib.hydro_ctx_create(ctypes.byref(h), None if tune_cache is None else os.fsencode(tune_cache))
        _check(st, "hydro_ctx_create")
        self.handle = h
        if require_tuned:
            _check(lib.hydro_ctx_set_require_tuned(h, 1), "hydro_ctx_set_require_tuned")

    def save(self) -> None:
        _check(load().hydro_ctx_save(self.handle), "hydro_ctx_save")

    def num_tuned(self) -> int:
        n = load().hydro_ctx_num_tuned(self.handle)
        if n < 0:
            raise HydroError("hydro_ctx_num_tuned", n)
        return int(n)

    def close(self) -> None:
        if self.handle is not None:
            load().hydro_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Optional[Context] = None


def default_context() -> Context:
    """The module's context, used by every call given ctx=None."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _ctx(ctx: Optional[Context]):
    return (ctx if ctx is not None else default_context()).handle


def check_unphysical(n_bad: torch.Tensor) -> int:
    """Wait for the current stream and return the unphysical count held in the
    device int32 n_bad (hydro_check_unphysical)."""
    if n_bad.dtype != torch.int32 or n_bad.numel() < 1:
        raise ValueError("n_bad must be an int32 tensor")
    v = ctypes.c_int32()
    st = load().hydro_check_unphysical(_dev(n_bad, "n_bad"), _stream(), ctypes.byref(v))
    if st not in (HYDRO_OK, HYDRO_UNPHYSICAL):
        raise HydroError("hydro_check_unphysical", st)
    return int(v.value)


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


def branch_record(U_pad: torch.Tensor, dt: float, dx: float, gamma: float, theta: float = 1.5,
                  scheme: int = SCHEME_MHM_PLM_HLLC, out: Optional[torch.Tensor] = None,
                  record: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """advance (FP64) that also returns every group's branch record, an int32
    [G] device tensor (hydro_branch_record): equal records, equal branches."""
    gh = ghost_of(U_pad)
    G = U_pad.shape[0]
    if U_pad.dtype != torch.float64:
        raise ValueError("branch_record runs in FP64")
    if out is None:
        out = torch.empty((G, 5, 16, 16, 16), dtype=U_pad.dtype, device=U_pad.device)
    if record is None:
        record = torch.empty(G, dtype=torch.int32, device=U_pad.device)
    if out.dtype != U_pad.dtype or tuple(out.shape) != (G, 5, 16, 16, 16):
        raise ValueError("out must be [G,5,16,16,16] of the input dtype")
    if record.dtype != torch.int32 or record.numel() < G:
        raise ValueError("record must hold G int32")
    st = load().hydro_branch_record(_dev(U_pad, "U_pad"), _dev(out, "out"), G, gh, _dtype_code(U_pad), float(dt),
                                    float(dx), float(gamma), int(scheme), float(theta), _dev(record, "record"),
                                    _stream())
    _check(st, "hydro_branch_record")
    return out, record


def ext_workspace(n_groups: int, ghost: int, dtype, scheme: int, device="cuda") -> torch.Tensor:
    """A uint8 device workspace for hydro_advance_ext on n_groups groups."""
    nb = load().hydro_ext_workspace_bytes(int(n_groups), int(ghost), F64 if dtype == torch.float64 else F32,
                                          int(scheme))
    if nb < 0:
        raise HydroError("hydro_ext_workspace_bytes", int(nb))
    return torch.empty(max(int(nb), 1), dtype=torch.uint8, device=device)


def advance_ext(U_pad: torch.Tensor, dt: float, dx: float, gamma: float, scheme: int, theta: float = 1.5,
                out: Optional[torch.Tensor] = None, n_bad: Optional[torch.Tensor] = None,
                dt_dev: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None,
                face_flux: Optional[torch.Tensor] = None, xi: float = 0.01) -> torch.Tensor:
    """One step of any scheme word (MHM / CTU, PLM / PPM, primitive /
    characteristic, any limiter, HLLC / Roe / HLLE): U_pad[G,5,P,P,P] ->
    U_out[G,5,16,16,16] (hydro_advance_ext).  work: uint8 device tensor of at
    least hydro_ext_workspace_bytes(1, ...) bytes (default: enough for all
    groups at once).  face_flux: optional [G,9,5,16,16] output, the fluxes
    on the patch-boundary faces (flux registers of coarse-fine coupling).
    With DUAL_ENERGY the arrays have 6 fields (field 5 the entropy s = p /
    rho^(gamma-1)) and xi is the dual-energy threshold."""
    G = U_pad.shape[0]
    nf = 6 if scheme & DUAL_ENERGY else 5
    if U_pad.dim() != 5 or U_pad.shape[1] != nf or U_pad.shape[2] != U_pad.shape[3] or \
            U_pad.shape[3] != U_pad.shape[4] or (U_pad.shape[2] - 16) % 2:
        raise ValueError("U_pad must be [G,%d,P,P,P]" % nf)
    gh = (U_pad.shape[2] - 16) // 2
    if out is None:
        out = torch.empty((G, nf, 16, 16, 16), dtype=U_pad.dtype, device=U_pad.device)
    if out.dtype != U_pad.dtype or tuple(out.shape) != (G, nf, 16, 16, 16):
        raise ValueError("out must be [G,%d,16,16,16] of the input dtype" % nf)
    if work is None:
        work = ext_workspace(G, gh, U_pad.dtype, scheme, U_pad.device)
    if work.dtype != torch.uint8:
        raise ValueError("work must be a uint8 tensor")
    if face_flux is not None and (face_flux.dtype != U_pad.dtype or tuple(face_flux.shape) != (G, 9, 5, 16, 16)):
        raise ValueError("face_flux must be [G,9,5,16,16] of the input dtype")
    st = load().hydro_advance_ext(_dev(U_pad, "U_pad"), _dev(out, "out"), G, gh, _dtype_code(U_pad), float(dt),
                                  float(dx), float(gamma), int(scheme), float(theta), float(xi),
                                  _opt(dt_dev, "dt_dev", torch.float64), _opt(n_bad, "n_bad", torch.int32),
                                  _dev(work, "work"), work.numel(),
                                  None if face_flux is None else _dev(face_flux, "face_flux"), _stream())
    _check(st, "hydro_advance_ext")
    return out


def repair_unphysical(level_in: torch.Tensor, level_out: torch.Tensor, ng: Sequence[int], bc: Sequence[int],
                      dt: float, dx: float, gamma: float, scheme: int = SCHEME_MHM_PLM_HLLC,
                      counts: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Steps (ii)-(iii) of the procedure for unphysical results on level_out
    (hydro_repair_unphysical); returns the int32 counters [repaired unsplit,
    repaired split, still unphysical] (added to `counts` if given)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level_in.shape) != (G, 5, 16, 16, 16) or level_out.shape != level_in.shape or \
            level_out.dtype != level_in.dtype:
        raise ValueError("levels must be [G,5,16,16,16] of one dtype")
    if counts is None:
        counts = torch.zeros(3, dtype=torch.int32, device=level_in.device)
    if counts.dtype != torch.int32 or counts.numel() < 3:
        raise ValueError("counts must hold 3 int32")
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_repair_unphysical(_dev(level_in, "level_in"), _dev(level_out, "level_out"), ngx, ngy, ngz, b,
                                        _dtype_code(level_in), float(dt), float(dx), float(gamma), int(scheme), None,
                                        _dev(counts, "counts"), _stream())
    _check(st, "hydro_repair_unphysical")
    return counts


def advance_level_fallback(level: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dt: float, dx: float,
                           gamma: float, theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC, dt_min: float = 0.0,
                           ratio: float = 0.8, out: Optional[torch.Tensor] = None,
                           work: Optional[torch.Tensor] = None, ctx: Optional[Context] = None):
    """One level step with the procedure for unphysical results
    (hydro_advance_level_fallback, synchronous).  Returns (out, ok, info) with
    ok False if cells remained unphysical at the smallest dt allowed and
    info = dict(dt, retries, unsplit, split) of the last attempt."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level.shape) != (G, 5, 16, 16, 16):
        raise ValueError("level must be [G,5,16,16,16] with G = ngx*ngy*ngz")
    if out is None:
        out = torch.empty_like(level)
    if out.dtype != level.dtype or out.shape != level.shape:
        raise ValueError("out must match the level")
    code = _dtype_code(level)
    if work is None:
        nb = load().hydro_fallback_workspace_bytes(ngx, ngy, ngz, code, int(scheme))
        if nb < 0:
            raise HydroError("hydro_fallback_workspace_bytes", int(nb))
        work = torch.empty(int(nb), dtype=torch.uint8, device=level.device)
    if work.dtype != torch.uint8:
        raise ValueError("work must be a uint8 tensor")
    info = (ctypes.c_double * 4)()
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_advance_level_fallback(_ctx(ctx), _dev(level, "level"), _dev(out, "out"), ngx, ngy, ngz, b, code,
                                             float(dt), float(dt_min), float(ratio), float(dx), float(gamma),
                                             int(scheme), float(theta), _dev(work, "work"), work.numel(), info,
                                             _stream())
    if st not in (HYDRO_OK, HYDRO_UNPHYSICAL):
        raise HydroError("hydro_advance_level_fallback", st)
    return out, st == HYDRO_OK, {"dt": info[0], "retries": int(info[1]), "unsplit": int(info[2]),
                                 "split": int(info[3])}


def advance_level(level: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dt: float, dx: float, gamma: float,
                  theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC, out: Optional[torch.Tensor] = None,
                  n_bad: Optional[torch.Tensor] = None, dt_dev: Optional[torch.Tensor] = None, c_cfl: float = 0.5,
                  dt_next: Optional[torch.Tensor] = None, dt_patch_next: Optional[torch.Tensor] = None,
                  dt_reset: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
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
    st = load().hydro_advance_level(_ctx(ctx), _dev(level, "level"), _dev(out, "out"), ngx, ngy, ngz, b, _dtype_code(level),
                                    float(dt), float(dx), float(gamma), int(scheme), float(theta),
                                    _opt(dt_dev, "dt_dev", torch.float64), _opt(n_bad, "n_bad", torch.int32),
                                    float(c_cfl), _opt(dt_next, "dt_next", torch.float64),
                                    _opt(dt_patch_next, "dt_patch_next", torch.float64),
                                    _opt(dt_reset, "dt_reset", torch.float64), _stream())
    _check(st, "hydro_advance_level")
    return out


def adjoint_workspace(n_groups: int, dtype, level: bool, device=None) -> torch.Tensor:
    """Scratch buffer for the adjoint calls (bytes from hydro_adjoint_workspace_bytes)."""
    nbytes = load().hydro_adjoint_workspace_bytes(int(n_groups), F64 if dtype == torch.float64 else F32, int(level))
    if nbytes < 0:
        raise HydroError("hydro_adjoint_workspace_bytes", int(nbytes))
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def _check_work(work: Optional[torch.Tensor]) -> None:
    # the byte size is checked by the library against hydro_adjoint_workspace_bytes
    if work is not None and (work.dtype != torch.uint8 or work.dim() != 1):
        raise ValueError("work must be a 1-D uint8 tensor (adjoint_workspace)")


def advance_adjoint(U_pad: torch.Tensor, gU_out: torch.Tensor, dt: float, dx: float, gamma: float,
                    theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC, out: Optional[torch.Tensor] = None,
                    work: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Cotangent of U_pad given that of the step's output (hydro_advance_adjoint)."""
    gh = ghost_of(U_pad)
    G = U_pad.shape[0]
    if gU_out.dtype != U_pad.dtype or tuple(gU_out.shape) != (G, 5, 16, 16, 16):
        raise ValueError("gU_out must be [G,5,16,16,16] of the state dtype")
    if out is not None and (out.dtype != U_pad.dtype or out.shape != U_pad.shape):
        raise ValueError("out must be [G,5,P,P,P] of the state dtype")
    _check_work(work)
    if out is None:
        out = torch.empty_like(U_pad)
    if work is None:
        work = adjoint_workspace(G, U_pad.dtype, False, U_pad.device)
    st = load().hydro_advance_adjoint(_ctx(ctx), _dev(U_pad, "U_pad"), _dev(gU_out, "gU_out"), _dev(out, "out"), G, gh,
                                      _dtype_code(U_pad), float(dt), float(dx), float(gamma), int(scheme), float(theta),
                                      _dev(work, "work"), work.numel(), _stream())
    _check(st, "hydro_advance_adjoint")
    return out


def advance_level_adjoint(level: torch.Tensor, g_out: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dt: float,
                          dx: float, gamma: float, theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC,
                          out: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None,
                          dt_dev: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Cotangent of a level's input state given that of its stepped state (hydro_advance_level_adjoint)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level.shape) != (G, 5, 16, 16, 16) or g_out.shape != level.shape or g_out.dtype != level.dtype:
        raise ValueError("level and g_out must be [G,5,16,16,16] of one dtype")
    if out is not None and (out.dtype != level.dtype or out.shape != level.shape):
        raise ValueError("out must be [G,5,16,16,16] of the level dtype")
    _check_work(work)
    if out is None:
        out = torch.empty_like(level)
    if work is None:
        work = adjoint_workspace(G, level.dtype, True, level.device)
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_advance_level_adjoint(_ctx(ctx), _dev(level, "level"), _dev(g_out, "g_out"), _dev(out, "out"), ngx, ngy,
                                            ngz, b, _dtype_code(level), float(dt), float(dx), float(gamma),
                                            int(scheme), float(theta), _opt(dt_dev, "dt_dev", torch.float64),
                                            _dev(work, "work"), work.numel(), _stream())
    _check(st, "hydro_advance_level_adjoint")
    return out


def autotune_adjoint(level: torch.Tensor, g_out: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dx: float,
                     gamma: float, reps: int = 3, work: Optional[torch.Tensor] = None,
                     out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> Tuple[int, list]:
    """Time both adjoint forms on this level and record the faster in the
    context for its dtype and lattice (hydro_autotune_adjoint); returns
    (form, [ms fused, ms two kernels])."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    if tuple(level.shape) != (G, 5, 16, 16, 16) or g_out.shape != level.shape or g_out.dtype != level.dtype:
        raise ValueError("level and g_out must be [G,5,16,16,16] of one dtype")
    if out is not None and (out.dtype != level.dtype or out.shape != level.shape):
        raise ValueError("out must be [G,5,16,16,16] of the level dtype")
    _check_work(work)
    if out is None:
        out = torch.empty_like(level)
    if work is None:
        work = adjoint_workspace(G, level.dtype, True, level.device)
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    times = (ctypes.c_float * 2)()
    st = load().hydro_autotune_adjoint(_ctx(ctx), _dev(level, "level"), _dev(g_out, "g_out"), _dev(out, "out"), ngx, ngy, ngz, b,
                                       _dtype_code(level), float(dx), float(gamma), _dev(work, "work"), work.numel(),
                                       int(reps), times, _stream())
    if st < 0:
        raise HydroError("hydro_autotune_adjoint", st)
    return int(st), list(times)


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


def gather_ghost_adjoint(g_pad: torch.Tensor, ng: Sequence[int], ghost: int, bc: Sequence[int],
                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Padded cotangents [G,5,P,P,P] -> level cotangents [G,5,16,16,16], the
    transpose of fill_ghosts (hydro_gather_ghost_adjoint)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    P = 16 + 2 * int(ghost)
    if tuple(g_pad.shape) != (G, 5, P, P, P):
        raise ValueError("g_pad must be [G,5,P,P,P] with G = ngx*ngy*ngz, P = 16 + 2 ghost")
    if out is None:
        out = torch.empty((G, 5, 16, 16, 16), dtype=g_pad.dtype, device=g_pad.device)
    if out.dtype != g_pad.dtype or tuple(out.shape) != (G, 5, 16, 16, 16):
        raise ValueError("out must be [G,5,16,16,16] of the g_pad dtype")
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_gather_ghost_adjoint(_dev(g_pad, "g_pad"), _dev(out, "out"), ngx, ngy, ngz, int(ghost),
                                           _dtype_code(g_pad), b, _stream())
    _check(st, "hydro_gather_ghost_adjoint")
    return out


def _levels_array(levels):
    arr = (HydroLevel * len(levels))()
    dtype = None
    for i, L in enumerate(levels):
        lin, lout, ng, bc, dt, dx = L[:6]
        dt_dev = L[6] if len(L) > 6 else None
        cfl = L[7] if len(L) > 7 and L[7] is not None else {}
        dtype = lin.dtype if dtype is None else dtype
        if lin.dtype != dtype or lout.dtype != dtype or lin.shape != lout.shape:
            raise ValueError("batched levels must share one dtype and match in/out shapes")
        G = int(ng[0]) * int(ng[1]) * int(ng[2])
        if tuple(lin.shape) != (G, 5, 16, 16, 16):
            raise ValueError("level %d must be [G,5,16,16,16] with G = ngx*ngy*ngz" % i)
        arr[i].level_dev = _dev(lin, "level")
        arr[i].level_out_dev = _dev(lout, "level_out")
        arr[i].ngx, arr[i].ngy, arr[i].ngz = (int(v) for v in ng)
        for k in range(6):
            arr[i].bc[k] = int(bc[k])
        arr[i].dt = float(dt)
        arr[i].dx = float(dx)
        arr[i].dt_dev = _opt(dt_dev, "dt_dev", torch.float64)
        arr[i].dt_dev_scale = float(cfl.get("dt_dev_scale", 1.0))
        arr[i].c_cfl = float(cfl.get("c_cfl", 0.0))
        arr[i].dt_next_scale = float(cfl.get("dt_next_scale", 1.0))
        arr[i].dt_next_dev = _opt(cfl.get("dt_next"), "dt_next", torch.float64)
        dtp = cfl.get("dt_patch")
        if dtp is not None and dtp.numel() < 8 * G:
            raise ValueError("dt_patch must hold 8 doubles per group")
        arr[i].dt_patch_next_dev = _opt(dtp, "dt_patch", torch.float64)
        arr[i].dt_reset_dev = _opt(cfl.get("dt_reset"), "dt_reset", torch.float64)
    return arr, dtype


def advance_batched(levels, gamma: float, work: torch.Tensor, theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC,
                    n_bad: Optional[torch.Tensor] = None, grid: int = 0, ctx: Optional[Context] = None) -> None:
    """One step of several levels in one persistent launch (hydro_advance_batched).

    levels: sequence of (level_in, level_out, ng, bc, dt, dx[, dt_dev[, cfl]]),
    cfl an optional dict of the level's CFL outputs and dt scale (keys
    dt_dev_scale, c_cfl, dt_next_scale, and device float64 tensors dt_next,
    dt_patch [G*8], dt_reset: the fields of hydro_level_t);
    work: int32 device tensor of BATCH_WORK_WORDS zeros (re-armed by every launch)."""
    if work.dtype != torch.int32 or work.numel() < BATCH_WORK_WORDS:
        raise ValueError("work must hold %d int32" % BATCH_WORK_WORDS)
    arr, dtype = _levels_array(levels)
    st = load().hydro_advance_batched(_ctx(ctx), ctypes.cast(arr, ctypes.c_void_p), len(levels), _dtype_code(levels[0][0]),
                                      float(gamma), int(scheme), float(theta), _opt(n_bad, "n_bad", torch.int32),
                                      _dev(work, "work"), int(grid), _stream())
    _check(st, "hydro_advance_batched")


def advance_batched_noalloc(levels, gamma: float, theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC,
                            n_bad: Optional[torch.Tensor] = None, grid: int = 0, ctx: Optional[Context] = None) -> None:
    """advance_batched without a work buffer (hydro_advance_batched_noalloc):
    the library keeps the work counters in its own per-device array, so the
    call allocates nothing; calls overlapping on one device race."""
    arr, _ = _levels_array(levels)
    st = load().hydro_advance_batched_noalloc(_ctx(ctx), ctypes.cast(arr, ctypes.c_void_p), len(levels),
                                              _dtype_code(levels[0][0]), float(gamma), int(scheme), float(theta),
                                              _opt(n_bad, "n_bad", torch.int32), int(grid), _stream())
    _check(st, "hydro_advance_batched_noalloc")


def autotune_batched(levels, gamma: float, work: torch.Tensor, reps: int = 5,
                     ctx: Optional[Context] = None) -> Tuple[int, list]:
    if work.dtype != torch.int32 or work.numel() < BATCH_WORK_WORDS:
        raise ValueError("work must hold %d int32" % BATCH_WORK_WORDS)
    arr, dtype = _levels_array(levels)
    times = (ctypes.c_float * BATCHED_VARIANTS)()
    st = load().hydro_autotune_batched(_ctx(ctx), ctypes.cast(arr, ctypes.c_void_p), len(levels), _dtype_code(levels[0][0]),
                                       float(gamma), _dev(work, "work"), int(reps), times, _stream())
    if st < 0:
        raise HydroError("hydro_autotune_batched", st)
    return int(st), list(times)


def set_batched_variant(dtype, v: int, ctx: Optional[Context] = None) -> None:
    _check(load().hydro_set_batched_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32, int(v)),
           "hydro_set_batched_variant")


def get_batched_variant(dtype, ctx: Optional[Context] = None) -> int:
    return int(load().hydro_get_batched_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32))


class Graph:
    """A captured sequence of library calls (hydro_graph_*), replayed on the
    current stream.  Capture happens on a private non-default stream."""

    def __init__(self, ctx: Optional[Context] = None):
        self.handle = None
        self.ctx = ctx if ctx is not None else default_context()
        self.stream = torch.cuda.Stream()

    def capture(self, fn) -> "Graph":
        lib = load()
        torch.cuda.synchronize()
        with torch.cuda.stream(self.stream):
            _check(lib.hydro_graph_begin(self.stream.cuda_stream), "hydro_graph_begin")
            err = None
            try:
                fn()
            except BaseException as e:  # always end the capture
                err = e
            h = ctypes.c_void_p()
            st = lib.hydro_graph_end(self.ctx.handle, self.stream.cuda_stream, ctypes.byref(h))
            if err is not None:
                if st == HYDRO_OK:
                    lib.hydro_graph_destroy(self.ctx.handle, h)
                raise err
            _check(st, "hydro_graph_end")
        self.handle = h
        torch.cuda.synchronize()
        return self

    def replay(self) -> None:
        _check(load().hydro_graph_launch(self.handle, _stream()), "hydro_graph_launch")

    def close(self) -> None:
        if self.handle is not None and self.ctx.handle is not None:
            load().hydro_graph_destroy(self.ctx.handle, self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiLevel:
    """Levels of an AMR-shaped workload advanced in the W-cycle order of
    Sec. 2.1 with dt_l = dt_0 / 2^l: per coarse step, level l takes 2^l
    substeps; stage s of the 2^(L-1) stages advances every level l with
    s % 2^(L-1-l) == 0.  batched=True runs each stage as one persistent launch
    over the union of the stage's groups; batched=False launches
    hydro_advance_level once per level per stage.  Levels are independent
    periodic bricks (no coarse-fine coupling).

    adaptive=True (batched only): the coarse time-step is chosen on the
    device (Sec. 2.6 Eq. 2 with C = c_cfl): the launch of each level's last
    substep of a coarse step reduces the Eq. 2 time-step of the state it
    writes, scaled by 2^l, into one device word, so that the next coarse step
    takes dt_0 = min_l 2^l dt_l and level l reads dt_0 / 2^l from it; three
    words rotate over coarse steps (read, reduce, reset), so nothing is
    synchronized with the host.  dt0 is the first coarse step's time-step."""

    def __init__(self, levels, gamma: float, dt0: float, dtype=torch.float64, batched: bool = True,
                 theta: float = 1.5, scheme: int = SCHEME_MHM_PLM_HLLC, device=None, ctx: Optional[Context] = None,
                 adaptive: bool = False, c_cfl: float = 0.5):
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.ctx = ctx
        self.geo = [(tuple(int(v) for v in lv[0]), float(lv[1]), tuple(int(v) for v in lv[2])) for lv in levels]
        self.L = len(self.geo)
        self.gamma, self.dt0, self.batched = float(gamma), float(dt0), bool(batched)
        self.theta, self.scheme = float(theta), int(scheme)
        self.bufs = [[torch.empty((ng[0] * ng[1] * ng[2], 5, 16, 16, 16), dtype=dtype, device=dev) for _ in range(2)]
                     for ng, _, _ in self.geo]
        self.cur = [0] * self.L
        self.dtype = dtype
        self.work = torch.zeros(BATCH_WORK_WORDS, dtype=torch.int32, device=dev)
        self.n_bad = torch.zeros(1, dtype=torch.int32, device=dev)
        self.adaptive, self.c_cfl = bool(adaptive), float(c_cfl)
        if self.adaptive:
            if not self.batched:
                raise ValueError("the adaptive coarse step runs in the batched form")
            self.dtw = torch.full((3,), float("inf"), dtype=torch.float64, device=dev)
            self.dtw[0] = self.dt0
            self.rot = 0

    def dt_coarse(self) -> torch.Tensor:
        """Device word holding the time-step of the next coarse step (adaptive)."""
        return self.dtw[self.rot:self.rot + 1]

    def load_state(self, l: int, U: torch.Tensor):
        self.bufs[l][self.cur[l]].copy_(U)

    def state(self, l: int) -> torch.Tensor:
        return self.bufs[l][self.cur[l]]

    def cells_per_coarse_step(self) -> int:
        return sum(ng[0] * ng[1] * ng[2] * 4096 * 2 ** l for l, (ng, _, _) in enumerate(self.geo))

    def stage_levels(self, s: int):
        return [l for l in range(self.L) if s % 2 ** (self.L - 1 - l) == 0]

    def _entries(self, lvls, s: int = 0):
        out = []
        n_stages = 2 ** (self.L - 1)
        for l in lvls:
            ng, dx, bc = self.geo[l]
            e = (self.bufs[l][self.cur[l]], self.bufs[l][1 - self.cur[l]], ng, bc, self.dt0 / 2 ** l, dx)
            if self.adaptive:
                a, b, c = self.rot, (self.rot + 1) % 3, (self.rot + 2) % 3
                cfl = {"dt_dev_scale": 2.0 ** -l}
                if s == n_stages - 2 ** (self.L - 1 - l):   # the level's last substep of the coarse step
                    cfl.update(c_cfl=self.c_cfl, dt_next_scale=2.0 ** l, dt_next=self.dtw[b:b + 1])
                if s == 0 and l == lvls[0]:
                    cfl.update(c_cfl=self.c_cfl, dt_reset=self.dtw[c:c + 1])
                e = e + (self.dtw[a:a + 1], cfl)
            out.append(e)
        return out

    def stage(self, s: int) -> None:
        lvls = self.stage_levels(s)
        ent = self._entries(lvls, s)
        if self.batched:
            advance_batched(ent, self.gamma, self.work, self.theta, self.scheme, n_bad=self.n_bad, ctx=self.ctx)
        else:
            for lin, lout, ng, bc, dt, dx in ent:
                advance_level(lin, ng, bc, dt, dx, self.gamma, self.theta, self.scheme, out=lout, n_bad=self.n_bad,
                              ctx=self.ctx)
        for l in lvls:
            self.cur[l] = 1 - self.cur[l]

    def coarse_step(self) -> None:
        for s in range(2 ** (self.L - 1)):
            self.stage(s)
        if self.adaptive:
            self.rot = (self.rot + 1) % 3

    def autotune(self, reps: int = 3) -> Tuple[int, list]:
        """Choose the batched launch shape by the time of a whole coarse step:
        hydro_autotune_batched times every shape on each distinct stage (its
        outputs go to the scratch halves, the state is kept) and the stage
        times are summed with the number of times the stage occurs."""
        n_stages = 2 ** (self.L - 1)
        counts, first = {}, {}
        for s in range(n_stages):
            lvls = tuple(self.stage_levels(s))
            # stages differ also in which levels reduce their CFL time-step
            key = (lvls, tuple(e[7].get("dt_next") is not None for e in self._entries(lvls, s))
                   if self.adaptive else ())
            counts[key] = counts.get(key, 0) + 1
            first.setdefault(key, s)
        total = [0.0] * BATCHED_VARIANTS
        # the tuner's launches write the CFL outputs too: give them scratch words
        scratch = torch.full((2,), float("inf"), dtype=torch.float64, device=self.work.device)
        for key, c in counts.items():
            ent = self._entries(list(key[0]), first[key])
            if self.adaptive:
                ent = [e[:7] + ({**e[7], **({"dt_next": scratch[0:1]} if "dt_next" in e[7] else {}),
                                 **({"dt_reset": scratch[1:2]} if "dt_reset" in e[7] else {})},) for e in ent]
            _, times = autotune_batched(ent, self.gamma, self.work, reps, ctx=self.ctx)
            total = [a + c * t for a, t in zip(total, times)]
        best = min(range(len(total)), key=total.__getitem__)
        set_batched_variant(self.dtype, best, ctx=self.ctx)
        return best, total

    def capture(self, n_coarse: int = 2) -> Graph:
        """Graph of n_coarse coarse steps (an even count returns every level's
        state to the buffer it started in, and with adaptive=True a multiple
        of 6 also the time-step words to their roles, so the graph can be
        replayed)."""
        start = list(self.cur)
        rot = getattr(self, "rot", 0)
        g = Graph(self.ctx).capture(lambda: [self.coarse_step() for _ in range(n_coarse)])
        if self.cur != start or getattr(self, "rot", 0) != rot:
            raise ValueError("captured steps must return every level to its starting buffer")
        return g


# ------------------------------------------------------------- launch shapes --

def num_variants() -> int:
    return int(load().hydro_num_variants())


def variant_name(v: int) -> str:
    buf = ctypes.create_string_buffer(128)
    _check(load().hydro_variant_name(int(v), buf, 128), "hydro_variant_name")
    return buf.value.decode()


def set_adjoint_variant(dtype, v: int, ctx: Optional[Context] = None) -> None:
    """Form of the step adjoint for a dtype: 0 fused sweep, 1 two kernels with a face workspace."""
    _check(load().hydro_set_adjoint_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32, int(v)),
           "hydro_set_adjoint_variant")


def get_adjoint_variant(dtype, ctx: Optional[Context] = None) -> int:
    v = load().hydro_get_adjoint_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32)
    if v < 0:
        raise HydroError("hydro_get_adjoint_variant", v)
    return int(v)


def set_variant(dtype, v: int, ctx: Optional[Context] = None) -> None:
    _check(load().hydro_set_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32, int(v)), "hydro_set_variant")


def get_variant(dtype, ctx: Optional[Context] = None) -> int:
    return int(load().hydro_get_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32))


def set_level_variant(dtype, with_cfl: bool, v: int, ctx: Optional[Context] = None) -> None:
    _check(load().hydro_set_level_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32, int(bool(with_cfl)),
                                          int(v)), "hydro_set_level_variant")


def get_level_variant(dtype, with_cfl: bool, ctx: Optional[Context] = None) -> int:
    return int(load().hydro_get_level_variant(_ctx(ctx), F64 if dtype == torch.float64 else F32,
                                              int(bool(with_cfl))))


def autotune(level: torch.Tensor, ng: Sequence[int], bc: Sequence[int], dx: float, gamma: float,
             reps: int = 5, ctx: Optional[Context] = None) -> Tuple[int, list]:
    """Time every launch shape on this level in both kernel forms (without and
    with the CFL epilogue), record the fastest of each in the context for this
    dtype and lattice (hydro_autotune).

    Returns (chosen variant of the CFL form, mean ms per variant: the form
    without CFL first, then the CFL form)."""
    ngx, ngy, ngz = (int(v) for v in ng)
    G = ngx * ngy * ngz
    scratch = torch.empty_like(level)
    cfl = torch.empty(3 + 8 * G, dtype=torch.float64, device=level.device)
    n = num_variants()
    times = (ctypes.c_float * (2 * n))()
    b = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    st = load().hydro_autotune(_ctx(ctx), _dev(level, "level"), _dev(scratch, "scratch"), ngx, ngy, ngz, b,
                               _dtype_code(level), float(dx), float(gamma), _dev(cfl, "cfl"), cfl.numel() * 8,
                               int(reps), times, _stream())
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
                 c_cfl: float = 0.5, device=None, fused: bool = True, ctx: Optional[Context] = None):
        self.ctx = ctx
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
                              dt_reset=c, ctx=self.ctx)
                self.dt_min = a
                self.turn = (self.turn + 1) % 3
            else:
                advance_level(self.bufs[self.cur], self.ng, self.bc, dt, self.dx, self.gamma, self.theta,
                              self.scheme, out=nxt, n_bad=self.n_bad, ctx=self.ctx)
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


# ------------------------------------------------------ differentiable rollout --

class Rollout(torch.autograd.Function):
    """n_steps fixed-dt MHM steps of a level as a differentiable function of
    the initial state.  Forward keeps a checkpoint every k_ckpt steps; backward
    replays each segment from its checkpoint and applies the hand-written
    step adjoint (hydro_advance_level_adjoint) from the last step back.

    Rollout.apply(U0, ng, bc, n_steps, dt, dx, gamma, k_ckpt, theta, scheme) -> U_N"""

    @staticmethod
    def forward(ctx, U0, ng, bc, n_steps, dt, dx, gamma, k_ckpt=4, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
        ng, bc = tuple(int(v) for v in ng), tuple(int(v) for v in bc)
        k = max(1, int(k_ckpt))
        ckpts = []
        # private ping-pong buffers: the caller's U0 is never written
        cur = U0.detach().contiguous().clone()
        nxt = torch.empty_like(cur)
        for n in range(int(n_steps)):
            if n % k == 0:
                ckpts.append(cur.clone())
            advance_level(cur, ng, bc, dt, dx, gamma, theta, scheme, out=nxt)
            cur, nxt = nxt, cur
        ctx.save_for_backward(*ckpts)
        ctx.args = (ng, bc, int(n_steps), float(dt), float(dx), float(gamma), k, float(theta), int(scheme))
        return cur.clone()

    @staticmethod
    def backward(ctx, g):
        ng, bc, n_steps, dt, dx, gamma, k, theta, scheme = ctx.args
        ckpts = ctx.saved_tensors
        g = g.contiguous().clone()
        gin = torch.empty_like(g)
        work = adjoint_workspace(g.shape[0], g.dtype, True, g.device)
        for s in range((n_steps + k - 1) // k - 1, -1, -1):
            n0, n1 = s * k, min((s + 1) * k, n_steps)
            states = [ckpts[s]]
            for n in range(n0, n1 - 1):          # replay the segment
                states.append(advance_level(states[-1], ng, bc, dt, dx, gamma, theta, scheme))
            for n in range(n1 - 1, n0 - 1, -1):
                advance_level_adjoint(states[n - n0], g, ng, bc, dt, dx, gamma, theta, scheme, out=gin, work=work)
                g, gin = gin, g
        return (g,) + (None,) * 9



# ------------------------------------------------------ coarse-fine coupling --

class AmrSolver:
    """Coarse steps of a nested AMR hierarchy on the device (Sec. 2.1 W-cycle:
    level l takes two steps of dt_l / 2 ... down the hierarchy, 2^l steps per
    coarse step; Sec. 2.2 restriction and flux fix-up; Sec. 3.2 ghost zones
    from siblings or interpolated from the coarse level).  Every operation is
    one of the library's kernels: hydro_amr_fill_ghosts, hydro_advance_ext
    (with its patch-boundary face fluxes), hydro_amr_flux_accumulate,
    hydro_amr_restrict and hydro_amr_fixup.

    positions[l]: int [G_l, 3] group positions on level l's lattice (n0 * 2^l
    per axis); states[l]: [G_l, 5, 16, 16, 16] device tensors (advanced in
    place).  Level 0 must cover the domain; each finer level must be properly
    nested (the 27 coarse patches around each fine group's parent exist)."""

    def __init__(self, n0, positions, states, dx0: float, gamma: float, bc=(0,) * 6,
                 scheme: int = SCHEME_MHM_PLM_HLLC, theta: float = 1.5, ghost: int = 3):
        import numpy as np
        self.n0 = tuple(int(v) for v in n0)
        self.nl = len(positions)
        self.dx0, self.gamma, self.bc = float(dx0), float(gamma), tuple(int(v) for v in bc)
        self.scheme, self.theta, self.ghost = int(scheme), float(theta), int(ghost)
        self.U = list(states)
        dtype, device = self.U[0].dtype, self.U[0].device
        self.maps, self.pos, self.pad, self.work, self.flux, self.old, self.reg = [], [], [], [], [], [], []
        maps_np = []
        for l, p in enumerate(positions):
            p = np.ascontiguousarray(p, np.int32).reshape(-1, 3)
            n = [v << l for v in self.n0]
            m = np.full((n[2], n[1], n[0]), -1, np.int32)
            if np.any(p < 0) or np.any(p >= np.array(n)):
                raise ValueError("level %d: a position is off the lattice" % l)
            m[p[:, 2], p[:, 1], p[:, 0]] = np.arange(len(p), dtype=np.int32)
            if int((m >= 0).sum()) != len(p):
                raise ValueError("level %d: repeated positions" % l)
            if l == 0 and len(p) != n[0] * n[1] * n[2]:
                raise ValueError("level 0 must cover the domain")
            if l > 0:
                self._check_nested(p, maps_np[l - 1], [v << (l - 1) for v in self.n0])
            maps_np.append(m)
            G = len(p)
            if tuple(self.U[l].shape) != (G, 5, 16, 16, 16) or self.U[l].dtype != dtype:
                raise ValueError("level %d: states must be [G,5,16,16,16] of one dtype" % l)
            self.pos.append(torch.from_numpy(p).to(device))
            self.maps.append(torch.from_numpy(m).to(device))
            P = 16 + 2 * self.ghost
            self.pad.append(torch.empty((G, 5, P, P, P), dtype=dtype, device=device))
            self.work.append(ext_workspace(G, self.ghost, dtype, self.scheme, device))
            self.flux.append(torch.empty((G, 9, 5, 16, 16), dtype=dtype, device=device))
            self.old.append(torch.empty_like(self.U[l]) if l + 1 < self.nl else None)
            self.reg.append(torch.zeros((G, 6, 5, 8, 8), dtype=dtype, device=device) if l > 0 else None)
        self.n_bad = torch.zeros(1, dtype=torch.int32, device=device)
        self._bcarr = (ctypes.c_int32 * 6)(*self.bc)

    @staticmethod
    def _check_nested(p, cmap, nc):
        np_ = [2 * v for v in nc]
        for gx, gy, gz in p:
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        q = [(gx + dx) % np_[0], (gy + dy) % np_[1], (gz + dz) % np_[2]]
                        if cmap[q[2] >> 1, q[1] >> 1, q[0] >> 1] < 0:
                            raise ValueError("a fine group at %s is not properly nested" % ((gx, gy, gz),))

    def _lvl(self, l: int, U=None) -> HydroAmrLevel:
        L = HydroAmrLevel()
        L.U_dev = _dev(self.U[l] if U is None else U, "states")
        L.pos_dev = self.pos[l].data_ptr()
        L.map_dev = self.maps[l].data_ptr()
        L.n_groups = self.pos[l].shape[0]
        for d in range(3):
            L.n[d] = self.n0[d] << l
        return L

    def cells_per_coarse_step(self) -> int:
        return sum(int(self.pos[l].shape[0]) * 4096 * 2 ** l for l in range(self.nl))

    def step(self, dt0: float) -> None:
        """One coarse step of dt0 (asynchronous on the current stream)."""
        self._advance(0, float(dt0), None, None, 0.0, None)

    def capture(self, dt0: float, n_coarse: int = 1, ctx: Optional[Context] = None) -> Graph:
        """Graph of n_coarse coarse steps of dt0 (every launch of the W-cycle,
        the level copies and register clears included); each replay advances
        the hierarchy by n_coarse steps in place.  Nothing runs at capture."""
        return Graph(ctx).capture(lambda: [self.step(dt0) for _ in range(n_coarse)])

    def _advance(self, l, dt, cold, cnew, a, R_parent):
        lib, s = load(), _stream()
        code = _dtype_code(self.U[l])
        dx = self.dx0 / 2 ** l
        if l + 1 < self.nl:
            self.old[l].copy_(self.U[l])
        fine = self._lvl(l)
        coarse = self._lvl(l - 1) if l > 0 else None
        st = lib.hydro_amr_fill_ghosts(ctypes.byref(fine), None if coarse is None else ctypes.byref(coarse),
                                       None if cold is None else _dev(cold, "cold"),
                                       None if cnew is None else _dev(cnew, "cnew"), float(a), self._bcarr,
                                       self.ghost, code, _dev(self.pad[l], "pad"), s)
        _check(st, "hydro_amr_fill_ghosts")
        advance_ext(self.pad[l], dt, dx, self.gamma, self.scheme, self.theta, out=self.U[l], n_bad=self.n_bad,
                    work=self.work[l], face_flux=self.flux[l])
        if R_parent is not None:
            st = lib.hydro_amr_flux_accumulate(ctypes.byref(fine), _dev(self.flux[l], "flux"), 0.5, self._bcarr, code,
                                               _dev(R_parent, "reg"), s)
            _check(st, "hydro_amr_flux_accumulate")
        if l + 1 < self.nl:
            R = self.reg[l + 1]
            R.zero_()
            self._advance(l + 1, 0.5 * dt, self.old[l], self.U[l], 0.0, R)
            self._advance(l + 1, 0.5 * dt, self.old[l], self.U[l], 0.5, R)
            child = self._lvl(l + 1)
            _check(lib.hydro_amr_restrict(ctypes.byref(child), ctypes.byref(fine), code, s), "hydro_amr_restrict")
            st = lib.hydro_amr_fixup(ctypes.byref(fine), ctypes.byref(child), _dev(self.flux[l], "flux"),
                                     _dev(R, "reg"), dt / dx, self._bcarr, code, s)
            _check(st, "hydro_amr_fixup")
