"""Plain FP64 CPU oracle for the MHM + PLM + HLLC patch-group step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  The arithmetic lives
in ``mhm_oracle.cpp`` (C++17, templated over the scalar so that the same code
also runs in dual numbers and in an operation-counting type); this module only
marshals numpy arrays through ctypes.  It shares no code with the HIP library.

Parity pins (what checks the oracle against something other than itself) are
in ``tests/test_oracle_*.py``: the exact Riemann solution of a Sod tube
(including Rankine-Hugoniot and isentrope checks of the exact solver), second
order convergence on a smooth translating wave, conservation to round-off in a
periodic box, uniform-flow and stationary-contact invariance, x/y/z cyclic and
mirror symmetry, block-decomposition invariance, limiter special cases
(theta = 1 minmod, theta = 2 MC), HLLC limiting cases, brute-force CFL, and
dual-number JVPs against central finite differences.

The other options of Sec. 2.2 (limiters, characteristic PLM, PPM, Roe, HLLE,
CTU, and the procedure for unphysical results) are reached through
``step_any`` / ``level_step_any`` / ``level_step_fallback`` and pinned in
``tests/test_oracle_ext_schemes.py`` and ``tests/test_oracle_fallback.py``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhm_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SCHEME_MHM_PLM_HLLC = 1
WAVESPEED_ROE = 0 << 8
WAVESPEED_DAVIS = 1 << 8
FIRST_ORDER = 1 << 10
# other schemes of Sec. 2.2 (scheme word bits beyond the default)
SCHEME_MHM = 1
SCHEME_CTU = 2
LIMITER_GMINMOD = 0 << 11
LIMITER_VANLEER = 1 << 11
LIMITER_VANALBADA = 2 << 11
LIMITER_HYBRID = 3 << 11
CHARACTERISTIC = 1 << 13
PPM = 1 << 14
RIEMANN_HLLC = 0 << 16
RIEMANN_ROE = 1 << 16
RIEMANN_HLLE = 2 << 16
DUAL_ENERGY = 1 << 18


def build_library(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP over groups, no FMA contraction)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build_library()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "oracle_mhm_step": (i64, [P, P, i64, i32, f64, f64, f64, f64, i32]),
        "oracle_mhm_step_block": (i64, [P, P, i32, i32, i32, i32, f64, f64, f64, f64, i32]),
        "oracle_dt": (i32, [P, i64, i32, f64, f64, f64, P]),
        "oracle_fill_ghosts": (i32, [P, P, i32, i32, i32, i32, P]),
        "oracle_rollout": (i64, [P, P, i32, i32, i32, i32, P, i32, f64, f64, f64, f64, f64, i32, P]),
        "oracle_rollout_jvp": (i64, [P, P, P, P, i32, i32, i32, i32, P, i32, f64, f64, f64, f64, i32]),
        "oracle_mhm_step_jvp": (i64, [P, P, P, P, i64, i32, f64, f64, f64, f64, i32]),
        "oracle_hllc": (i32, [P, P, i32, f64, i32, P]),
        "oracle_limited_slope": (f64, [f64, f64, f64, f64]),
        "oracle_hancock_cell": (None, [P, P, P, f64, f64, f64, i32, P]),
        "oracle_cons_to_prim": (None, [P, f64, P]),
        "oracle_prim_to_cons": (None, [P, f64, P]),
        "oracle_exact_star": (i32, [f64] * 7 + [P]),
        "oracle_exact_sample": (i32, [f64] * 7 + [P, i64, P, P, P]),
        "oracle_exact_residual": (f64, [f64] * 8),
        "oracle_count_ops": (None, [P, P, P, P, P, P, f64, f64, f64, P]),
        "oracle_rollout_box": (i64, [P, P, P, P, i32, i32, i32, i32, f64, f64, f64, f64, i32, P]),
        "oracle_step_any": (i64, [P, P, i64, i32, f64, f64, f64, f64, i32]),
        "oracle_step_block_any": (i64, [P, P, i32, i32, i32, i32, f64, f64, f64, f64, i32]),
        "oracle_step_any_flux": (i64, [P, P, P, i64, i32, f64, f64, f64, f64, i32]),
        "oracle_step_any_jvp": (i64, [P, P, P, P, i64, i32, f64, f64, f64, f64, i32]),
        "oracle_riemann": (i32, [P, P, i32, f64, i32, P]),
        "oracle_step_any_de": (i64, [P, P, i64, i32, f64, f64, f64, f64, i32, f64]),
        "oracle_step_block_any_de": (i64, [P, P, i32, i32, i32, i32, f64, f64, f64, f64, i32, f64]),
        "oracle_limit_diffs": (f64, [f64, f64, f64, f64, i32]),
        "oracle_limited_slopes": (None, [P, P, P, i32, f64, f64, i32, P]),
        "oracle_face_values": (None, [P, i32, f64, f64, i32, P]),
        "oracle_to_characteristic": (None, [P, i32, f64, f64, P]),
        "oracle_from_characteristic": (None, [P, i32, f64, f64, P]),
        "oracle_level_step_any": (i64, [P, P, i32, i32, i32, i32, P, f64, f64, f64, f64, i32]),
        "oracle_level_step_fallback": (i64, [P, P, i32, i32, i32, i32, P, f64, f64, f64, f64, f64, f64, i32, P]),
        "oracle_first_order_cell": (None, [P, i32, i32, i32, P, i32, i32, i32, f64, f64, i32, i32, P]),
        "oracle_amr_step": (i64, [i32, P, P, P, P, P, i32, f64, f64, f64, f64, i32]),
        "oracle_amr_fill": (i32, [i32, P, P, P, P, P, i32, P, P, f64, i32, P]),
        "oracle_num_threads": (i32, []),
        "oracle_set_num_threads": (None, [i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bc(bc: Sequence[int]) -> np.ndarray:
    b = np.ascontiguousarray(bc, dtype=np.int32)
    assert b.shape == (6,)
    return b


# ----------------------------------------------------------------- step API --

def mhm_step(U_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """One MHM step of padded 16^3 groups U_pad[G,5,P,P,P] -> (U_out[G,5,16,16,16], n_bad)."""
    U = _f64(U_pad)
    G, nf, P = U.shape[0], U.shape[1], U.shape[2]
    assert nf == 5 and U.shape[2:] == (P, P, P) and (P - 16) % 2 == 0
    out = np.empty((G, 5, 16, 16, 16), np.float64)
    n_bad = _load().oracle_mhm_step(_p(U), _p(out), G, (P - 16) // 2, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_mhm_step: bad arguments")
    return out, int(n_bad)


def mhm_step_block(U_pad, ghost, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """One MHM step of one padded block U_pad[5,nz+2g,ny+2g,nx+2g] -> (U_out[5,nz,ny,nx], n_bad)."""
    U = _f64(U_pad)
    nz, ny, nx = (s - 2 * ghost for s in U.shape[1:])
    out = np.empty((5, nz, ny, nx), np.float64)
    n_bad = _load().oracle_mhm_step_block(_p(U), _p(out), nx, ny, nz, ghost, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_mhm_step_block: bad arguments")
    return out, int(n_bad)


def mhm_step_jvp(U_pad, T_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """Dual-number JVP of one padded-group step: returns (U_out, T_out, n_bad)."""
    U, T = _f64(U_pad), _f64(T_pad)
    assert U.shape == T.shape
    G, P = U.shape[0], U.shape[2]
    out = np.empty((G, 5, 16, 16, 16), np.float64)
    tout = np.empty_like(out)
    n_bad = _load().oracle_mhm_step_jvp(_p(U), _p(T), _p(out), _p(tout), G, (P - 16) // 2, dt, dx, gamma,
                                        theta, scheme)
    return out, tout, int(n_bad)


def dt_patch(U_pad, dx, gamma, c_cfl=0.5):
    """Per-patch CFL time-step (Eq. 2) of padded groups: returns dt[G, 8]."""
    U = _f64(U_pad)
    G, P = U.shape[0], U.shape[2]
    out = np.empty((G, 8), np.float64)
    if _load().oracle_dt(_p(U), G, (P - 16) // 2, dx, gamma, c_cfl, _p(out)) != 0:
        raise ValueError("oracle_dt: bad arguments")
    return out


def fill_ghosts(level, ng, ghost, bc):
    """Group-major interiors level[G,5,16,16,16] -> padded groups [G,5,P,P,P]."""
    L = _f64(level)
    ngx, ngy, ngz = ng
    G = ngx * ngy * ngz
    assert L.shape == (G, 5, 16, 16, 16)
    P = 16 + 2 * ghost
    out = np.empty((G, 5, P, P, P), np.float64)
    if _load().oracle_fill_ghosts(_p(L), _p(out), ngx, ngy, ngz, ghost, _p(_bc(bc))) != 0:
        raise ValueError("oracle_fill_ghosts: bad arguments")
    return out


def rollout(level, ng, ghost, bc, n_steps, dx, gamma, dt=None, c_cfl=0.5, theta=1.5,
            scheme=SCHEME_MHM_PLM_HLLC):
    """n_steps MHM steps with ghost fill every step.  dt=None: CFL time-step each step.

    Returns (level_out, dts[n_steps], n_bad)."""
    L = _f64(level)
    ngx, ngy, ngz = ng
    out = np.empty_like(L)
    dts = np.empty(n_steps, np.float64)
    n_bad = _load().oracle_rollout(_p(L), _p(out), ngx, ngy, ngz, ghost, _p(_bc(bc)), n_steps,
                                   -1.0 if dt is None else float(dt), c_cfl, dx, gamma, theta, scheme, _p(dts))
    if n_bad < 0:
        raise ValueError("oracle_rollout: bad arguments")
    return out, dts, int(n_bad)


def rollout_jvp(level, tangent, ng, ghost, bc, n_steps, dt, dx, gamma, theta=1.5,
                scheme=SCHEME_MHM_PLM_HLLC):
    """Exact JVP of a fixed-dt rollout (dual numbers): returns (level_out, tangent_out, n_bad)."""
    L, T = _f64(level), _f64(tangent)
    assert L.shape == T.shape
    ngx, ngy, ngz = ng
    out, tout = np.empty_like(L), np.empty_like(L)
    n_bad = _load().oracle_rollout_jvp(_p(L), _p(T), _p(out), _p(tout), ngx, ngy, ngz, ghost, _p(_bc(bc)),
                                       n_steps, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_rollout_jvp: bad arguments")
    return out, tout, int(n_bad)


def rollout_box(box, n_steps, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC, tangent=None,
                signature=False):
    """n_steps MHM steps of one box [5, nz, ny, nx] without ghost refills: each
    step drops a 2-cell margin, so the result is [5, nz-4n, ny-4n, nx-4n], the
    cells the box alone determines.  tangent: optional dual-number tangent of
    the box.  Returns (out, tangent_out or None, n_bad, signature or None),
    signature being the hash of every branch decision taken (limiter one-sign
    tests, |.| signs, min/max arguments, HLLC branches) in evaluation order."""
    b = _f64(box)
    assert b.ndim == 4 and b.shape[0] == 5
    nz, ny, nx = b.shape[1:]
    m = [s - 4 * n_steps for s in (nz, ny, nx)]
    if min(m) < 1:
        raise ValueError("box too small for %d steps" % n_steps)
    out = np.empty([5] + m, np.float64)
    t = None if tangent is None else _f64(tangent)
    tout = None if t is None else np.empty_like(out)
    sig = np.zeros(1, np.uint64)
    nb = _load().oracle_rollout_box(_p(b), None if t is None else _p(t), _p(out), None if t is None else _p(tout),
                                    nx, ny, nz, n_steps, dt, dx, gamma, theta, scheme,
                                    _p(sig) if signature else None)
    if nb < 0:
        raise ValueError("oracle_rollout_box: bad arguments")
    return out, tout, int(nb), (int(sig[0]) if signature else None)


# ------------------------------------------------------------ component API --

def hllc(UL, UR, d, gamma, wavespeed=0):
    """HLLC flux across a face normal to axis d; returns (F[5], bad)."""
    l, r = _f64(UL), _f64(UR)
    F = np.empty(5, np.float64)
    bad = _load().oracle_hllc(_p(l), _p(r), d, gamma, wavespeed, _p(F))
    return F, bool(bad)


def limited_slope(qm, q0, qp, theta):
    return _load().oracle_limited_slope(float(qm), float(q0), float(qp), float(theta))


def hancock_cell(Wc, Wm, Wp, gamma, theta, half_dtdx, first_order=False):
    """Six half-step-evolved face states of one cell: returns Ut[3, 2, 5]."""
    c, m, p = _f64(Wc), _f64(Wm).reshape(3, 5), _f64(Wp).reshape(3, 5)
    out = np.empty((3, 2, 5), np.float64)
    _load().oracle_hancock_cell(_p(c), _p(m), _p(p), gamma, theta, half_dtdx, int(first_order), _p(out))
    return out


def cons_to_prim(U, gamma):
    u, W = _f64(U), np.empty(5, np.float64)
    _load().oracle_cons_to_prim(_p(u), gamma, _p(W))
    return W


def prim_to_cons(W, gamma):
    w, U = _f64(W), np.empty(5, np.float64)
    _load().oracle_prim_to_cons(_p(w), gamma, _p(U))
    return U


def exact_star(left, right, gamma):
    """Star state of the exact Riemann problem: (p*, u*, rho*_L, rho*_R, newton_iterations)."""
    out = np.empty(5, np.float64)
    if _load().oracle_exact_star(*left, *right, gamma, _p(out)) != 0:
        raise ValueError("vacuum-generating data")
    return tuple(out[:4]) + (int(out[4]),)


def exact_sample(left, right, gamma, xi):
    """Exact self-similar solution (rho, u, p) at xi = x/t."""
    x = _f64(xi).ravel()
    r, u, p = (np.empty_like(x) for _ in range(3))
    if _load().oracle_exact_sample(*left, *right, gamma, _p(x), x.size, _p(r), _p(u), _p(p)) != 0:
        raise ValueError("vacuum-generating data")
    return r, u, p


def exact_residual(left, right, gamma, p):
    return _load().oracle_exact_residual(*left, *right, gamma, float(p))


def num_threads() -> int:
    """OpenMP threads used by the oracle's loops over groups."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's loops over groups (n >= 1)."""
    _load().oracle_set_num_threads(int(n))


def count_ops(U, Wc, Wm, Wp, UL, UR, gamma, theta, half_dtdx):
    """Operation counts {add, mul, div, sqrt} of cons_to_prim, hancock_cell, hllc_flux, update."""
    args = [_f64(a) for a in (U, Wc, Wm, Wp, UL, UR)]
    ops = np.zeros(16, np.int64)
    _load().oracle_count_ops(*[_p(a) for a in args], gamma, theta, half_dtdx, _p(ops))
    names = ("cons_to_prim", "hancock_cell", "hllc_flux", "update")  # hllc_flux: the branch UL, UR select
    return {n: dict(zip(("add", "mul", "div", "sqrt"), ops[4 * i:4 * i + 4].tolist())) for i, n in enumerate(names)}


# ----------------------------------------------- other schemes of Sec. 2.2 --

def step_any(U_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """One step of padded 16^3 groups with any scheme word (MHM or CTU; PLM or
    PPM; primitive or characteristic; any limiter; HLLC, Roe or HLLE):
    returns (U_out[G,5,16,16,16], n_bad)."""
    U = _f64(U_pad)
    G, P = U.shape[0], U.shape[2]
    out = np.empty((G, 5, 16, 16, 16), np.float64)
    n_bad = _load().oracle_step_any(_p(U), _p(out), G, (P - 16) // 2, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_step_any: bad arguments")
    return out, int(n_bad)


def step_any_flux(U_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """step_any that also returns the fluxes the update used on the faces of
    the patch boundaries: (U_out[G,5,16,16,16], face_flux[G,9,5,16,16],
    n_bad); plane 3 axis + k holds the axis' faces at normal coordinate 8 k,
    entry [field][b][a] with (a, b) the transverse coordinates in cyclic
    order."""
    U = _f64(U_pad)
    G, P = U.shape[0], U.shape[2]
    out = np.empty((G, 5, 16, 16, 16), np.float64)
    ff = np.empty((G, 9, 5, 16, 16), np.float64)
    n_bad = _load().oracle_step_any_flux(_p(U), _p(out), _p(ff), G, (P - 16) // 2, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_step_any_flux: bad arguments")
    return out, ff, int(n_bad)


def step_block_any(U_pad, ghost, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """step_any for one padded block [5, nz+2g, ny+2g, nx+2g]: returns (U_out[5,nz,ny,nx], n_bad)."""
    U = _f64(U_pad)
    nz, ny, nx = (s - 2 * ghost for s in U.shape[1:])
    out = np.empty((5, nz, ny, nx), np.float64)
    n_bad = _load().oracle_step_block_any(_p(U), _p(out), nx, ny, nz, ghost, dt, dx, gamma, theta, scheme)
    if n_bad < 0:
        raise ValueError("oracle_step_block_any: bad arguments")
    return out, int(n_bad)


def step_any_jvp(U_pad, T_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """Dual-number JVP of step_any: returns (U_out, T_out, n_bad)."""
    U, T = _f64(U_pad), _f64(T_pad)
    G, P = U.shape[0], U.shape[2]
    out = np.empty((G, 5, 16, 16, 16), np.float64)
    tout = np.empty_like(out)
    n_bad = _load().oracle_step_any_jvp(_p(U), _p(T), _p(out), _p(tout), G, (P - 16) // 2, dt, dx, gamma, theta,
                                        scheme)
    if n_bad < 0:
        raise ValueError("oracle_step_any_jvp: bad arguments")
    return out, tout, int(n_bad)


def riemann(UL, UR, d, gamma, scheme=SCHEME_MHM_PLM_HLLC):
    """Flux of the scheme word's Riemann solver across a face normal to axis d: (F[5], bad)."""
    l, r = _f64(UL), _f64(UR)
    F = np.empty(5, np.float64)
    bad = _load().oracle_riemann(_p(l), _p(r), d, gamma, scheme, _p(F))
    if bad < 0:
        raise ValueError("bad Riemann solver id")
    return F, bool(bad)


def limit_diffs(dm, dp, dc, theta, limiter):
    """Limited slope from one-sided differences (limiter 0..3: generalized minmod, van Leer, van Albada, hybrid)."""
    return _load().oracle_limit_diffs(float(dm), float(dp), float(dc), float(theta), int(limiter))


def limited_slopes(Wm, Wc, Wp, d, gamma, theta, scheme):
    out = np.empty(5, np.float64)
    a, b, c = _f64(Wm), _f64(Wc), _f64(Wp)
    _load().oracle_limited_slopes(_p(a), _p(b), _p(c), d, gamma, theta, scheme, _p(out))
    return out


def face_values(Ws, d, gamma, theta, scheme):
    """Face values (low, high) of the centre cell of a 5-cell stencil Ws[5, 5] along axis d."""
    w = _f64(Ws).reshape(5, 5)
    out = np.empty((2, 5), np.float64)
    _load().oracle_face_values(_p(w), d, gamma, theta, scheme, _p(out))
    return out


def to_characteristic(dW, d, rho, c):
    a, out = _f64(dW), np.empty(5, np.float64)
    _load().oracle_to_characteristic(_p(a), d, float(rho), float(c), _p(out))
    return out


def from_characteristic(a, d, rho, c):
    x, out = _f64(a), np.empty(5, np.float64)
    _load().oracle_from_characteristic(_p(x), d, float(rho), float(c), _p(out))
    return out


def level_step_any(level, ng, ghost, bc, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC):
    """Ghost fill + one step of any scheme over a level: returns (level_out, n_bad)."""
    L = _f64(level)
    ngx, ngy, ngz = ng
    out = np.empty_like(L)
    n_bad = _load().oracle_level_step_any(_p(L), _p(out), ngx, ngy, ngz, ghost, _p(_bc(bc)), dt, dx, gamma, theta,
                                          scheme)
    if n_bad < 0:
        raise ValueError("oracle_level_step_any: bad arguments")
    return out, int(n_bad)


def level_step_fallback(level, ng, ghost, bc, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC,
                        dt_min=0.0, ratio=0.8):
    """One level step with the procedure for unphysical results (Sec. 2.2):
    returns (level_out, cells_still_unphysical, info) with info = dict(dt,
    retries, unsplit, split) of the accepted (or last) attempt."""
    L = _f64(level)
    ngx, ngy, ngz = ng
    out = np.empty_like(L)
    info = np.zeros(4, np.float64)
    left = _load().oracle_level_step_fallback(_p(L), _p(out), ngx, ngy, ngz, ghost, _p(_bc(bc)), dt, dt_min, ratio,
                                              dx, gamma, theta, scheme, _p(info))
    if left < 0:
        raise ValueError("oracle_level_step_fallback: bad arguments")
    return out, int(left), {"dt": float(info[0]), "retries": int(info[1]), "unsplit": int(info[2]),
                            "split": int(info[3])}


def first_order_cell(level, ng, bc, X, Y, Z, dtdx, gamma, scheme=SCHEME_MHM_PLM_HLLC, split=False):
    """First-order recomputation of one level cell (global indices): unsplit or x, y, z split."""
    L = _f64(level)
    out = np.empty(5, np.float64)
    _load().oracle_first_order_cell(_p(L), *ng, _p(_bc(bc)), X, Y, Z, dtdx, gamma, scheme, int(split), _p(out))
    return out


# --------------------------------------------------- coarse-fine coupling --

def _amr_pack(n0, positions, states):
    G = np.ascontiguousarray([len(p) for p in positions], np.int64)
    pos = np.ascontiguousarray(np.concatenate([np.asarray(p, np.int32).reshape(-1, 3) for p in positions]), np.int32)
    U = np.ascontiguousarray(np.concatenate([np.asarray(u, np.float64) for u in states]), np.float64)
    n = np.ascontiguousarray(n0, np.int32)
    return n, G, pos, U


def amr_step(n0, positions, states, bc, dt0, dx0, gamma, theta=1.5, scheme=SCHEME_MHM_PLM_HLLC, ghost=3):
    """One coarse step of a nested AMR hierarchy (W-cycle with ghost-zone
    interpolation, flux registers, restriction and flux fix-up): returns
    (new states per level, n_bad)."""
    n, G, pos, U = _amr_pack(n0, positions, states)
    nb = _load().oracle_amr_step(len(positions), _p(n), _p(G), _p(pos), _p(U), _p(_bc(bc)), ghost, dt0, dx0, gamma,
                                 theta, scheme)
    if nb < 0:
        raise ValueError("oracle_amr_step: bad arguments (positions, nesting or scheme)")
    out, o = [], 0
    for g in G:
        out.append(U[o:o + g].copy())
        o += g
    return out, int(nb)


def amr_fill(n0, positions, states, bc, level, coarse_old, coarse_new, a, ghost=3):
    """Padded groups of one level of a hierarchy: ghosts from sibling groups,
    else interpolated from the coarse level between coarse_old and coarse_new."""
    n, G, pos, U = _amr_pack(n0, positions, states)
    P = 16 + 2 * ghost
    pad = np.empty((G[level], 5, P, P, P), np.float64)
    co = _f64(coarse_old) if level > 0 else np.zeros(1)
    cn = _f64(coarse_new) if level > 0 else np.zeros(1)
    st = _load().oracle_amr_fill(len(positions), _p(n), _p(G), _p(pos), _p(U), _p(_bc(bc)), level, _p(co), _p(cn),
                                 float(a), ghost, _p(pad))
    if st != 0:
        raise ValueError("oracle_amr_fill: bad arguments")
    return pad


def step_any_de(U_pad, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM | DUAL_ENERGY, xi=0.01):
    """Dual-energy step of padded groups with 6 fields (field 5 the entropy
    s = p / rho^(gamma-1)): U_pad[G,6,P,P,P] -> (U_out[G,6,16,16,16], n_bad)."""
    U = _f64(U_pad)
    G, P = U.shape[0], U.shape[2]
    assert U.shape[1] == 6
    out = np.empty((G, 6, 16, 16, 16), np.float64)
    n_bad = _load().oracle_step_any_de(_p(U), _p(out), G, (P - 16) // 2, dt, dx, gamma, theta, scheme, xi)
    if n_bad < 0:
        raise ValueError("oracle_step_any_de: bad arguments")
    return out, int(n_bad)


def step_block_any_de(U_pad, ghost, dt, dx, gamma, theta=1.5, scheme=SCHEME_MHM | DUAL_ENERGY, xi=0.01):
    """Dual-energy step of one padded block [6, nz+2g, ny+2g, nx+2g]: (U_out[6,nz,ny,nx], n_bad)."""
    U = _f64(U_pad)
    nz, ny, nx = (s - 2 * ghost for s in U.shape[1:])
    out = np.empty((6, nz, ny, nx), np.float64)
    n_bad = _load().oracle_step_block_any_de(_p(U), _p(out), nx, ny, nz, ghost, dt, dx, gamma, theta, scheme, xi)
    if n_bad < 0:
        raise ValueError("oracle_step_block_any_de: bad arguments")
    return out, int(n_bad)
