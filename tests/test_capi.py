"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/hydro.h, and rejects bad arguments before any HIP call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hydro.h")


def declared_entry_points():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1712_07070_amd import hydro
    if not os.path.exists(hydro.LIB_PATH):
        pytest.fail("libhydro.so is not built")
    return hydro.load()


def test_header_declares_entry_points():
    names = declared_entry_points()
    for n in ("hydro_advance", "hydro_dt", "hydro_fill_ghosts", "hydro_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_entry_points():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.hydro_strerror(0) == b"ok"
    assert lib.hydro_strerror(-1) == b"invalid argument"
    assert lib.hydro_version() >= 1


def _adv(lib, **kw):
    a = dict(U=ctypes.c_void_p(4096), O=ctypes.c_void_p(1 << 40), G=1, gh=3, dtype=0, dt=1e-3, dx=1.0 / 64,
             gamma=5.0 / 3.0, scheme=1, theta=1.5, dt_dev=None, nbad=None, stream=None)
    a.update(kw)
    return lib.hydro_advance(a["U"], a["O"], a["G"], a["gh"], a["dtype"], a["dt"], a["dx"], a["gamma"], a["scheme"],
                             a["theta"], a["dt_dev"], a["nbad"], a["stream"])


@pytest.mark.parametrize("bad", [
    dict(G=-1), dict(gh=1), dict(gh=17), dict(dtype=2), dict(dt=0.0), dict(dt=float("nan")), dict(dx=-1.0),
    dict(gamma=1.0), dict(theta=0.9), dict(theta=2.5), dict(scheme=2), dict(scheme=1 | (2 << 8)),
    dict(scheme=1 | (1 << 12)), dict(U=None), dict(O=None),
    dict(O=ctypes.c_void_p(4096 + 8)),          # output overlaps the input
])
def test_advance_rejects_bad_arguments(lib, bad):
    assert _adv(lib, **bad) == -1


def test_advance_zero_groups_is_a_no_op(lib):
    assert _adv(lib, G=0, U=None, O=None) == 0


def test_dt_and_fill_reject_bad_arguments(lib):
    P = ctypes.c_void_p
    assert lib.hydro_dt(P(4096), 1, 3, 0, -1.0, 1.4, 0.5, P(1 << 40), None, None) == -1
    assert lib.hydro_dt(P(4096), 1, 3, 0, 0.1, 1.4, 0.0, P(1 << 40), None, None) == -1
    assert lib.hydro_dt(None, 1, 3, 0, 0.1, 1.4, 0.5, P(1 << 40), None, None) == -1
    assert lib.hydro_dt(None, 0, 3, 0, 0.1, 1.4, 0.5, None, None, None) == 0  # nothing to do, no launch
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    badbc = (ctypes.c_int32 * 6)(0, 0, 2, 0, 0, 0)
    assert lib.hydro_fill_ghosts(P(4096), P(1 << 40), 0, 1, 1, 3, 0, bc, None) == -1
    assert lib.hydro_fill_ghosts(P(4096), P(1 << 40), 1, 1, 1, 17, 0, bc, None) == -1
    assert lib.hydro_fill_ghosts(P(4096), P(1 << 40), 1, 1, 1, 3, 0, badbc, None) == -1
    assert lib.hydro_fill_ghosts(P(4096), P(4096 + 64), 1, 1, 1, 3, 0, bc, None) == -1


def test_gather_ghost_adjoint_rejects_bad_arguments(lib):
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    badbc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 5)
    f = lib.hydro_gather_ghost_adjoint
    assert f(P(4096), P(1 << 40), 1, 0, 1, 3, 0, bc, None) == -1
    assert f(P(4096), P(1 << 40), 1, 1, 1, -1, 0, bc, None) == -1
    assert f(P(4096), P(1 << 40), 1, 1, 1, 17, 0, bc, None) == -1
    assert f(P(4096), P(1 << 40), 1, 1, 1, 3, 2, bc, None) == -1
    assert f(P(4096), P(1 << 40), 1, 1, 1, 3, 0, badbc, None) == -1
    assert f(P(4096), P(1 << 40), 1, 1, 1, 3, 0, None, None) == -1
    assert f(None, P(1 << 40), 1, 1, 1, 3, 0, bc, None) == -1
    assert f(P(4096), P(4096 + 8), 1, 1, 1, 3, 0, bc, None) == -1   # output overlaps the input


@pytest.mark.parametrize("ng", [(0, 1, 1), (1, -3, 1), ((1 << 26) + 1, 1, 1), (1 << 11, 1 << 10, 1 << 10)])
def test_level_entry_points_reject_bad_geometry(lib, ng):
    """Every level entry point takes 1 <= ng <= 2^26 per axis and fewer than
    2^31 - 8 groups; larger lattices are refused before any HIP call."""
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    a, b = P(4096), P(1 << 46)
    assert lib.hydro_advance_level(a, b, *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None, None, 0.5, None, None, None,
                                   None) == -1
    assert lib.hydro_advance_level_adjoint(a, b, P(1 << 47), *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None, P(1 << 45),
                                           1 << 40, None) == -1
    assert lib.hydro_fill_ghosts(a, b, *ng, 3, 0, bc, None) == -1
    assert lib.hydro_gather_ghost_adjoint(a, b, *ng, 3, 0, bc, None) == -1
    assert lib.hydro_autotune_adjoint(a, b, P(1 << 47), *ng, bc, 0, 0.01, 1.4, P(1 << 45), 1 << 40, 1, None,
                                      None) == -1


def test_autotune_adjoint_rejects_bad_arguments(lib):
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    f = lib.hydro_autotune_adjoint
    a, b, c, w = P(4096), P(1 << 44), P(1 << 45), P(1 << 46)
    assert f(a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, w, 1 << 30, 0, None, None) == -1      # reps < 1
    assert f(a, b, c, 1, 1, 1, bc, 2, 0.01, 1.4, w, 1 << 30, 1, None, None) == -1      # dtype
    assert f(a, b, c, 1, 1, 1, bc, 0, -0.01, 1.4, w, 1 << 30, 1, None, None) == -1     # dx
    assert f(a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, w, 16, 1, None, None) == -1           # workspace too small
    assert f(a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, None, 1 << 30, 1, None, None) == -1   # no workspace


@pytest.mark.parametrize("ng", [(1 << 19, 1, 1), (1, 1, 1 << 19), (1 << 14, 1 << 14, 1)])
def test_adjoint_entry_points_reject_their_extra_limits(lib, ng):
    """The level adjoint and the ghost gather also need every axis below 2^19
    groups and fewer than 2^28 - 1 groups."""
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    a, b = P(4096), P(1 << 46)
    assert lib.hydro_advance_level_adjoint(a, b, P(1 << 47), *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None, P(1 << 45),
                                           1 << 62, None) == -1
    assert lib.hydro_gather_ghost_adjoint(a, b, *ng, 3, 0, bc, None) == -1
