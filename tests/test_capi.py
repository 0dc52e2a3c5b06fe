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


class Ctx:
    """A hydro_ctx for the duration of a with-block."""

    def __init__(self, lib, path=None):
        self.lib, self.path = lib, path

    def __enter__(self):
        h = ctypes.c_void_p()
        assert self.lib.hydro_ctx_create(ctypes.byref(h), None if self.path is None else os.fsencode(self.path)) == 0
        self.h = h
        return h

    def __exit__(self, *a):
        assert self.lib.hydro_ctx_destroy(self.h) == 0


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
    assert lib.hydro_advance_level(None, a, b, *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None, None, 0.5, None, None,
                                   None, None) == -1
    assert lib.hydro_advance_level_adjoint(None, a, b, P(1 << 47), *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None,
                                           P(1 << 45), 1 << 40, None) == -1
    assert lib.hydro_fill_ghosts(a, b, *ng, 3, 0, bc, None) == -1
    assert lib.hydro_gather_ghost_adjoint(a, b, *ng, 3, 0, bc, None) == -1
    with Ctx(lib) as c:
        assert lib.hydro_autotune_adjoint(c, a, b, P(1 << 47), *ng, bc, 0, 0.01, 1.4, P(1 << 45), 1 << 40, 1, None,
                                          None) == -1


def test_autotune_adjoint_rejects_bad_arguments(lib):
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    f = lib.hydro_autotune_adjoint
    a, b, c, w = P(4096), P(1 << 44), P(1 << 45), P(1 << 46)
    with Ctx(lib) as x:
        assert f(x, a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, w, 1 << 30, 0, None, None) == -1      # reps < 1
        assert f(x, a, b, c, 1, 1, 1, bc, 2, 0.01, 1.4, w, 1 << 30, 1, None, None) == -1      # dtype
        assert f(x, a, b, c, 1, 1, 1, bc, 0, -0.01, 1.4, w, 1 << 30, 1, None, None) == -1     # dx
        assert f(x, a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, w, 16, 1, None, None) == -1           # workspace too small
        assert f(x, a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, None, 1 << 30, 1, None, None) == -1   # no workspace
    assert f(None, a, b, c, 1, 1, 1, bc, 0, 0.01, 1.4, w, 1 << 30, 1, None, None) == -1      # tuning needs a ctx


@pytest.mark.parametrize("ng", [(1 << 19, 1, 1), (1, 1, 1 << 19), (1 << 14, 1 << 14, 1)])
def test_adjoint_entry_points_reject_their_extra_limits(lib, ng):
    """The level adjoint and the ghost gather also need every axis below 2^19
    groups and fewer than 2^28 - 1 groups."""
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    a, b = P(4096), P(1 << 46)
    assert lib.hydro_advance_level_adjoint(None, a, b, P(1 << 47), *ng, bc, 0, 1e-3, 0.01, 1.4, 1, 1.5, None,
                                           P(1 << 45), 1 << 62, None) == -1
    assert lib.hydro_gather_ghost_adjoint(a, b, *ng, 3, 0, bc, None) == -1


# ------------------------------------------------------------- contexts ----

def _level(lib, ctx, ng=(2, 2, 2), dtype=0, cfl=False):
    """hydro_advance_level with valid arguments and fake device pointers: it
    returns before any HIP call only if the shape lookup refuses."""
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    return lib.hydro_advance_level(ctx, P(4096), P(1 << 44), *ng, bc, dtype, 1e-3, 0.01, 1.4, 1, 1.5, None, None,
                                   0.5, P(1 << 45) if cfl else None, None, None, None)


def test_status_codes_of_the_context_api(lib):
    assert lib.hydro_strerror(1).startswith(b"unphysical")
    assert lib.hydro_strerror(-3).startswith(b"no tuned")
    assert lib.hydro_strerror(-4).startswith(b"tuning cache")
    assert lib.hydro_ctx_create(None, None) == -1
    assert lib.hydro_ctx_destroy(None) == -1
    assert lib.hydro_check_unphysical(None, None, None) == -1


def test_two_contexts_keep_separate_selections(lib):
    with Ctx(lib) as a, Ctx(lib) as b:
        assert lib.hydro_set_level_variant(a, 0, 1, 3) == 0
        assert lib.hydro_set_batched_variant(b, 1, 5) == 0
        assert lib.hydro_set_adjoint_variant(a, 1, 1) == 0
        assert lib.hydro_get_level_variant(a, 0, 1) == 3
        assert lib.hydro_get_level_variant(b, 0, 1) == 6          # default
        assert lib.hydro_get_batched_variant(b, 1) == 5
        assert lib.hydro_get_batched_variant(a, 1) == 0
        assert lib.hydro_get_adjoint_variant(a, 1) == 1
        assert lib.hydro_get_adjoint_variant(b, 1) == 0
    # setters need a context, getters without one report the defaults
    assert lib.hydro_set_level_variant(None, 0, 1, 1) == -1
    assert lib.hydro_get_level_variant(None, 0, 1) == 6
    assert lib.hydro_set_variant(None, 0, 1) == -1


def test_require_tuned_refuses_untuned_launches(lib, tmp_path):
    path = tmp_path / "tune.json"
    path.write_text('{"version": 1, "entries": {\n  "level/f64/plain/2x2x2": 1,\n  "adjoint/f32/4x4x4": 0\n}}\n')
    with Ctx(lib, str(path)) as c:
        assert lib.hydro_ctx_num_tuned(c) == 2
        assert lib.hydro_ctx_set_require_tuned(c, 1) == 0
        assert _level(lib, c, ng=(2, 2, 3)) == -3               # no entry for this lattice
        assert _level(lib, c, ng=(2, 2, 2), cfl=True) == -3     # nor for the CFL form
        assert _level(lib, c, ng=(2, 2, 2), dtype=1) == -3      # nor for FP32
        # an explicit selection configures the form
        assert lib.hydro_set_level_variant(c, 0, 1, 2) == 0
        assert lib.hydro_get_level_variant(c, 0, 1) == 2
    with Ctx(lib) as c:  # without the requirement the default is used (no refusal)
        assert lib.hydro_ctx_num_tuned(c) == 0


def test_tune_cache_round_trip_and_malformed_files(lib, tmp_path):
    path = tmp_path / "tune.json"
    path.write_text('{"version": 1, "entries": {"batched/f64/8x8x8+8x8x24": 4, "level/f32/cfl/16x16x16": 3}}')
    with Ctx(lib, str(path)) as c:
        assert lib.hydro_ctx_num_tuned(c) == 2
        path.unlink()
        assert lib.hydro_ctx_save(c) == 0
    text = path.read_text()
    assert '"batched/f64/8x8x8+8x8x24": 4' in text and '"level/f32/cfl/16x16x16": 3' in text
    with Ctx(lib, str(path)) as c:
        assert lib.hydro_ctx_num_tuned(c) == 2
        # an explicit selection replaces the tuned entries of its dtype and form
        assert lib.hydro_set_level_variant(c, 1, 1, 0) == 0
        assert lib.hydro_ctx_num_tuned(c) == 1
    for bad in ('{"entries": {"a": "x"}}', '{"entries": {"a" 1}}', "[1, 2]", '{"entries": {"a": -2}}'):
        path.write_text(bad)
        h = ctypes.c_void_p()
        assert lib.hydro_ctx_create(ctypes.byref(h), os.fsencode(str(path))) == -4, bad
    # a missing file is an empty cache
    h = ctypes.c_void_p()
    assert lib.hydro_ctx_create(ctypes.byref(h), os.fsencode(str(tmp_path / "none.json"))) == 0
    assert lib.hydro_ctx_num_tuned(h) == 0
    assert lib.hydro_ctx_destroy(h) == 0


def test_autotune_needs_a_context_and_cfl_scratch(lib):
    P = ctypes.c_void_p
    bc = (ctypes.c_int32 * 6)(0, 0, 0, 0, 0, 0)
    f = lib.hydro_autotune
    a, b, s = P(4096), P(1 << 44), P(1 << 45)
    need = 8 * (3 + 8 * 8)
    assert f(None, a, b, 2, 2, 2, bc, 0, 0.01, 1.4, s, need, 1, None, None) == -1
    with Ctx(lib) as c:
        assert f(c, a, b, 2, 2, 2, bc, 0, 0.01, 1.4, s, need - 8, 1, None, None) == -1      # scratch too small
        assert f(c, a, b, 2, 2, 2, bc, 0, 0.01, 1.4, None, need, 1, None, None) == -1       # no scratch
        assert f(c, a, P(4096 + 64), 2, 2, 2, bc, 0, 0.01, 1.4, s, need, 1, None, None) == -1   # out overlaps in
        assert f(c, a, b, 2, 2, 2, bc, 0, 0.01, 1.4, P(4096 + 64), need, 1, None, None) == -1   # scratch overlaps
        assert lib.hydro_ctx_num_tuned(c) == 0
