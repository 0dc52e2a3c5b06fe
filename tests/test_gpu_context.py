"""GPU checks of the context API: tuning through a context, the tuning cache
saved and reloaded, a context that requires tuned shapes, two contexts in one
process, and the unphysical-status helper."""

import sys

import numpy as np
import pytest

from paper_1712_07070_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hydro():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1712_07070_amd import hydro as h
    h.load()
    return h


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_tune_save_reload_require_tuned(hydro, tmp_path):
    say("context tune / cache / require_tuned")
    lv = W.white_noise(64)
    U = torch.from_numpy(lv.U).cuda()
    cache = str(tmp_path / "tune.json")
    a = hydro.Context(cache)
    best, times = hydro.autotune(U, lv.ng, lv.bc, lv.dx, lv.gamma, reps=2, ctx=a)
    assert 0 <= best < hydro.num_variants() and len(times) == 2 * hydro.num_variants()
    assert a.num_tuned() == 2                               # both kernel forms of this lattice
    ref = hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, ctx=a)
    a.close()
    # a new context reads the cache and, requiring tuned shapes, runs the
    # tuned lattice and refuses an untuned one
    b = hydro.Context(cache, require_tuned=True)
    assert b.num_tuned() == 2
    got = hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, ctx=b)
    assert torch.equal(got, ref)
    small = U[:8].contiguous()
    with pytest.raises(hydro.HydroError) as e:
        hydro.advance_level(small, (2, 2, 2), lv.bc, 1e-3, lv.dx, lv.gamma, ctx=b)
    assert e.value.status == hydro.HYDRO_ENOTUNED
    b.close()


def test_two_contexts_and_every_shape_give_the_same_bits(hydro):
    say("two contexts")
    lv = W.white_noise(64)
    U = torch.from_numpy(lv.U).cuda()
    a, b = hydro.Context(), hydro.Context()
    hydro.set_variant(torch.float64, 3, ctx=a)
    hydro.set_variant(torch.float64, 1, ctx=b)
    assert hydro.get_variant(torch.float64, ctx=a) == 3 and hydro.get_variant(torch.float64, ctx=b) == 1
    ra = hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, ctx=a)
    rb = hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, ctx=b)
    assert torch.equal(ra, rb)
    a.close()
    b.close()


def test_graphs_are_owned_by_their_context(hydro):
    say("graph ownership")
    lv = W.white_noise(32)
    U = torch.from_numpy(lv.U).cuda()
    out = torch.empty_like(U)
    ctx = hydro.Context()
    g = hydro.Graph(ctx).capture(lambda: hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, out=out,
                                                             ctx=ctx))
    ref = hydro.advance_level(U, lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    # destroying the context frees the graph it still owns
    ctx.close()
    g.handle = None


def test_check_unphysical(hydro):
    say("check unphysical")
    lv = W.white_noise(32)
    U = lv.U.copy()
    n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    hydro.advance_level(torch.from_numpy(U).cuda(), lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, n_bad=n_bad)
    assert hydro.check_unphysical(n_bad) == 0
    U[3, 4, 5, 6, 7] = -1.0                                  # negative total energy in one cell
    hydro.advance_level(torch.from_numpy(U).cuda(), lv.ng, lv.bc, 1e-3, lv.dx, lv.gamma, n_bad=n_bad)
    assert hydro.check_unphysical(n_bad) > 0
