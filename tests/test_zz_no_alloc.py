"""The allocation-free batched entry point (hydro_advance_batched_noalloc)
against hydro_advance_batched with a caller work buffer: identical bits, on
two calls in a row (the second with fewer levels and groups), in FP64 and
FP32, with and without the unphysical counter."""

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


def _levels(lattices, dtype, seed):
    out = []
    for i, ng in enumerate(lattices):
        n = [16 * v for v in ng]
        rng = np.random.default_rng(seed + i)
        shape = (n[2], n[1], n[0])
        grid = W.conserved(rng.uniform(0.5, 2, shape), rng.normal(0, 0.3, shape), rng.normal(0, 0.3, shape),
                           rng.normal(0, 0.3, shape), rng.uniform(0.5, 2, shape), 5.0 / 3.0)
        U = torch.from_numpy(np.ascontiguousarray(W.grid_to_groups(grid).astype(dtype))).cuda()
        dx = 1.0 / (64 * 2 ** i)
        out.append((U, ng, (0,) * 6, 0.1 * dx, dx))
    return out


def _run(hydro, lv, noalloc):
    outs = [torch.full_like(U, float("nan")) for U, *_ in lv]
    n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    entries = [(U, o, ng, bc, dt, dx) for (U, ng, bc, dt, dx), o in zip(lv, outs)]
    if noalloc:
        hydro.advance_batched_noalloc(entries, 5.0 / 3.0, n_bad=n_bad)
    else:
        work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
        hydro.advance_batched(entries, 5.0 / 3.0, work, n_bad=n_bad)
    torch.cuda.synchronize()
    return [o.cpu() for o in outs], int(n_bad.cpu()[0])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_batched_matches_work_buffer_form(hydro, dtype):
    print("noalloc batched", dtype.__name__, file=sys.stderr, flush=True)
    big = _levels([(2, 2, 2), (2, 2, 4), (2, 4, 4)], dtype, 11)
    small = _levels([(1, 2, 2)], dtype, 23)
    for lv in (big, small):
        ref, nb_ref = _run(hydro, lv, noalloc=False)
        got, nb_got = _run(hydro, lv, noalloc=True)
        assert nb_ref == nb_got == 0
        for r, g in zip(ref, got):
            assert not torch.isnan(g).any()
            assert torch.equal(r, g)
    # and once more with the large input after the small one
    ref, _ = _run(hydro, big, noalloc=False)
    got, _ = _run(hydro, big, noalloc=True)
    assert all(torch.equal(r, g) for r, g in zip(ref, got))
