"""CFL epilogue of the batched multi-level step (Sec. 2.6 Eq. 2 reduced in
the persistent launch) and the W-cycle whose coarse time-step is chosen on
the device (Sec. 2.1: dt_l = dt_0 / 2^l, dt_0 = min_l 2^l dt_l of the levels'
states).

* per-patch time-steps of every level's output equal hydro_dt on it, bit
  for bit; the folded minimum equals min_l scale_l min(dt_patch_l); the
  reset word becomes +inf; the states equal the launch without CFL outputs
* the adaptive W-cycle (eager and as a replayed graph of 6 coarse steps)
  equals a per-level W-cycle driven from the host with the time-steps
  hydro_dt gives on each coarse step's final states, bit for bit, and its
  device word holds the next coarse step's dt_0
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def hydro():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1712_07070_amd import hydro as h
    h.load()
    return h


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _levels():
    return W.sedov_levels(((2, 2, 2), (2, 2, 6), (2, 4, 6)), dx0=1.0 / 32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_cfl_outputs_equal_hydro_dt(hydro, dtype):
    say("batched cfl outputs", dtype)
    lvs = _levels()
    ins = [torch.from_numpy(np.ascontiguousarray(lv.U)).to(dtype).cuda() for lv in lvs]
    dt0 = 0.3 * min(float(oracle.dt_patch(lv.U, lv.dx, lv.gamma).min()) * 2 ** l for l, lv in enumerate(lvs))
    work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
    plain = [torch.empty_like(u) for u in ins]
    hydro.advance_batched([(u, o, lv.ng, lv.bc, dt0 / 2 ** l, lv.dx) for l, (u, o, lv) in
                           enumerate(zip(ins, plain, lvs))], G53, work)
    words = torch.tensor([float("inf"), 7.0], dtype=torch.float64, device="cuda")
    outs = [torch.empty_like(u) for u in ins]
    patches = [torch.full((lv.n_groups * 8,), -1.0, dtype=torch.float64, device="cuda") for lv in lvs]
    ent = []
    for l, (u, o, lv, p) in enumerate(zip(ins, outs, lvs, patches)):
        cfl = {"c_cfl": 0.5, "dt_next_scale": 2.0 ** l, "dt_next": words[0:1], "dt_patch": p}
        if l == 1:
            cfl["dt_reset"] = words[1:2]
        ent.append((u, o, lv.ng, lv.bc, dt0 / 2 ** l, lv.dx, None, cfl))
    hydro.advance_batched(ent, G53, work)
    torch.cuda.synchronize()
    want = float("inf")
    for l, (o, lv, p) in enumerate(zip(outs, lvs, patches)):
        assert torch.equal(o, plain[l])
        ref = hydro.cfl_dt(o, lv.dx, G53, 0.5)
        assert torch.equal(p.view(-1, 8), ref), l
        want = min(want, float(ref.min()) * 2 ** l)
    w = words.cpu().numpy()
    assert w[0] == want and np.isinf(w[1])


@pytest.mark.parametrize("graph", [False, True])
def test_adaptive_wcycle_matches_host_driven(hydro, graph):
    say("adaptive w-cycle", "graph" if graph else "eager")
    lvs = _levels()
    geo = [(lv.ng, lv.dx, lv.bc) for lv in lvs]
    dt0 = 0.3 * min(float(oracle.dt_patch(lv.U, lv.dx, lv.gamma).min()) * 2 ** l for l, lv in enumerate(lvs))
    ml = hydro.MultiLevel(geo, G53, dt0, batched=True, adaptive=True, c_cfl=0.5)
    ref = hydro.MultiLevel(geo, G53, dt0, batched=False)
    for l, lv in enumerate(lvs):
        ml.load_state(l, torch.from_numpy(lv.U).cuda())
        ref.load_state(l, torch.from_numpy(lv.U).cuda())
    n = 6
    if graph:
        g = ml.capture(n)
        _ = torch.ones(1000, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        g.close()
    else:
        for _ in range(n):
            ml.coarse_step()
    dt = dt0
    for _ in range(n):
        ref.dt0 = dt
        ref.coarse_step()
        dt = min(float(hydro.cfl_dt(ref.state(l), geo[l][1], G53, 0.5).min()) * 2 ** l for l in range(len(lvs)))
    torch.cuda.synchronize()
    for l in range(len(lvs)):
        assert torch.equal(ml.state(l), ref.state(l)), l
    assert float(ml.dt_coarse().cpu()[0]) == dt
    assert dt != dt0
    assert int(ml.n_bad.cpu()[0]) == 0 and int(ref.n_bad.cpu()[0]) == 0


def test_adaptive_autotune_keeps_words_and_state(hydro):
    """Tuning an adaptive W-cycle leaves the levels and the time-step words
    untouched (the tuner's CFL outputs go to scratch words)."""
    say("adaptive autotune")
    lvs = _levels()
    geo = [(lv.ng, lv.dx, lv.bc) for lv in lvs]
    dt0 = 0.3 * min(float(oracle.dt_patch(lv.U, lv.dx, lv.gamma).min()) * 2 ** l for l, lv in enumerate(lvs))
    ml = hydro.MultiLevel(geo, G53, dt0, batched=True, adaptive=True)
    for l, lv in enumerate(lvs):
        ml.load_state(l, torch.from_numpy(lv.U).cuda())
    before = ml.dtw.clone()
    saved = hydro.get_batched_variant(torch.float64)
    try:
        ml.autotune(reps=1)
        torch.cuda.synchronize()
        assert torch.equal(ml.dtw, before)
        for l, lv in enumerate(lvs):
            assert np.array_equal(ml.state(l).cpu().numpy(), lv.U)
    finally:
        hydro.set_batched_variant(torch.float64, saved)


def test_batched_cfl_argument_errors(hydro):
    lvs = _levels()
    lv = lvs[0]
    u = torch.from_numpy(lv.U).cuda()
    o = torch.empty_like(u)
    work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
    w = torch.full((3,), float("inf"), dtype=torch.float64, device="cuda")
    with pytest.raises(hydro.HydroError):   # CFL output without a CFL factor
        hydro.advance_batched([(u, o, lv.ng, lv.bc, 1e-3, lv.dx, None, {"dt_next": w[0:1]})], G53, work)
    with pytest.raises(hydro.HydroError):   # reset word is the word read
        hydro.advance_batched([(u, o, lv.ng, lv.bc, 1e-3, lv.dx, w[0:1], {"c_cfl": 0.5, "dt_reset": w[0:1]})],
                              G53, work)
    with pytest.raises(hydro.HydroError):   # reduction into the word read
        hydro.advance_batched([(u, o, lv.ng, lv.bc, 1e-3, lv.dx, w[0:1], {"c_cfl": 0.5, "dt_next": w[0:1]})],
                              G53, work)
