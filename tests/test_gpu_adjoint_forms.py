"""Both forms of the step adjoint (fused sweep; two kernels with a face
workspace) against each other and against the oracle's exact JVP."""

import sys

import numpy as np
import pytest

import oracle
from tests.test_oracle_scheme import smooth_all_fields

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


def _forms(hydro, dtype, fn):
    saved = hydro.get_adjoint_variant(dtype)
    try:
        out = []
        for form in (0, 1):
            hydro.set_adjoint_variant(dtype, form)
            out.append(fn())
        return out
    finally:
        hydro.set_adjoint_variant(dtype, saved)


@pytest.mark.parametrize("n,bc", [(32, (0, 0, 0, 0, 0, 0)), (48, (1, 0, 0, 1, 1, 0))])
def test_level_adjoint_forms_agree_with_oracle(hydro, n, bc):
    print("adjoint forms", n, bc, file=sys.stderr, flush=True)
    U, ng, dx = smooth_all_fields(n)
    rng = np.random.default_rng(11)
    v = rng.normal(size=U.shape)
    w = rng.normal(size=U.shape)
    dt = 0.3 * dx
    _, Jv, _ = oracle.rollout_jvp(U, v, ng, 3, bc, 1, dt, dx, G53)
    lhs = float(np.sum(Jv * w))
    t, tw = torch.from_numpy(U).cuda(), torch.from_numpy(w).cuda()
    outs = _forms(hydro, torch.float64,
                  lambda: hydro.advance_level_adjoint(t, tw, ng, bc, dt, dx, G53).cpu().numpy())
    for o in outs:
        rhs = float(np.sum(v * o))
        assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), abs(rhs)), (lhs, rhs)
    scale = np.max(np.abs(outs[0]))
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-12 * scale


def test_padded_adjoint_forms_agree(hydro):
    print("padded adjoint forms", file=sys.stderr, flush=True)
    U, ng, dx = smooth_all_fields(32)
    pad = oracle.fill_ghosts(U, ng, 3, (0,) * 6)
    w = np.random.default_rng(12).normal(size=(pad.shape[0], 5, 16, 16, 16))
    t, tw = torch.from_numpy(pad).cuda(), torch.from_numpy(w).cuda()
    outs = _forms(hydro, torch.float64, lambda: hydro.advance_adjoint(t, tw, 0.3 * dx, dx, G53).cpu().numpy())
    scale = np.max(np.abs(outs[0]))
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-12 * scale
    # FP32 forms agree to FP32 round-off
    t32, tw32 = t.float(), tw.float()
    o32 = _forms(hydro, torch.float32, lambda: hydro.advance_adjoint(t32, tw32, 0.3 * dx, dx, G53).cpu().numpy())
    assert np.max(np.abs(o32[0] - o32[1])) <= 1e-5 * np.max(np.abs(o32[0]))


def test_autotune_adjoint_selects_a_form(hydro):
    print("adjoint autotune", file=sys.stderr, flush=True)
    U, ng, dx = smooth_all_fields(32)
    t = torch.from_numpy(U).cuda()
    g = torch.ones_like(t)
    saved = hydro.get_adjoint_variant(torch.float64)
    try:
        form, times = hydro.autotune_adjoint(t, g, ng, (0,) * 6, dx, G53, reps=1)
        assert form in (0, 1) and len(times) == 2 and all(x > 0 for x in times)
        assert form == (1 if times[1] < times[0] else 0)
        assert hydro.get_adjoint_variant(torch.float64) == form
        # the tuned form gives the cotangents of either form
        a = hydro.advance_level_adjoint(t, g, ng, (0,) * 6, 0.3 * dx, dx, G53)
        hydro.set_adjoint_variant(torch.float64, 1 - form)
        b = hydro.advance_level_adjoint(t, g, ng, (0,) * 6, 0.3 * dx, dx, G53)
        assert float((a - b).abs().max()) <= 1e-12 * float(a.abs().max())
        # argument errors come back as status codes, the selection is kept
        hydro.set_adjoint_variant(torch.float64, 0)
        with pytest.raises(hydro.HydroError):
            hydro.autotune_adjoint(t, g, ng, (0,) * 6, -dx, G53)
        assert hydro.get_adjoint_variant(torch.float64) == 0
    finally:
        hydro.set_adjoint_variant(torch.float64, saved)
