"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times (the fused level step with its CFL epilogue, the batched
multi-level kernel, the level adjoint): sampled groups against the oracle,
and properties that hold at any size."""

import sys

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W
from tests.oracle_runs import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def hydro():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1712_07070_amd import hydro as h
    h.load()
    return h


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fused_step_sampled(hydro, lv, dtype, n_sample, seed):
    """One fused level step (ghost fill in the loads, CFL epilogue) at dt from
    the GPU CFL kernel; sampled groups and their patch time-steps against the
    oracle (FP32: the oracle starts from the FP32-rounded state)."""
    U = np.ascontiguousarray(lv.U.astype(dtype))
    t = torch.from_numpy(U).cuda()
    G = lv.n_groups
    dt_now = torch.empty(1, dtype=torch.float64, device="cuda")
    dt_next = torch.empty(1, dtype=torch.float64, device="cuda")
    dt_reset = torch.empty(1, dtype=torch.float64, device="cuda")
    dt_patch = torch.empty(8 * G, dtype=torch.float64, device="cuda")
    U64 = U.astype(np.float64)
    pad = oracle.fill_ghosts(U64, lv.ng, 3, lv.bc)
    dt = float(oracle.dt_patch(pad, lv.dx, lv.gamma).min())
    dt_now.fill_(dt)
    dt_next.fill_(float("inf"))  # the epilogue folds its minimum into this
    out = hydro.advance_level(t, lv.ng, lv.bc, 1.0, lv.dx, lv.gamma, dt_dev=dt_now, c_cfl=0.5, dt_next=dt_next,
                              dt_patch_next=dt_patch, dt_reset=dt_reset)
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(G, n_sample, replace=False))
    ref, _ = oracle.mhm_step(pad[sample], dt, lv.dx, lv.gamma)
    del pad
    got = host(out)
    assert_parity(got[sample], ref, TOL[dtype])
    # the epilogue's patch time-steps of the written state, recomputed by the
    # oracle from the GPU's output (same state, so the same bits)
    gp = host(dt_patch).reshape(G, 8)[sample]
    opad = oracle.fill_ghosts(got.astype(np.float64), lv.ng, 3, lv.bc)[sample]
    np.testing.assert_array_equal(gp, oracle.dt_patch(opad, lv.dx, lv.gamma))
    assert float(host(dt_next)[0]) == float(host(dt_patch).min())
    return got


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_shear_layer_256_fused_step_sampled(hydro, dtype):
    say("fullsize shear 256^3 fused", dtype.__name__)
    fused_step_sampled(hydro, W.shear_layer(256), dtype, 16, 1)


def test_turbulence_384_fp32_fused_step_sampled(hydro):
    say("fullsize turbulence 384^3 fp32 fused")
    lv = W.turbulence(384)
    got = fused_step_sampled(hydro, lv, np.float32, 12, 2)
    # conservation of mass over the periodic box (FP32 sums in FP64)
    m0 = float(lv.U.astype(np.float32).astype(np.float64)[:, 0].sum())
    assert abs(float(got.astype(np.float64)[:, 0].sum()) - m0) <= 1e-5 * m0


def test_amr_full_size_batched_vs_per_level_and_oracle(hydro):
    """The 3-level workload at its full size (512 / 1536 / 3072 groups): one
    batched launch per W-cycle stage 0 equals one launch per level, bitwise,
    and sampled groups of every level match the oracle."""
    say("fullsize amr")
    lvs = W.sedov_levels()
    ins = [torch.from_numpy(lv.U).cuda() for lv in lvs]
    dt0 = 0.3 * min(float(oracle.dt_patch(oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc), lv.dx, lv.gamma).min()) * 2 ** l
                    for l, lv in enumerate(lvs))
    ref = [hydro.advance_level(t, lv.ng, lv.bc, dt0 / 2 ** l, lv.dx, lv.gamma) for l, (t, lv) in
           enumerate(zip(ins, lvs))]
    work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
    outs = [torch.empty_like(t) for t in ins]
    hydro.advance_batched([(t, o, lv.ng, lv.bc, dt0 / 2 ** l, lv.dx) for l, (t, o, lv) in
                           enumerate(zip(ins, outs, lvs))], lvs[0].gamma, work)
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    rng = np.random.default_rng(3)
    for l, (lv, r) in enumerate(zip(lvs, ref)):
        sample = np.sort(rng.choice(lv.n_groups, 6, replace=False))
        pad = oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc)[sample]
        o, _ = oracle.mhm_step(pad, dt0 / 2 ** l, lv.dx, lv.gamma)
        assert_parity(host(r)[sample], o, TOL[np.float64])


def test_smooth_wave_128_adjoint_full_size(hydro):
    """The level adjoint at the workload's full size (512 groups): <J v, w> from
    the oracle's dual-number JVP against <v, J^T w> from the GPU."""
    say("fullsize adjoint 128^3")
    lv, _ = W.smooth_wave(128, smooth_vp=0.01)
    rng = np.random.default_rng(4)
    v = rng.normal(size=lv.U.shape)
    w = rng.normal(size=lv.U.shape)
    dt = 0.2 * lv.dx
    _, Jv, _ = oracle.rollout_jvp(lv.U, v, lv.ng, 3, lv.bc, 1, dt, lv.dx, lv.gamma)
    JTw = host(hydro.advance_level_adjoint(torch.from_numpy(lv.U).cuda(), torch.from_numpy(w).cuda(), lv.ng, lv.bc,
                                           dt, lv.dx, lv.gamma))
    lhs, rhs = float(np.sum(Jv * w)), float(np.sum(v * JTw))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def _neighbourhood(U, ng, g):
    """The 3x3x3 groups around group g of a device level (periodic wrap),
    copied to the host as a 3x3x3 level whose centre is group g."""
    ngx, ngy, ngz = ng
    gx, gy, gz = g % ngx, (g // ngx) % ngy, g // (ngx * ngy)
    idx = [(((gz + dz) % ngz) * ngy + (gy + dy) % ngy) * ngx + (gx + dxx) % ngx
           for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dxx in (-1, 0, 1)]
    return host(U[torch.tensor(idx, device=U.device)]).astype(np.float64)


def test_level_beyond_32bit_offsets_fp32(hydro):
    """A level of more than 2^32 elements (64 x 64 x 52 groups, FP32, 17.4 GB
    per copy) runs the kernels with 64-bit element offsets: sampled groups,
    the last ones of the level included, against the oracle on their 3x3x3
    neighbourhoods (the centre group's ghost cells all lie inside it), their
    patch time-steps bit for bit, and the batched kernel bit for bit against
    the level step."""
    ng, bc = (64, 64, 52), (0, 0, 0, 0, 0, 0)
    G = ng[0] * ng[1] * ng[2]
    assert G * 5 * 4096 > 2 ** 32
    say("level beyond 32-bit offsets", G)
    U = W.white_noise_device(ng, torch.float32, "cuda")
    dx, gamma, dt = 1.0 / 1024, 5.0 / 3.0, 1e-5
    dt_next = torch.full((1,), float("inf"), dtype=torch.float64, device="cuda")
    dt_patch = torch.empty(8 * G, dtype=torch.float64, device="cuda")
    out = hydro.advance_level(U, ng, bc, dt, dx, gamma, c_cfl=0.5, dt_next=dt_next, dt_patch_next=dt_patch)
    for g in (0, G // 2 + 17, G - ng[0] * ng[1] - 1, G - 2, G - 1):
        pad = oracle.fill_ghosts(_neighbourhood(U, ng, g), (3, 3, 3), 3, bc)[13:14]
        ref, _ = oracle.mhm_step(pad, dt, dx, gamma)
        assert_parity(host(out[g:g + 1]), ref, TOL[np.float32], g)
        opad = oracle.fill_ghosts(_neighbourhood(out, ng, g), (3, 3, 3), 3, bc)[13:14]
        np.testing.assert_array_equal(host(dt_patch[8 * g:8 * g + 8]), oracle.dt_patch(opad, dx, gamma)[0])
    del dt_patch
    work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
    out2 = torch.empty_like(U)
    hydro.advance_batched([(U, out2, ng, bc, dt, dx)], gamma, work)
    assert torch.equal(out2, out)
    assert not host(work).any()
