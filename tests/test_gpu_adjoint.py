"""GPU adjoint: the hand-written VJP of the MHM step against the oracle.

The oracle gives exact Jacobian-vector products J v (dual numbers through its
own step); the HIP path gives J^T w.  For random v, w the two sides of
<J v, w> = <v, J^T w> must agree to round-off (FP64: 1e-11 relative).  States
vary smoothly along every axis so that no limiter / wave-speed branch sits at
a switch (where the two codes could legitimately take different one-sided
derivatives).  The rollout gradient is also checked against central finite
differences of the GPU forward and for bitwise invariance under the
checkpoint interval."""

import sys

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


STEP_CASES = {
    "full": dict(theta=1.5, scheme=1),
    "first-order": dict(theta=1.5, scheme=1 | (1 << 10)),
    "davis": dict(theta=1.5, scheme=1 | (1 << 8)),
    "theta=1": dict(theta=1.0, scheme=1),
    "theta=2": dict(theta=2.0, scheme=1),
}


@pytest.mark.parametrize("case", list(STEP_CASES))
@pytest.mark.parametrize("state", ["smooth", "white-noise"])
def test_step_adjoint_dot_product(hydro, case, state):
    say("step adjoint", case, state)
    if state == "smooth":
        U, ng, dx = smooth_all_fields(32)
    else:
        lv = W.white_noise(32)
        U, ng, dx = lv.U, lv.ng, lv.dx
    kw = STEP_CASES[case]
    pad = oracle.fill_ghosts(U, ng, 3, (0,) * 6)
    rng = np.random.default_rng(1)
    v = rng.normal(size=pad.shape)
    w = rng.normal(size=(pad.shape[0], 5, 16, 16, 16))
    dt = 0.3 * dx
    _, Jv, _ = oracle.mhm_step_jvp(pad, v, dt, dx, G53, kw["theta"], kw["scheme"])
    JTw = host(hydro.advance_adjoint(dev(pad), dev(w), dt, dx, G53, kw["theta"], kw["scheme"]))
    lhs, rhs = float(np.sum(Jv * w)), float(np.sum(v * JTw))
    assert rel(lhs, rhs) <= 1e-11, (lhs, rhs)


def test_step_adjoint_elementwise(hydro):
    """(J^T w)_j = <J e_j, w> for input elements in the interior, on the
    group boundary, in the 2-deep ghost slab and on a ghost edge."""
    say("step adjoint elementwise")
    U, ng, dx = smooth_all_fields(16)
    pad = oracle.fill_ghosts(U, ng, 3, (0,) * 6)
    w = np.random.default_rng(2).normal(size=(1, 5, 16, 16, 16))
    dt = 0.3 * dx
    JTw = host(hydro.advance_adjoint(dev(pad), dev(w), dt, dx, G53))
    g = 3
    picks = [(0, 7 + g, 5 + g, 9 + g), (4, 0 + g, 8 + g, 3 + g), (1, 15 + g, 15 + g, 15 + g), (2, -1 + g, 4 + g, 6 + g),
             (3, 8 + g, -2 + g, 10 + g), (0, -1 + g, -1 + g, 7 + g), (4, 17 + g, 3 + g, 3 + g), (1, -3 + g, 4 + g, 4 + g)]
    for q, z, y, x in picks:
        e = np.zeros_like(pad)
        e[0, q, z, y, x] = 1.0
        _, Je, _ = oracle.mhm_step_jvp(pad, e, dt, dx, G53)
        ref = float(np.sum(Je * w))
        got = float(JTw[0, q, z, y, x])
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), ((q, z, y, x), got, ref)


@pytest.mark.parametrize("n,bc", [(32, (0, 0, 0, 0, 0, 0)), (32, (1, 1, 0, 0, 1, 0)),
                                  (48, (1, 0, 0, 1, 1, 0))])   # one-sided periodic faces, 3 groups per axis
def test_level_adjoint_dot_product(hydro, n, bc):
    say("level adjoint", n, bc)
    U, ng, dx = smooth_all_fields(n)
    rng = np.random.default_rng(3)
    v = rng.normal(size=U.shape)
    w = rng.normal(size=U.shape)
    dt = 0.3 * dx
    _, Jv, _ = oracle.rollout_jvp(U, v, ng, 3, bc, 1, dt, dx, G53)
    JTw = host(hydro.advance_level_adjoint(dev(U), dev(w), ng, bc, dt, dx, G53))
    lhs, rhs = float(np.sum(Jv * w)), float(np.sum(v * JTw))
    assert rel(lhs, rhs) <= 1e-11, (lhs, rhs)


GATHER_CASES = [((1, 1, 1), 3, (0, 0, 0, 0, 0, 0)), ((1, 1, 1), 16, (1, 1, 0, 1, 1, 0)),
                 ((3, 2, 1), 3, (1, 0, 0, 1, 1, 1)), ((4, 1, 3), 2, (0, 1, 1, 0, 0, 0)),
                 ((2, 3, 2), 0, (1, 1, 1, 1, 1, 1)), ((3, 3, 3), 5, (1, 0, 0, 1, 1, 0))]


@pytest.mark.parametrize("ng,ghost,bc", GATHER_CASES)
def test_gather_ghost_adjoint_is_transpose_of_fill(hydro, ng, ghost, bc):
    """<fill(x), y> = <x, gather(y)>, with fill the oracle's ghost fill."""
    say("gather transpose", ng, ghost, bc)
    G = ng[0] * ng[1] * ng[2]
    P = 16 + 2 * ghost
    rng = np.random.default_rng(G * 100 + ghost)
    x = rng.normal(size=(G, 5, 16, 16, 16))
    y = rng.normal(size=(G, 5, P, P, P))
    lhs = float(np.sum(oracle.fill_ghosts(x, ng, ghost, bc) * y))
    gx = host(hydro.gather_ghost_adjoint(dev(y), ng, ghost, bc))
    rhs = float(np.sum(x * gx))
    assert rel(lhs, rhs) <= 1e-12, (lhs, rhs)
    # FP32 sums the same copies
    gx32 = host(hydro.gather_ghost_adjoint(dev(y.astype(np.float32)), ng, ghost, bc)).astype(np.float64)
    assert np.max(np.abs(gx32 - gx)) <= 1e-5 * max(1.0, np.max(np.abs(gx)))


@pytest.mark.parametrize("n,bc", [(32, (1, 1, 0, 0, 1, 0)), (48, (1, 0, 0, 1, 1, 0))])
def test_level_adjoint_equals_padded_adjoint_plus_gather(hydro, n, bc):
    """The level path (box + gather) and the padded path (hydro_advance_adjoint
    on filled groups, then hydro_gather_ghost_adjoint) sum the same terms in
    the same order."""
    say("level == padded + gather", n, bc)
    U, ng, dx = smooth_all_fields(n)
    w = dev(np.random.default_rng(n).normal(size=U.shape))
    dt = 0.3 * dx
    t = dev(U)
    a = hydro.advance_level_adjoint(t, w, ng, bc, dt, dx, G53)
    pad = hydro.fill_ghosts(t, ng, 3, bc)
    gpad = hydro.advance_adjoint(pad, w, dt, dx, G53)
    b = hydro.gather_ghost_adjoint(gpad, ng, 3, bc)
    assert torch.equal(a, b)


def test_level_adjoint_single_group_and_two_groups(hydro):
    """1 and 2 groups along an axis: periodic neighbours coincide with the group itself."""
    say("level adjoint small lattices")
    for n, ngs in ((16, (1, 1, 1)), (32, (2, 1, 1))):
        x = (np.arange(n) + 0.5) / n
        y = (np.arange(16) + 0.5) / 16
        Z, Y, X = np.meshgrid(y, y, x, indexing="ij")
        tp = 2 * np.pi
        rho = 1 + 0.1 * np.sin(tp * (X + Y + Z) + 0.2)
        u = 0.2 + 0.05 * np.cos(tp * (X - Y + 2 * Z) + 0.4)
        # every field varies along every axis (a field constant along an axis sits on the limiter kink)
        grid = W.conserved(rho, u, 0.1 * np.sin(tp * (X + 2 * Y + Z) + 0.9),
                           0.05 + 0.02 * np.cos(tp * (Y + X - Z) + 0.3),
                           1 + 0.05 * np.sin(tp * (X + Y - Z) + 0.1), G53)
        U = W.grid_to_groups(grid)
        rng = np.random.default_rng(n)
        v, w = rng.normal(size=U.shape), rng.normal(size=U.shape)
        dt = 0.2 / n
        _, Jv, _ = oracle.rollout_jvp(U, v, ngs, 3, (0,) * 6, 1, dt, 1 / n, G53)
        JTw = host(hydro.advance_level_adjoint(dev(U), dev(w), ngs, (0,) * 6, dt, 1 / n, G53))
        assert rel(float(np.sum(Jv * w)), float(np.sum(v * JTw))) <= 1e-11


def test_adjoint_fp32(hydro):
    say("adjoint fp32")
    U, ng, dx = smooth_all_fields(32)
    U32 = U.astype(np.float32)
    rng = np.random.default_rng(4)
    v = rng.normal(size=U.shape)
    w = rng.normal(size=U.shape).astype(np.float32)
    dt = 0.3 * dx
    _, Jv, _ = oracle.rollout_jvp(U32.astype(np.float64), v, ng, 3, (0,) * 6, 1, dt, dx, G53)
    JTw = host(hydro.advance_level_adjoint(dev(U32), dev(w), ng, (0,) * 6, dt, dx, G53)).astype(np.float64)
    assert rel(float(np.sum(Jv * w)), float(np.sum(v * JTw))) <= 1e-4


def test_adjoint_deterministic(hydro):
    say("adjoint determinism")
    U, ng, dx = smooth_all_fields(32)
    w = dev(np.random.default_rng(5).normal(size=U.shape))
    t = dev(U)
    outs = [hydro.advance_level_adjoint(t, w, ng, (0,) * 6, 1e-3, dx, G53).clone() for _ in range(3)]
    assert all(torch.equal(outs[0], o) for o in outs[1:])


# --------------------------------------------------------------- rollout ----

def _loss_grad(hydro, U0, ng, dt, dx, target, n_steps, k):
    x = dev(U0).requires_grad_(True)
    out = hydro.Rollout.apply(x, ng, (0,) * 6, n_steps, dt, dx, G53, k)
    loss = ((out[:, 0] - target) ** 2).sum()
    loss.backward()
    return float(loss), x.grad.detach()


def test_rollout_gradient_matches_oracle_and_is_checkpoint_invariant(hydro):
    say("rollout gradient")
    U0, ng, dx = smooth_all_fields(32)
    rng = np.random.default_rng(6)
    target = dev(U0[:, 0] + 0.01 * rng.normal(size=U0[:, 0].shape))
    dt = 0.2 * dx
    grads = {}
    for k in (1, 2, 4, 8):
        _, grads[k] = _loss_grad(hydro, U0, ng, dt, dx, target, 8, k)
    for k in (2, 4, 8):
        assert torch.equal(grads[k], grads[1]), k
    # dL/d(eps) along v from the oracle's exact JVP of the same rollout
    v = rng.normal(size=U0.shape)
    UN, Jv, _ = oracle.rollout_jvp(U0, v, ng, 3, (0,) * 6, 8, dt, dx, G53)
    dLdv = float(np.sum(2 * (UN[:, 0] - host(target)) * Jv[:, 0]))
    got = float(np.sum(host(grads[1]) * v))
    assert rel(dLdv, got) <= 1e-10, (dLdv, got)


def test_rollout_gradient_central_differences(hydro):
    """Gradient entries against central differences of the GPU forward.  A
    sample whose central differences at eps and eps/2 disagree (a limiter or
    wave-speed switch lies within +-eps, where a one-sided slope changes) is
    rejected; accepted samples agree to 1e-6."""
    say("rollout fd")
    U0, ng, dx = smooth_all_fields(32)
    rng = np.random.default_rng(7)
    target = dev(U0[:, 0] + 0.01 * rng.normal(size=U0[:, 0].shape))
    dt = 0.2 * dx
    _, grad = _loss_grad(hydro, U0, ng, dt, dx, target, 4, 2)
    grad = host(grad)

    def resid(U):
        out = hydro.Rollout.apply(dev(U), ng, (0,) * 6, 4, dt, dx, G53, 2)
        return out[:, 0] - target

    def central(idx, eps):
        up, um = U0.copy(), U0.copy()
        up[idx] += eps
        um[idx] -= eps
        rp, rm = resid(up), resid(um)
        # L+ - L- = sum (r+ - r-)(r+ + r-): avoids cancelling two large sums
        return float(((rp - rm) * (rp + rm)).sum()) / (2 * eps)

    accepted, errs = 0, []
    for _ in range(32):
        idx = tuple(int(rng.integers(0, s)) for s in U0.shape)
        eps = 1e-6 * max(1.0, abs(U0[idx]))
        f1, f2 = central(idx, eps), central(idx, eps / 2)
        if abs(f1 - f2) > 1e-7 * max(abs(f1), abs(f2), 1e-8):
            continue
        accepted += 1
        errs.append(abs(f2 - grad[idx]) / max(abs(f2), 1e-8))
    assert accepted >= 24, accepted
    assert max(errs) <= 1e-6, max(errs)


def test_rollout_leaves_its_input_unchanged(hydro):
    """The rollout steps through private buffers: the caller's initial state is
    bitwise unchanged after forward and backward, for any checkpoint interval."""
    say("rollout input untouched")
    U0, ng, dx = smooth_all_fields(32)
    for k in (1, 3):
        x = dev(U0).requires_grad_(True)
        keep = x.detach().clone()
        out = hydro.Rollout.apply(x, ng, (0,) * 6, 4, 0.2 * dx, dx, G53, k)
        out.sum().backward()
        assert torch.equal(x.detach(), keep), k


def _box_around(grid, c, R):
    x, y, z = c
    nz, ny, nx = grid.shape[1:]
    iz = np.arange(z - R, z + R + 1) % nz
    iy = np.arange(y - R, y + R + 1) % ny
    ix = np.arange(x - R, x + R + 1) % nx
    return grid[:, iz][:, :, iy][:, :, :, ix]


def _fd_branch_protocol(hydro, lv, target, n_steps, draws, eps=1e-7, seed=20171223):
    """Central differences of L = sum (rho_N - rho_target)^2 at sampled
    (cell, field) entries against the adjoint gradient, eps = 1e-7.  A draw is
    rejected when the oracle's +eps and -eps rollouts of the perturbation's
    cone (a periodic box of radius 4 n around the cell, which determines every
    value the perturbation can reach) take different branches anywhere.
    Returns (rejected, errors of the accepted draws): |fd - g| / (|g| + ref_f),
    ref_f the largest |g| of the draw's field among the accepted draws (the
    three momentum components on one scale), the per-entry norm of the
    parity checks.  Central differences at eps = 1e-7 carry an absolute
    round-off of ~1e-9 in this loss (the oracle's own exact JVP and its own
    central differences differ by that much on entries with no branch
    switch), so an entry's plain relative error exceeds 1e-6 whenever its
    gradient is below ~2e-3; the field scale keeps the bound meaningful there."""
    from concurrent.futures import ThreadPoolExecutor
    U0 = lv.U
    dt = 0.2 * lv.dx
    tgt = dev(target)
    x = dev(U0).requires_grad_(True)
    out = hydro.Rollout.apply(x, lv.ng, lv.bc, n_steps, dt, lv.dx, lv.gamma, 4)
    ((out[:, 0] - tgt) ** 2).sum().backward()
    grad = host(x.grad)
    grid = W.groups_to_grid(U0, lv.ng)
    R = 4 * n_steps
    rng = np.random.default_rng(seed)
    picks = [(int(rng.integers(0, 5)), tuple(int(v) for v in rng.integers(0, grid.shape[1], 3)))
             for _ in range(draws)]

    def signatures(pick):
        f, c = pick
        box = _box_around(grid, c, R)
        sig = []
        for s in (1.0, -1.0):
            b = box.copy()
            b[f, R, R, R] += s * eps
            sig.append(oracle.rollout_box(b, n_steps, dt, lv.dx, lv.gamma, signature=True)[3])
        return sig[0] != sig[1]

    with ThreadPoolExecutor(8) as ex:
        differ = list(ex.map(signatures, picks))

    def resid(U):
        o = hydro.Rollout.apply(dev(U), lv.ng, lv.bc, n_steps, dt, lv.dx, lv.gamma, n_steps)
        return o[:, 0] - tgt

    acc, rejected = [], 0
    for (f, c), d in zip(picks, differ):
        if d:
            rejected += 1
            continue
        gx, gy, gz = c[0] // 16, c[1] // 16, c[2] // 16
        g = (gz * lv.ng[1] + gy) * lv.ng[0] + gx
        idx = (g, f, c[2] % 16, c[1] % 16, c[0] % 16)
        up, um = U0.copy(), U0.copy()
        up[idx] += eps
        um[idx] -= eps
        rp, rm = resid(up), resid(um)
        fd = float(((rp - rm) * (rp + rm)).sum()) / (2 * eps)
        acc.append((f, fd, float(grad[idx])))
    key = [0, 1, 1, 1, 4]
    ref = {}
    for f, _, gv in acc:
        ref[key[f]] = max(ref.get(key[f], 0.0), abs(gv))
    errs = [abs(fd - gv) / (abs(gv) + ref[key[f]]) for f, fd, gv in acc]
    return rejected, errs


def test_rollout_fd_branch_protocol_workload_as_stated(hydro):
    """The differentiation workload's recipe (uniform v and p) on a 64^3 grid,
    8 steps: draws whose +-eps runs branch differently are rejected (on this
    state nearly all: its velocity and pressure slopes are round-off on the
    limiter's kink), and every accepted draw agrees to 1e-6."""
    say("rollout fd branch protocol, as stated")
    lv, target = W.smooth_wave(64)
    rejected, errs = _fd_branch_protocol(hydro, lv, target, 8, 24)
    say("  rejected %d of 24, accepted errors %s" % (rejected, ["%.1e" % e for e in errs]))
    assert rejected >= 1
    assert all(e <= 1e-6 for e in errs), errs


def test_rollout_fd_branch_protocol_smooth_v_and_p(hydro):
    say("rollout fd branch protocol, smooth v and p")
    lv, target = W.smooth_wave(64, smooth_vp=0.01)
    rejected, errs = _fd_branch_protocol(hydro, lv, target, 8, 24)
    say("  rejected %d of 24, max error %.2e" % (rejected, max(errs) if errs else float("nan")))
    assert len(errs) >= 16
    assert max(errs) <= 1e-6, errs


def test_fp32_level_adjoint_turbulence_384_sampled(hydro):
    """The FP32 level adjoint at the turbulence workload's full size (384^3,
    13,824 groups): sampled entries of J^T w against <J e, w> from the
    oracle's dual-number JVP of a unit tangent e on the FP32-rounded state
    (one step, on the radius-4 box that determines the radius-2 cone of e).
    Tolerance 1e-4 of the field's scale (the largest |entry| of that field
    among the samples; momentum on one scale): each entry sums ~600 terms whose
    FP32 rounding (6e-8 each) compounds through the predictor, HLLC and update
    chains.  An entry whose evaluation passes within FP32 rounding of a branch
    switch (which the FP64 oracle may resolve the other way) would differ at
    O(1); none may occur among the samples for the test to pass."""
    say("fullsize fp32 adjoint 384^3")
    lv = W.turbulence(384).astype(np.float32)
    U = dev(lv.U)
    dt = float(hydro.cfl_dt(U, lv.dx, lv.gamma, 0.5).min())
    rng = np.random.default_rng(8)
    w = rng.normal(size=lv.U.shape).astype(np.float32)
    JTw = host(hydro.advance_level_adjoint(U, dev(w), lv.ng, lv.bc, dt, lv.dx, lv.gamma))
    del U
    torch.cuda.empty_cache()
    grid = W.groups_to_grid(lv.U.astype(np.float64), lv.ng)
    wgrid = W.groups_to_grid(w.astype(np.float64), lv.ng)
    gT = W.groups_to_grid(JTw.astype(np.float64), lv.ng)
    N = grid.shape[1]
    picks = [(int(rng.integers(0, 5)), tuple(int(v) for v in rng.integers(0, N, 3))) for _ in range(60)]
    got, ref = [], []
    for f, c in picks:
        box = _box_around(grid, c, 4)
        t = np.zeros_like(box)
        t[f, 4, 4, 4] = 1.0
        _, tout, _, _ = oracle.rollout_box(box, 1, dt, lv.dx, lv.gamma, tangent=t)
        ref.append(float(np.sum(tout * _box_around(wgrid, c, 2))))
        got.append(float(gT[(f, c[2], c[1], c[0])]))
    got, ref = np.array(got), np.array(ref)
    fields = np.array([f for f, _ in picks])
    scale = np.array([np.abs(ref[fields == f]).max() if np.any(fields == f) else 1.0 for f in range(5)])
    scale[1:4] = scale[1:4].max()
    err = np.abs(got - ref) / (np.abs(ref) + scale[fields])
    say("  max scaled error %.2e, median %.2e" % (err.max(), np.median(err)))
    assert err.max() <= 1e-4, err.max()


def test_branch_record_equals_advance_and_repeats(hydro):
    """The recording step writes hydro_advance's state bit for bit, and its
    records repeat exactly; a perturbation that flips a limiter case (v_x,
    uniform in this workload, raised by 1e-7 and 2e-7 in two neighbouring
    cells: the first cell's one-sided differences become equal and
    positive, so its v_x slope turns from zero to active) changes the record
    of the perturbed group and of no other (no other group reads those
    cells)."""
    say("branch record")
    lv, _ = W.smooth_wave(64)
    pad = hydro.fill_ghosts(dev(lv.U), lv.ng, 3, lv.bc)
    dt = 0.2 * lv.dx
    ref = hydro.advance(pad, dt, lv.dx, lv.gamma)
    out, r1 = hydro.branch_record(pad, dt, lv.dx, lv.gamma)
    _, r2 = hydro.branch_record(pad, dt, lv.dx, lv.gamma)
    assert torch.equal(out, ref) and torch.equal(r1, r2)
    U = lv.U.copy()
    U[5, 1, 8, 8, 8] += 1e-7 * U[5, 0, 8, 8, 8]
    U[5, 1, 8, 8, 9] += 2e-7 * U[5, 0, 8, 8, 9]
    pad2 = hydro.fill_ghosts(dev(U), lv.ng, 3, lv.bc)
    _, r3 = hydro.branch_record(pad2, dt, lv.dx, lv.gamma)
    diff = (r3 != r1).nonzero().flatten().tolist()
    assert diff == [5], diff


def _fd_gpu_record_protocol(hydro, lv, target, n_steps, draws, eps=1e-7, seed=20171223):
    """_fd_branch_protocol with the rejection taken from the library's branch
    records of the +eps and -eps rollouts (every group, every step)."""
    U0 = lv.U
    dt = 0.2 * lv.dx
    tgt = dev(target)
    x = dev(U0).requires_grad_(True)
    out = hydro.Rollout.apply(x, lv.ng, lv.bc, n_steps, dt, lv.dx, lv.gamma, 4)
    ((out[:, 0] - tgt) ** 2).sum().backward()
    grad = host(x.grad)
    rng = np.random.default_rng(seed)

    def run(U):
        s = dev(U)
        recs = []
        for _ in range(n_steps):
            s, r = hydro.branch_record(hydro.fill_ghosts(s, lv.ng, 3, lv.bc), dt, lv.dx, lv.gamma)
            recs.append(r)
        return s[:, 0] - tgt, torch.stack(recs)

    acc, rejected = [], 0
    for _ in range(draws):
        idx = tuple(int(rng.integers(0, s)) for s in U0.shape)
        up, um = U0.copy(), U0.copy()
        up[idx] += eps
        um[idx] -= eps
        (rp, sp), (rm, sm) = run(up), run(um)
        if not torch.equal(sp, sm):
            rejected += 1
            continue
        fd = float(((rp - rm) * (rp + rm)).sum()) / (2 * eps)
        acc.append((idx[1], fd, float(grad[idx])))
    key = [0, 1, 1, 1, 4]
    ref = {}
    for f, _, gv in acc:
        ref[key[f]] = max(ref.get(key[f], 0.0), abs(gv))
    return rejected, [abs(fd - gv) / (abs(gv) + ref[key[f]]) for f, fd, gv in acc]


@pytest.mark.parametrize("smooth_vp", [0.0, 0.01])
def test_rollout_fd_with_library_branch_records(hydro, smooth_vp):
    """The FD protocol the bench runs: rejection from the GPU's own branch
    records; every accepted draw agrees to 1e-6 (as stated: nearly all draws
    straddle a switch; smooth v and p: nearly none)."""
    say("rollout fd, library branch records, smooth_vp", smooth_vp)
    lv, target = W.smooth_wave(64, smooth_vp=smooth_vp) if smooth_vp else W.smooth_wave(64)
    rejected, errs = _fd_gpu_record_protocol(hydro, lv, target, 8, 24)
    say("  rejected %d of 24, accepted errors %s" % (rejected, ["%.1e" % e for e in errs]))
    assert all(e <= 1e-6 for e in errs), errs
    if smooth_vp:
        assert len(errs) >= 16
    else:
        assert rejected >= 1
