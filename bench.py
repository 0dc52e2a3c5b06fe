"""Benchmark of the patch-group MHM hot path on one MI355X.

A step is one pass of the whole per-level path over every patch group of the
level: ghost fill, MHM update and the per-patch CFL time-step (Eq. 2) that the
next step uses.  By default this is one fused launch per step
(hydro_advance_level: neighbour groups are read directly instead of a padded
copy, and the CFL reduction of the written state runs in the epilogue); the
first timed step also computes the CFL time-step of the initial state
(hydro_dt).  --unfused times hydro_fill_ghosts + hydro_dt + hydro_advance per
step instead.  The default workload is the
256^3 periodic shear layer (4096 groups of 16^3 cells, 3 ghost zones,
gamma = 1.4) advanced at CFL 0.5 in double precision; inputs are resident in
HBM before the timed region starts.

Prints one JSON line.  `value` is cell updates per second of the timed steps
(whole job); `roofline` describes the dominant kernel (the MHM update), whose
average duration is measured with HIP events on the stream it runs on;
`cpu_baseline` is the CPU oracle timed on a bounded sample of the same
workload on the host cores.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VEC_PEAK_TFLOPS = 78.6    # MI355X vector FP64
FP32_VEC_PEAK_TFLOPS = 157.3   # MI355X vector FP32
# Algorithmic HBM bytes per cell update of the MHM kernel: the stencil-reachable
# input (7360 cells of a padded group: interior, 2-deep face slabs, 1-deep
# edges) plus the 4096 interior outputs, 5 fields each, per 4096 cells updated.
REACH_CELLS = 7360
ALG_BYTES_PADDED = {"f64": (REACH_CELLS + 4096) * 5 * 8 / 4096, "f32": (REACH_CELLS + 4096) * 5 * 4 / 4096}
# The fused level step reads every level cell once and writes it once.
ALG_BYTES_LEVEL = {"f64": 2 * 5 * 8, "f32": 2 * 5 * 4}


def _alg_flops_per_cell() -> float:
    """Algorithmic floating-point operations per cell update (add, mul, div,
    sqrt each one): the oracle's operation count of the four per-item stages
    (every limiter active, HLLC star branch) times their multiplicities per
    group (7360 primitive conversions, 5632 Hancock cells, 13056 HLLC faces,
    4096 updates), as written to oracle/flops_per_cell.json by
    oracle/count_flops.py (read here as data)."""
    with open(os.path.join(ROOT, "oracle", "flops_per_cell.json")) as fh:
        return float(json.load(fh)["flops_per_cell_update"])


ALG_FLOPS_PER_CELL = _alg_flops_per_cell()


def kernel_source_sha() -> str:
    """sha256 of the code of the MHM kernels' sources: comments and blank
    lines are dropped, so it changes whenever the code does and not when
    only a comment does."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("hydro_device.h", "ext_device.h", "mhm_group.h", "mhm_level.h", "mhm_fwd.hip"):
        with open(os.path.join(ROOT, "paper_1712_07070_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()


def measured_profile(kernel_key: str, variant, field: str):
    """A per-launch figure (HBM bytes, VALU wave-instructions) from the
    committed counter profile of this launch shape, or None when the kernel
    sources differ from what was measured or the shape was not measured."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            rec = json.load(fh).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != kernel_source_sha():
        return None
    shape = rec.get("by_variant", {}).get(str(variant))
    return shape.get(field) if shape else None


def measured_traffic(kernel_key: str, variant):
    return measured_profile(kernel_key, variant, "bytes_per_launch")


# VALU issue capacity: one wave-instruction (64 lanes) occupies a SIMD for 4
# cycles (16 lanes per cycle, FP64 and unpacked FP32 alike); 256 CUs x 4
# SIMDs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=40,
                    help="untimed steps first: the first few dozen steps after the tuner run up to 10%% slower")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--n", type=int, default=256, help="grid cells per axis (multiple of 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the extra FP32 measurement")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--unfused", action="store_true", help="time fill + dt + padded advance per step")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--variant", type=int, default=None,
                    help="launch shape of the level step (implies --no-autotune), e.g. for counter runs")
    ap.add_argument("--no-amr", action="store_true", help="skip the batched multi-level measurement")
    ap.add_argument("--amr-coarse-steps", type=int, default=4)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the fwd+adjoint rollout measurements")
    ap.add_argument("--fd-samples", type=int, default=64)
    ap.add_argument("--no-ext", action="store_true",
                    help="skip the other schemes, the unphysical-result procedure and the coupled AMR hierarchy")
    ap.add_argument("--counter-sweep", type=int, default=0, metavar="REPS",
                    help="only launch every shape of the fused level step (with the CFL epilogue), FP64 then FP32, "
                         "REPS launches each in a fixed order, for hardware-counter runs")
    ap.add_argument("--adjoint-counter-run", type=int, default=0, metavar="REPS",
                    help="only launch the forward level step and the step adjoint (fused form) REPS times each on "
                         "the 128^3 FP64 smooth wave and the 384^3 FP32 turbulence state, for hardware-counter runs")
    ap.add_argument("--batched-counter-run", type=int, default=0, metavar="REPS",
                    help="only launch the level step (launch shapes 6 and 2) and the batched kernel on the same "
                         "single level (variants 0, 2, 12, 14) REPS times each on the n^3 FP64 shear layer, for "
                         "hardware-counter runs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="after the run, copy a device buffer of this size (reference for HBM byte counters)")
    return ap.parse_args()


def run_workload(hydro, torch, lv, dtype, steps, warmup, fused=True, autotune=True):
    """Time `steps` full steps; return (seconds, mean MHM kernel ms, solver, last dt, n_bad, tune info)."""
    tdt = torch.float64 if dtype == "f64" else torch.float32
    solver = hydro.LevelSolver(lv.ng, lv.dx, lv.gamma, lv.bc, ghost=3, dtype=tdt, fused=fused)
    U0 = torch.from_numpy(np.ascontiguousarray(lv.U.astype(np.float64 if dtype == "f64" else np.float32))).cuda()
    tune = None
    if fused and autotune:
        # choose the launch shape (all shapes give bit-identical results) before timing
        best, times = hydro.autotune(U0, lv.ng, lv.bc, lv.dx, lv.gamma, reps=5)
        n = hydro.num_variants()
        tune = {"variant": best, "name": hydro.variant_name(best),
                "ms": [round(t, 4) for t in times[n:]], "ms_without_cfl": [round(t, 4) for t in times[:n]],
                "variant_without_cfl": hydro.get_level_variant(tdt, False)}
    solver.load_state(U0)
    for _ in range(warmup):
        solver.step()
    solver.load_state(U0)
    solver.n_bad.zero_()
    # the MHM update is bracketed by HIP events on the stream it is launched on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        solver.step(events=ev[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    dts = solver.dt_min.cpu().numpy()
    return elapsed, kms, solver, dts, int(solver.n_bad.cpu()[0]), tune


def amr_small_levels(hydro, torch, W, coarse_steps):
    """Three levels that leave partial rounds of workgroups (125 / 343 / 1000
    groups: 5^3, 7^3, 10^3 bricks, dx and dt halving per level, Sedov-like
    blast), FP64: the batched and per-level W-cycles, both graph-captured."""
    lvs = W.sedov_levels(((5, 5, 5), (7, 7, 7), (10, 10, 10)), dx0=1.0 / 80)
    r = amr_workload(hydro, torch, W, coarse_steps, lvs=lvs, forms=("batched_graph", "per_level_graph"),
                     adaptive=False)
    r["workload"] = ("3 levels of 125/343/1000 groups (5x5x5, 7x7x7, 10x10x10), dx_l = dx_0/2^l, dt_l = dt_0/2^l, "
                     "1/2/4 substeps per coarse step, Sedov-like blast, FP64")
    return r


def amr_workload(hydro, torch, W, coarse_steps, lvs=None, forms=None, adaptive=True):
    """Three uneven levels (512 / 1536 / 3072 groups, dx and dt halving per
    level, Sedov-like blast), FP64: W-cycle coarse steps as one persistent
    launch per stage vs one launch per level per stage, both graph-captured."""
    lvs = lvs if lvs is not None else W.sedov_levels()
    geo = [(lv.ng, lv.dx, lv.bc) for lv in lvs]
    states = [torch.from_numpy(lv.U).cuda() for lv in lvs]
    dt0 = float("inf")
    for l, (lv, U) in enumerate(zip(lvs, states)):
        dt0 = min(dt0, float(hydro.cfl_dt(U, lv.dx, lv.gamma, 0.5).min()) * 2 ** l)
    res = {"workload": "3 levels of 512/1536/3072 groups (8x8x8, 8x8x24, 8x16x24), dx_l = dx_0/2^l, "
                       "dt_l = dt_0/2^l, 1/2/4 substeps per coarse step, Sedov-like blast, FP64",
           "dt0": dt0}
    out = {}
    n = max(2, coarse_steps - coarse_steps % 2)
    runs = {}
    for name, batched, graph in (("batched_graph", True, True), ("per_level_graph", False, True),
                                 ("per_level_eager", False, False), ("batched_eager", True, False)):
        if forms is not None and name not in forms:
            continue
        ml = hydro.MultiLevel(geo, lvs[0].gamma, dt0, batched=batched)
        for l, U in enumerate(states):
            ml.load_state(l, U)
        if batched and "batched_tune" not in res:
            # launch shape chosen on whole coarse steps (every stage, weighted)
            best, times = ml.autotune(reps=3)
            res["batched_tune"] = {"variant": best, "ms_per_coarse_step": [round(t, 4) for t in times]}
        g = ml.capture(2) if graph else None
        run = (lambda g=g: g.replay()) if graph else (lambda ml=ml: (ml.coarse_step(), ml.coarse_step()))
        run()                                   # warm-up (2 coarse steps)
        runs[name] = (ml, g, run)
        res["cells_per_coarse_step"] = ml.cells_per_coarse_step()
    # the four forms are timed in turn, three rounds; each keeps its best round
    best_el = {}
    for _ in range(3):
        for name, (ml, g, run) in runs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n // 2):
                run()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best_el[name] = min(el, best_el.get(name, el))
    for name, (ml, g, run) in runs.items():
        el = best_el[name]
        out[name] = {"cell_updates_per_s": ml.cells_per_coarse_step() * n / el, "ms_per_coarse_step": el / n * 1e3,
                     "n_bad": int(ml.n_bad.cpu()[0])}
        if g is not None:
            g.close()
    runs.clear()
    res.update(out)
    res["batched_over_per_level"] = out["batched_graph"]["cell_updates_per_s"] / out["per_level_graph"][
        "cell_updates_per_s"]
    if not adaptive:
        return res
    # the adaptive W-cycle: the batched launches also reduce the next coarse
    # step's dt_0 = min_l 2^l dt_l (Eq. 2, C = 0.5) on the device; a graph of
    # six coarse steps (the period of the buffer and time-step-word rotation)
    ml = hydro.MultiLevel(geo, lvs[0].gamma, dt0, batched=True, adaptive=True, c_cfl=0.5)
    for l, U in enumerate(states):
        ml.load_state(l, U)
    ml.autotune(reps=3)
    g = ml.capture(6)
    g.replay()
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    res["batched_adaptive_graph"] = {"cell_updates_per_s": ml.cells_per_coarse_step() * 6 / best,
                                     "ms_per_coarse_step": best / 6 * 1e3, "n_bad": int(ml.n_bad.cpu()[0]),
                                     "dt0_next": float(ml.dt_coarse().cpu()[0])}
    g.close()
    return res


def adjoint_rollout(hydro, torch, lv, dtype, n_steps, k_ckpt, dt, target=None, reps=3):
    """Time a differentiable rollout (forward with checkpoints, backward with
    segment replay and the step adjoint); returns timings and the gradient."""
    U0 = torch.from_numpy(np.ascontiguousarray(lv.U.astype(dtype))).cuda()
    tgt = None if target is None else torch.from_numpy(np.ascontiguousarray(target.astype(dtype))).cuda()
    res = []
    for _ in range(reps + 1):
        x = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = hydro.Rollout.apply(x, lv.ng, lv.bc, n_steps, dt, lv.dx, lv.gamma, k_ckpt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if tgt is None:
            gout = torch.ones_like(out)
            out.backward(gout)
        else:
            loss = ((out[:, 0] - tgt) ** 2).sum()
            loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res.append((t1 - t0, t2 - t1))
    fwd = float(np.median([r[0] for r in res[1:] or res]))
    bwd = float(np.median([r[1] for r in res[1:] or res]))
    cell_steps = lv.n_cells * n_steps
    return {"t_fwd_ms": fwd * 1e3, "t_bwd_ms": bwd * 1e3, "bwd_over_fwd": bwd / fwd,
            "cell_steps_per_s_fwd_bwd": cell_steps / (fwd + bwd), "cell_steps_per_s_fwd": cell_steps / fwd}, x.grad


def fd_protocol(hydro, torch, lv, target, n_steps, dt, grad, samples, seed=20171223, eps=1e-7, max_draws=None):
    """Central differences of the loss at seeded (cell, field) entries, each
    perturbed by +-eps (eps = 1e-7), against the adjoint gradient.  A draw is
    rejected when the +eps and -eps rollouts take different branches anywhere
    (limiter case or argument, wave-speed argument, HLLC region): each
    rollout runs with the library's branch record (hydro_branch_record, the
    step's own decisions per group and step, bitwise the same states), and a
    draw whose two record sequences differ straddles a switch, where central
    differences do not measure the derivative the adjoint follows.  Up to
    max_draws (default 4 x samples) draws are taken until `samples` are
    accepted; the rejection count is reported.  The loss differences are
    formed as sum (r1 - r2)(r1 + r2) to avoid cancelling two large sums."""
    U0 = lv.U
    tgt = torch.from_numpy(np.ascontiguousarray(target)).cuda()
    rng = np.random.default_rng(seed)
    max_draws = max_draws or 4 * samples

    def run(U):
        x = torch.from_numpy(U).cuda()
        recs = []
        for _ in range(n_steps):
            pad = hydro.fill_ghosts(x, lv.ng, 3, lv.bc)
            x, rec = hydro.branch_record(pad, dt, lv.dx, lv.gamma)
            recs.append(rec)
        return x[:, 0] - tgt, torch.stack(recs)

    def dloss(ra, rb):
        return float(((ra - rb) * (ra + rb)).sum())

    g = grad.cpu().numpy()
    acc, rejected, draws = [], 0, 0
    while len(acc) < samples and draws < max_draws:
        draws += 1
        idx = tuple(int(rng.integers(0, s)) for s in U0.shape)
        up, um = U0.copy(), U0.copy()
        up[idx] += eps
        um[idx] -= eps
        (rp, sp), (rm, sm) = run(up), run(um)
        if not torch.equal(sp, sm):
            rejected += 1
            continue
        fd = dloss(rp, rm) / (2 * eps)
        acc.append((idx[1], fd, float(g[idx])))
    # error norm of the parity checks: |fd - g| / (|g| + ref_f), ref_f the
    # largest |g| of the entry's field among the accepted entries (momentum
    # components on one scale); central differences at eps = 1e-7 carry an
    # absolute round-off of ~1e-9 in this loss, which a plain relative error
    # of a small gradient entry would magnify
    key = [0, 1, 1, 1, 4]
    ref = {}
    for f, _, gv in acc:
        ref[key[f]] = max(ref.get(key[f], 0.0), abs(gv))
    e = np.array([abs(fd - gv) / (abs(gv) + ref[key[f]]) for f, fd, gv in acc]) if acc else np.array([np.nan])
    r = np.array([abs(fd - gv) / max(abs(fd), abs(gv), 1e-300) for f, fd, gv in acc]) if acc else np.array([np.nan])
    return {"draws": draws, "rejected": rejected, "accepted": len(acc), "eps": eps,
            "rule": "reject when the +eps and -eps rollouts' branch records (every group, every step) differ",
            "norm": "|fd - g| / (|g| + max |g| of the field among accepted entries)",
            "max_err": float(np.nanmax(e)), "median_err": float(np.nanmedian(e)),
            "within_1e-6": int(np.sum(e <= 1e-6)),
            "all_accepted_within_1e-6": bool(np.all(e <= 1e-6)) if acc else None,
            "max_plain_rel_err": float(np.nanmax(r)), "median_plain_rel_err": float(np.nanmedian(r))}


def step_ratio(hydro, torch, lv, dtype, dt, reps=10):
    """One forward level step and one step adjoint on the same state, timed
    with events on the stream they run on (median of reps)."""
    U = torch.from_numpy(np.ascontiguousarray(lv.U.astype(dtype))).cuda()
    O = torch.empty_like(U)
    g = torch.ones_like(U)
    gi = torch.empty_like(U)
    work = hydro.adjoint_workspace(lv.n_groups, U.dtype, True)
    fwd = time_events(torch, lambda: hydro.advance_level(U, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=O), reps)
    adj = time_events(torch, lambda: hydro.advance_level_adjoint(U, g, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=gi,
                                                                 work=work), reps)
    del U, O, g, gi, work
    torch.cuda.empty_cache()
    return {"fwd_step_ms": fwd, "adjoint_step_ms": adj, "adjoint_over_fwd": adj / fwd}


def tune_adjoint(hydro, torch, lv, dtype):
    """Choose the adjoint form (fused / two kernels) on this workload's state."""
    U = torch.from_numpy(np.ascontiguousarray(lv.U.astype(dtype))).cuda()
    g = torch.ones_like(U)
    form, times = hydro.autotune_adjoint(U, g, lv.ng, lv.bc, lv.dx, lv.gamma, reps=3)
    del U, g
    torch.cuda.empty_cache()
    return {"form": form, "ms": [round(t, 4) for t in times]}


def time_events(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def differentiation_workloads(hydro, torch, W, fd_samples):
    out = {}
    # 128^3 smooth wave, 512 groups, FP64, 8 steps at dt = 0.2 dx; every state
    # checkpointed (k = 1, no replay: 8 x 84 MB), and k = 4 with segment replay
    lv, target = W.smooth_wave(128)
    dt = 0.2 * lv.dx
    form = tune_adjoint(hydro, torch, lv, np.float64)
    r, grad = adjoint_rollout(hydro, torch, lv, np.float64, 8, 1, dt, target)
    r["adjoint_form"] = form
    r4, _ = adjoint_rollout(hydro, torch, lv, np.float64, 8, 4, dt, target)
    r["workload"] = "smooth wave 128^3 (512 groups), FP64, 8 steps at dt = 0.2 dx, every state checkpointed, " \
                    "loss sum (rho_8 - rho_target)^2"
    r["checkpoint_every_4"] = r4
    r["step"] = step_ratio(hydro, torch, lv, np.float64, dt)
    r["fd"] = fd_protocol(hydro, torch, lv, target, 8, dt, grad, fd_samples)
    out["smooth128_f64"] = r
    del grad
    torch.cuda.empty_cache()
    # the same protocol with v and p varying smoothly along every axis (1e-2),
    # so that no velocity / pressure slope of the initial state is a round-off
    # difference sitting on the limiter's kink
    lvs, target_s = W.smooth_wave(128, smooth_vp=0.01)
    _, grad = adjoint_rollout(hydro, torch, lvs, np.float64, 8, 4, dt, target_s, reps=0)
    out["smooth128_f64"]["fd_smooth_vp"] = fd_protocol(hydro, torch, lvs, target_s, 8, dt, grad, fd_samples)
    del grad
    torch.cuda.empty_cache()
    # 384^3 turbulence-like state, 13824 groups, FP32, 4 steps at the initial CFL time-step (FP64 reduction)
    lv = W.turbulence(384).astype(np.float32)
    U = torch.from_numpy(lv.U).cuda()
    dt = float(hydro.cfl_dt(U, lv.dx, lv.gamma, 0.5).min())
    del U
    form = tune_adjoint(hydro, torch, lv, np.float32)
    r, grad = adjoint_rollout(hydro, torch, lv, np.float32, 4, 1, dt, None, reps=2)
    r["adjoint_form"] = form
    r["workload"] = "turbulence 384^3 (13824 groups), FP32 state, 4 steps at the initial CFL time-step " \
                    "(FP64 reduction), every state checkpointed, cotangent of ones"
    r["dt"] = dt
    del grad
    torch.cuda.empty_cache()
    r["step"] = step_ratio(hydro, torch, lv, np.float32, dt)
    out["turb384_f32"] = r
    return out


# Scheme words of the other schemes measured on the shear layer (the AMR runs
# of the paper's comparisons use MHM + PPM + HLLC with the hybrid limiter, and
# CTU with Roe's solver)
EXT_SCHEMES = {
    "mhm-ppm-hllc-hybrid": 1 | (1 << 14) | (3 << 11),
    "ctu-plm-roe": 2 | (1 << 16),
    "mhm-plm-char-vanleer-hllc": 1 | (1 << 13) | (1 << 11),
    "mhm-plm-hlle": 1 | (2 << 16),
}


def ext_schemes(hydro, torch, W, reps=5):
    """One step (ghost fill + the multi-kernel step) of the 256^3 shear layer
    per scheme word, timed with events on the stream the kernels run on."""
    lv = W.shear_layer(256)
    out = {"workload": "shear-layer 256^3 (4096 groups), 3 ghost zones, one step at the initial CFL time-step"}
    for dtype in ("f64", "f32"):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        U = torch.from_numpy(np.ascontiguousarray(lv.U.astype(np.float64 if dtype == "f64" else np.float32))).cuda()
        pad = hydro.fill_ghosts(U, lv.ng, 3, lv.bc)
        dt = float(hydro.cfl_dt(pad, lv.dx, lv.gamma, 0.5).min())
        for name, sch in EXT_SCHEMES.items():
            if dtype == "f32" and name != "mhm-ppm-hllc-hybrid":
                continue
            work = hydro.ext_workspace(lv.n_groups, 3, tdt, sch)
            O = torch.empty_like(U)

            def step():
                hydro.fill_ghosts(U, lv.ng, 3, lv.bc, out=pad)
                hydro.advance_ext(pad, dt, lv.dx, lv.gamma, sch, out=O, work=work)
            ms = time_events(torch, step, reps)
            out["%s/%s" % (name, dtype)] = {"ms_per_step": ms, "cell_updates_per_s": lv.n_cells / (ms * 1e-3),
                                           "scheme_word": sch, "workspace_bytes": work.numel()}
            del work, O
            torch.cuda.empty_cache()
        del U, pad
        torch.cuda.empty_cache()
    # dual energy (6 fields, the entropy s = p / rho^(gamma-1) as field 5) with
    # the AGORA scheme word, FP64
    U5 = lv.U
    r = U5[:, 0]
    ekin = 0.5 * (U5[:, 1] ** 2 + U5[:, 2] ** 2 + U5[:, 3] ** 2) / r
    ent = (lv.gamma - 1.0) * (U5[:, 4] - ekin) / r ** (lv.gamma - 1.0)
    Ud = torch.from_numpy(np.ascontiguousarray(U5)).cuda()
    Ed = torch.from_numpy(np.ascontiguousarray(np.repeat(ent[:, None], 5, axis=1))).cuda()
    pad6 = torch.cat([hydro.fill_ghosts(Ud, lv.ng, 3, lv.bc), hydro.fill_ghosts(Ed, lv.ng, 3, lv.bc)[:, :1]], dim=1)
    del Ud, Ed
    torch.cuda.empty_cache()
    sch = EXT_SCHEMES["mhm-ppm-hllc-hybrid"] | (1 << 18)
    dt = float(hydro.cfl_dt(pad6[:, :5].contiguous(), lv.dx, lv.gamma, 0.5).min())
    work = hydro.ext_workspace(lv.n_groups, 3, torch.float64, sch)
    O = torch.empty((lv.n_groups, 6, 16, 16, 16), dtype=torch.float64, device="cuda")
    ms = time_events(torch, lambda: hydro.advance_ext(pad6, dt, lv.dx, lv.gamma, sch, out=O, work=work, xi=0.01), reps)
    out["mhm-ppm-hllc-hybrid-dual-energy/f64"] = {"ms_per_step": ms, "cell_updates_per_s": lv.n_cells / (ms * 1e-3),
                                                 "scheme_word": sch, "fill_in_timed_region": False}
    del pad6, work, O
    torch.cuda.empty_cache()
    return out


def fallback_workload(hydro, torch, W, reps=3):
    """The procedure for unphysical results on a 128^3 low-pressure white-noise
    state at its CFL time-step: MHM's update fails on ~0.15% of the cells,
    which are recomputed first-order; the plain step is timed beside it."""
    n = 128
    rng = np.random.default_rng(20171219 + 6)
    rho = rng.uniform(0.05, 2, (n, n, n))
    p = np.exp(rng.uniform(np.log(1e-3), np.log(2.0), (n, n, n)))
    v = rng.normal(0, 0.5, (3, n, n, n))
    Uh = W.grid_to_groups(W.conserved(rho, v[0], v[1], v[2], p, 5.0 / 3.0))
    ng, bc, dx = (n // 16,) * 3, (0,) * 6, 1.0 / n
    U = torch.from_numpy(Uh).cuda()
    pad = hydro.fill_ghosts(U, ng, 3, bc)
    dt = float(hydro.cfl_dt(pad, dx, 5.0 / 3.0, 0.5).min())
    del pad
    O = torch.empty_like(U)
    work = torch.empty(int(hydro.load().hydro_fallback_workspace_bytes(*ng, 0, 1)), dtype=torch.uint8, device="cuda")
    info = {}

    def fb():
        _, ok, inf = hydro.advance_level_fallback(U, ng, bc, dt, dx, 5.0 / 3.0, out=O, work=work)
        info.update(inf, ok=ok)
    ms_fb = time_events(torch, fb, reps)
    ms_plain = time_events(torch, lambda: hydro.advance_level(U, ng, bc, dt, dx, 5.0 / 3.0, out=O), reps)
    return {"workload": "white noise 128^3, rho U(0.05,2), p log-uniform [1e-3, 2], v N(0, 0.5), CFL 0.5, FP64",
            "ms_fallback_step": ms_fb, "ms_plain_step": ms_plain, "repaired": info,
            "cell_updates_per_s": Uh.shape[0] * 4096 / (ms_fb * 1e-3)}


def amr_coupled(hydro, torch, W, coarse_steps=2):
    """The blast workload on a coupled hierarchy (512 / 1536 / 3072 groups,
    nested, W-cycle with ghost interpolation, flux registers, restriction and
    fix-up): coarse steps timed with events, FP64, MHM+PLM+HLLC."""
    h = W.sedov_hierarchy()
    dev = [torch.from_numpy(np.ascontiguousarray(s)).cuda() for s in h.states]
    solver = hydro.AmrSolver(h.n0, h.positions, dev, h.dx0, h.gamma, h.bc)
    dt0 = 1.25e-6
    solver.step(dt0)                                   # warm-up
    torch.cuda.synchronize()
    ms = time_events(torch, lambda: solver.step(dt0), coarse_steps)
    # the same coarse steps as one captured graph per two coarse steps
    g = solver.capture(dt0, 2)
    ms_graph = time_events(torch, g.replay, max(1, coarse_steps // 2)) / 2
    g.close()
    cells = solver.cells_per_coarse_step()
    return {"workload": "coupled blast hierarchy: 8^3 level-0 groups, 16x12x8 level-1 and 24x16x8 level-2 groups "
                        "(nested boxes), dt_l = dt_0 / 2^l, FP64",
            "groups": [len(p) for p in h.positions], "ms_per_coarse_step": ms,
            "cells_per_coarse_step": cells, "cell_updates_per_s": cells / (ms * 1e-3),
            "graph": {"ms_per_coarse_step": ms_graph, "cell_updates_per_s": cells / (ms_graph * 1e-3)},
            "n_bad": int(solver.n_bad.cpu()[0])}


def cpu_baseline(lv_factory, seconds):
    """The oracle (fill + CFL + MHM step) on a bounded sample of the workload."""
    import oracle
    lv = lv_factory()
    # sample: the first two z-layers of groups as their own periodic brick
    ngx, ngy, _ = lv.ng
    nsub = ngx * ngy * 2
    U = np.ascontiguousarray(lv.U[:nsub])
    ng = (ngx, ngy, 2)
    cells = nsub * 4096

    def timed(budget):
        V, steps, t0 = U, 0, time.perf_counter()
        while True:
            V, _, _ = oracle.rollout(V, ng, 3, lv.bc, 1, lv.dx, lv.gamma)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return steps, el

    threads = oracle.num_threads()
    steps, el = timed(seconds)
    # the same sample on one thread (shorter budget, at least one step)
    oracle.set_num_threads(1)
    try:
        steps1, el1 = timed(seconds / 3)
    finally:
        oracle.set_num_threads(threads)
    others = cpu_other_workloads(seconds / 3)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": cells * steps / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps (ghost fill + CFL + MHM) of %d groups (%dx%dx%d cells, a %dx%dx2-group slab of "
                      "the workload as its own periodic brick), FP64, OpenMP over groups" %
                      (steps, nsub, ngx * 16, ngy * 16, 32, ngx, ngy),
            "single_thread": {"value": cells * steps1 / el1, "steps": steps1},
            "other_workloads": others,
            "host": {"cpu_count": os.cpu_count(), "model": model}}


def cpu_other_workloads(budget):
    """The oracle on bounded samples of the other workloads (all host threads):
    the blast levels (one level-2 brick step), the 128^3 smooth wave (its
    8-step rollout) and a 2-group-deep slab of the 384^3 turbulence state, in
    cell-updates/s."""
    import oracle
    from paper_1712_07070_amd import workloads as W
    out = {}

    def rate(run, cells):
        n, t0 = 0, time.perf_counter()
        while True:
            run()
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return cells * n / el, n

    lv = W.sedov_levels()[2]
    r, n = rate(lambda: oracle.rollout(lv.U, lv.ng, 3, lv.bc, 1, lv.dx, lv.gamma, dt=1e-7), lv.n_cells)
    out["blast_level2_3072_groups"] = {"value": r, "steps": n}
    lv, _ = W.smooth_wave(128)
    r, n = rate(lambda: oracle.rollout(lv.U, lv.ng, 3, lv.bc, 8, lv.dx, lv.gamma, dt=0.2 * lv.dx),
                lv.n_cells * 8)
    out["smooth_wave_128_rollout_8_steps"] = {"value": r, "rollouts": n}
    lv = W.turbulence(384)
    ngx, ngy, _ = lv.ng
    nsub = ngx * ngy * 2
    U = np.ascontiguousarray(lv.U[:nsub])
    r, n = rate(lambda: oracle.rollout(U, (ngx, ngy, 2), 3, lv.bc, 1, lv.dx, lv.gamma), nsub * 4096)
    out["turbulence_384_slab_1152_groups"] = {"value": r, "steps": n}
    out["unit"] = "cell-updates/s"
    out["cores"] = oracle.num_threads()
    return out


def counter_sweep(hydro, torch, W, n, reps, calibrate_mib):
    """Launch every shape of the fused level step with the CFL epilogue (the
    bench's timed kernel) on the n^3 shear layer, FP64 then FP32, `reps`
    launches per shape in shape order, then the calibration copy: a counter
    run maps the kernel's dispatches to shapes by this order."""
    lv = W.shear_layer(n)
    order = []
    for dtype in (torch.float64, torch.float32):
        solver = hydro.LevelSolver(lv.ng, lv.dx, lv.gamma, lv.bc, ghost=3, dtype=dtype, fused=True)
        U0 = torch.from_numpy(np.ascontiguousarray(lv.U.astype(np.float64 if dtype == torch.float64 else np.float32)))
        solver.load_state(U0.cuda())
        for v in range(hydro.num_variants()):
            hydro.set_level_variant(dtype, True, v)
            for _ in range(reps):
                solver.step()
            torch.cuda.synchronize()
            order.append({"dtype": "f64" if dtype == torch.float64 else "f32", "variant": v, "launches": reps,
                          "name": hydro.variant_name(v)})
        del solver
        torch.cuda.empty_cache()
    if calibrate_mib > 0:
        m = calibrate_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"counter_sweep": order, "cells_per_launch": lv.n_cells,
                      "copy_calibration_bytes": calibrate_mib * (1 << 20)}), flush=True)


def batched_counter_run(hydro, torch, W, n, reps, calibrate_mib):
    """The same single level (the n^3 FP64 shear layer, no CFL epilogue)
    through the level step (launch shapes 6 and 2: XCD-blocked, low occupancy
    target, column-tile and linear order) and through the persistent batched
    kernel (variants 0 and 2: one queue, 12 and 14: per-XCD column-tile
    queues; high and low occupancy target),
    `reps` launches each in that order after 30 untimed level steps (the
    clock ramp of a fresh process), then the calibration copy: the per-item
    cost of the persistent form, in counters."""
    lv = W.shear_layer(n)
    U = torch.from_numpy(np.ascontiguousarray(lv.U)).cuda()
    O = torch.empty_like(U)
    dt = 0.2 * lv.dx
    work = torch.zeros(hydro.BATCH_WORK_WORDS, dtype=torch.int32, device="cuda")
    order = []
    saved_l, saved_b = hydro.get_level_variant(torch.float64, False), hydro.get_batched_variant(torch.float64)
    try:
        hydro.set_level_variant(torch.float64, False, 2)
        for _ in range(30):
            hydro.advance_level(U, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=O)
        torch.cuda.synchronize()
        order.append({"form": "warm-up", "variant": 2, "launches": 30})
        for v in (6, 2):
            hydro.set_level_variant(torch.float64, False, v)
            for _ in range(reps):
                hydro.advance_level(U, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=O)
            torch.cuda.synchronize()
            order.append({"form": "level", "variant": v, "launches": reps, "name": hydro.variant_name(v)})
        for v in (0, 2, 12, 14):
            hydro.set_batched_variant(torch.float64, v)
            for _ in range(reps):
                hydro.advance_batched([(U, O, lv.ng, lv.bc, dt, lv.dx)], lv.gamma, work)
            torch.cuda.synchronize()
            order.append({"form": "batched", "variant": v, "launches": reps})
    finally:
        hydro.set_level_variant(torch.float64, False, saved_l)
        hydro.set_batched_variant(torch.float64, saved_b)
    if calibrate_mib > 0:
        m = calibrate_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"batched_counter_run": order, "cells_per_launch": lv.n_cells,
                      "copy_calibration_bytes": calibrate_mib * (1 << 20)}), flush=True)


def adjoint_counter_run(hydro, torch, W, reps, calibrate_mib):
    """Forward level step, then step adjoint (fused form), `reps` launches
    each, on the 128^3 FP64 smooth wave and then the 384^3 FP32 turbulence
    state (the differentiation workloads), then the calibration copy."""
    order = []
    for name, lv, dtype in (("smooth128_f64", W.smooth_wave(128)[0], np.float64),
                            ("turb384_f32", W.turbulence(384), np.float32)):
        U = torch.from_numpy(np.ascontiguousarray(lv.U.astype(dtype))).cuda()
        tdt = U.dtype
        dt = float(hydro.cfl_dt(U, lv.dx, lv.gamma, 0.5).min())
        O = torch.empty_like(U)
        g = torch.ones_like(U)
        gi = torch.empty_like(U)
        work = hydro.adjoint_workspace(lv.n_groups, tdt, True)
        hydro.set_adjoint_variant(tdt, 0)
        for _ in range(reps):
            hydro.advance_level(U, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=O)
        for _ in range(reps):
            hydro.advance_level_adjoint(U, g, lv.ng, lv.bc, dt, lv.dx, lv.gamma, out=gi, work=work)
        torch.cuda.synchronize()
        order.append({"workload": name, "groups": lv.n_groups, "launches": reps})
        del U, O, g, gi, work
        torch.cuda.empty_cache()
    if calibrate_mib > 0:
        m = calibrate_mib * (1 << 20) // 8
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps({"adjoint_counter_run": order, "copy_calibration_bytes": calibrate_mib * (1 << 20)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1712_07070_amd import hydro
    from paper_1712_07070_amd import workloads as W
    hydro.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.counter_sweep > 0:
        counter_sweep(hydro, torch, W, args.n, args.counter_sweep, args.calibrate_copy)
        return
    if args.adjoint_counter_run > 0:
        adjoint_counter_run(hydro, torch, W, args.adjoint_counter_run, args.calibrate_copy)
        return
    if args.batched_counter_run > 0:
        batched_counter_run(hydro, torch, W, args.n, args.batched_counter_run, args.calibrate_copy)
        return
    print("bench: building workload", file=sys.stderr, flush=True)
    lv = W.shear_layer(args.n)
    cells = lv.n_cells
    print("bench: timing %s" % args.dtype, file=sys.stderr, flush=True)
    fused = not args.unfused
    if args.variant is not None:
        args.no_autotune = True
        hydro.set_variant(torch.float64 if args.dtype == "f64" else torch.float32, args.variant)
    el, kms, solver, dts, n_bad, tune = run_workload(hydro, torch, lv, args.dtype, args.steps, args.warmup, fused,
                                                     not args.no_autotune)
    value = cells * args.steps / el
    alg_b = (ALG_BYTES_LEVEL if fused else ALG_BYTES_PADDED)[args.dtype]
    k_rate = cells / (kms * 1e-3)                       # cell updates/s of the MHM kernel alone
    hbm_gbs = alg_b * k_rate / 1e9
    peak_flops = FP64_VEC_PEAK_TFLOPS if args.dtype == "f64" else FP32_VEC_PEAK_TFLOPS
    alu_tflops = ALG_FLOPS_PER_CELL * k_rate / 1e12
    tname = "double" if args.dtype == "f64" else "float"
    hbm = {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
           "alg_bytes_per_cell": alg_b}
    alu = {"achieved": round(alu_tflops, 2), "peak": peak_flops, "unit": "TFLOP/s",
           "frac": round(alu_tflops / peak_flops, 4), "alg_flops_per_cell": ALG_FLOPS_PER_CELL}
    # the binding roof is the one with the lower ceiling for this kernel's
    # algorithmic bytes and flops per cell
    alu_binds = peak_flops * 1e12 / ALG_FLOPS_PER_CELL < HBM_PEAK_GBS * 1e9 / alg_b
    main, other = (alu, hbm) if alu_binds else (hbm, alu)
    roof = {"bound": "alu" if alu_binds else "hbm", "achieved": main["achieved"], "peak": main["peak"],
            "unit": main["unit"], "frac": main["frac"], "traffic": None,
            "kernel": ("mhm_level_kernel<%s, true>" % tname) if fused else ("mhm_padded_kernel<%s>" % tname),
            "kernel_ms": round(kms, 4), "cells_per_launch": cells, "other_roof": other}
    roof["alg_per_cell"] = main.get("alg_flops_per_cell", main.get("alg_bytes_per_cell"))
    if fused:
        shape = tune["variant"] if tune else hydro.get_variant(solver.state.dtype)
        roof["traffic"] = measured_traffic("mhm_level_kernel<%s, true>" % tname, shape)
        # how much of the VALU issue capacity the kernel's measured instruction
        # count uses at this duration (context for the flop roofline: divisions
        # and square roots cost several instructions, selects and moves none)
        valu = measured_profile("mhm_level_kernel<%s, true>" % tname, shape, "valu_insts_per_launch")
        if valu:
            rate = valu / (kms * 1e-3)
            roof["valu_issue"] = {"achieved": round(rate / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
                                  "unit": "G wave-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4),
                                  "per_cell": round(valu / cells, 2)}
    extra = {"kernel_cell_updates_per_s": k_rate, "n_bad": n_bad, "dt_last_step": float(dts[0]),
             "path": "fused level step" if fused else "fill + dt + padded advance", "launch_shape": tune}
    if not args.no_f32 and args.dtype == "f64":
        print("bench: timing f32", file=sys.stderr, flush=True)
        el32, kms32, _, _, nb32, tune32 = run_workload(hydro, torch, lv, "f32", args.steps, args.warmup, fused,
                                                       not args.no_autotune)
        r32 = cells / (kms32 * 1e-3)
        b32 = (ALG_BYTES_LEVEL if fused else ALG_BYTES_PADDED)["f32"]
        extra["f32"] = {"value": cells * args.steps / el32, "ms_per_step": el32 / args.steps * 1e3,
                        "kernel_ms": kms32, "kernel_cell_updates_per_s": r32,
                        "hbm_frac": b32 * r32 / 1e9 / HBM_PEAK_GBS,
                        "alu_frac": ALG_FLOPS_PER_CELL * r32 / 1e12 / FP32_VEC_PEAK_TFLOPS, "n_bad": nb32,
                        "launch_shape": tune32}
        if fused:
            shape32 = tune32["variant"] if tune32 else hydro.get_variant(torch.float32)
            extra["f32"]["traffic"] = measured_traffic("mhm_level_kernel<float, true>", shape32)
    del solver
    torch.cuda.empty_cache()
    if not args.no_amr:
        print("bench: batched multi-level", file=sys.stderr, flush=True)
        extra["amr"] = amr_workload(hydro, torch, W, args.amr_coarse_steps)
        extra["amr_small_levels"] = amr_small_levels(hydro, torch, W, args.amr_coarse_steps)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        print("bench: differentiation workloads", file=sys.stderr, flush=True)
        extra["adjoint"] = differentiation_workloads(hydro, torch, W, args.fd_samples)
        torch.cuda.empty_cache()
    if not args.no_ext:
        print("bench: other schemes", file=sys.stderr, flush=True)
        extra["schemes"] = ext_schemes(hydro, torch, W)
        torch.cuda.empty_cache()
        print("bench: procedure for unphysical results", file=sys.stderr, flush=True)
        extra["fallback"] = fallback_workload(hydro, torch, W)
        torch.cuda.empty_cache()
        print("bench: coupled AMR hierarchy", file=sys.stderr, flush=True)
        extra["amr_coupled"] = amr_coupled(hydro, torch, W)
        torch.cuda.empty_cache()
    if args.calibrate_copy > 0:
        # a plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counter readings calibrate the byte counters of the kernels above
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_calibration_bytes"] = n * 8
        del src, dst
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(lambda: W.shear_layer(args.n), args.cpu_seconds)
    line = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "shear-layer %d^3 periodic, %d patch groups of 16^3 (3 ghost zones), gamma=1.4, "
                               "MHM+PLM+HLLC at CFL 0.5: ghost fill + update + CFL per step" % (args.n, lv.n_groups),
                   "grid": args.n, "groups": lv.n_groups, "ghost": 3, "theta": 1.5},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
