"""Test-side drivers that run the CPU oracle over time (no solver arithmetic here)."""

import numpy as np

import oracle


def evolve_to(level, t_end, ghost=3, c_cfl=0.5, theta=1.5, scheme=oracle.SCHEME_MHM_PLM_HLLC, max_steps=100000):
    """Advance a workloads.Level to t_end with the CFL time-step (Eq. 2), the
    last step clipped to land on t_end.  Returns (U, n_steps, n_bad)."""
    U = np.array(level.U, np.float64)
    t, n, n_bad = 0.0, 0, 0
    while t < t_end and n < max_steps:
        pad = oracle.fill_ghosts(U, level.ng, ghost, level.bc)
        dt = float(oracle.dt_patch(pad, level.dx, level.gamma, c_cfl).min())
        if t + dt > t_end:
            dt = t_end - t
        U, nb = oracle.mhm_step(pad, dt, level.dx, level.gamma, theta, scheme)
        n_bad += nb
        t += dt
        n += 1
    return U, n, n_bad


def field_scale_error(got, ref):
    """max over cells of |g - o| / (|o| + ref_f).

    ref_f is the largest |o| of field f over the grid, except that the three
    momentum components share one reference, the largest |o| of any of them:
    a component that vanishes up to round-off (e.g. m_z of a flow in the x-y
    plane) is judged on the momentum scale, not on its own round-off."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    f_axis = 1 if ref.ndim == 5 else 0
    moved_r = np.moveaxis(ref, f_axis, 0).reshape(5, -1)
    moved_g = np.moveaxis(got, f_axis, 0).reshape(5, -1)
    scale = np.abs(moved_r).max(axis=1)
    scale[1:4] = scale[1:4].max()
    scale = np.where(scale > 0, scale, 1.0)[:, None]
    return float((np.abs(moved_g - moved_r) / (np.abs(moved_r) + scale)).max())


def positive_rel_error(got, ref):
    """max over cells of |g - o| / |o| for the strictly positive fields rho and E
    (a per-cell relative check: a field spanning many decades, like the blast
    wave's energy, is not judged on its largest value)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    f_axis = 1 if ref.ndim == 5 else 0
    r = np.moveaxis(ref, f_axis, 0)[[0, 4]].reshape(2, -1)
    g = np.moveaxis(got, f_axis, 0)[[0, 4]].reshape(2, -1)
    return float((np.abs(g - r) / np.abs(r)).max())


def assert_parity(got, ref, tol, msg=""):
    """Per-cell parity: the field-scaled error (momentum on one scale) within
    tol, and for FP64 tolerances (tol <= 1e-11) also the per-cell relative
    error of rho and E.  FP32 results are held to the field scale only: a
    cell's rounding error scales with the largest value its update combines,
    which on a blast wave's exponentially graded flank exceeds the cell's own
    value by up to ~1e3, i.e. ~5e-5 of it in FP32 (FP64: ~1e-13)."""
    e1 = field_scale_error(got, ref)
    e2 = positive_rel_error(got, ref) if tol <= 1e-11 else 0.0
    assert e1 <= tol and e2 <= tol, "%s field-scaled %.3e, rho/E per-cell relative %.3e, tol %.1e" % (
        msg, e1, e2, tol)
