"""Pins of the finite-difference protocol for the rollout gradient (CPU).

The differentiation workload (128^3 smooth density wave, uniform v and p)
has every velocity and pressure slope of its initial state equal to a
round-off difference, i.e. on the generalized minmod's kink: along any single
input entry the rollout is only piecewise smooth, with a switch within
round-off of the base point.  A central difference then straddles the switch
and averages the two one-sided derivatives, while the exact derivative (the
oracle's dual numbers, like the adjoint) takes the branch of the base point.
The protocol therefore rejects a sample whose +eps and -eps evaluations take
different branches anywhere, which the oracle reports as a hash of every
branch decision (``oracle.rollout_box(signature=True)``).  These tests pin
that finding and the rejection rule on a smaller grid of the same recipe:
signatures differ and FD != JVP on the workload as stated; signatures agree
and FD == JVP to 1e-6 when v and p vary smoothly.
"""

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W

EPS = 1e-7


def box_around(grid, c, R):
    """The periodic box [5, 2R+1, 2R+1, 2R+1] centred on cell c = (x, y, z)."""
    x, y, z = c
    nz, ny, nx = grid.shape[1:]
    iz = np.arange(z - R, z + R + 1) % nz
    iy = np.arange(y - R, y + R + 1) % ny
    ix = np.arange(x - R, x + R + 1) % nx
    return grid[:, iz][:, :, iy][:, :, :, ix]


def sample(lv, n_steps, f, c):
    """(signatures of the +-EPS runs, max |FD - JVP| / max |JVP| over the cone)."""
    grid = W.groups_to_grid(lv.U, lv.ng)
    R = 4 * n_steps            # the 2n cone plus the 2n the cone depends on
    dt = 0.2 * lv.dx
    box = box_around(grid, c, R)
    t = np.zeros_like(box)
    t[f, R, R, R] = 1.0
    _, jvp, _, _ = oracle.rollout_box(box, n_steps, dt, lv.dx, lv.gamma, tangent=t)
    runs = []
    for s in (1.0, -1.0):
        b = box.copy()
        b[f, R, R, R] += s * EPS
        o, _, _, sig = oracle.rollout_box(b, n_steps, dt, lv.dx, lv.gamma, signature=True)
        runs.append((o, sig))
    fd = (runs[0][0] - runs[1][0]) / (2 * EPS)
    return runs[0][1], runs[1][1], float(np.abs(fd - jvp).max() / np.abs(jvp).max())


CELLS = [(0, (20, 16, 8)), (1, (1, 2, 0)), (2, (19, 31, 23)), (3, (17, 17, 29)), (4, (23, 27, 5))]


@pytest.mark.parametrize("f,c", CELLS)
def test_workload_as_stated_sits_on_limiter_kinks(f, c):
    """Uniform v and p: the +eps and -eps runs branch differently and the
    central difference misses the exact derivative by far more than 1e-6."""
    lv, _ = W.smooth_wave(32)
    sp, sm, err = sample(lv, 2, f, c)
    assert sp != sm
    assert err > 1e-3


@pytest.mark.parametrize("f,c", CELLS)
def test_smooth_v_and_p_central_difference_equals_jvp(f, c):
    lv, _ = W.smooth_wave(32, smooth_vp=0.01)
    sp, sm, err = sample(lv, 2, f, c)
    assert sp == sm
    assert err < 1e-6


def test_signature_sees_a_single_limiter_switch():
    """Density rising along x by 1e-12 per cell through the centre: perturbing
    the centre cell by +-1e-9 makes the one-sided differences of its +x
    neighbour of one sign in one run and of opposite signs in the other."""
    lv, _ = W.smooth_wave(32, smooth_vp=0.01)
    grid = W.groups_to_grid(lv.U, lv.ng)
    box = box_around(grid, (5, 5, 5), 8)
    box[0] = box[0, 8, 8, 8] + 1e-12 * np.arange(17)[None, None, :]
    dt = 0.2 * lv.dx
    sigs = []
    for s in (1.0, -1.0):
        b = box.copy()
        b[0, 8, 8, 8] += s * 1e-9
        sigs.append(oracle.rollout_box(b, 1, dt, lv.dx, lv.gamma, signature=True)[3])
    assert sigs[0] != sigs[1]
    same = [oracle.rollout_box(box, 1, dt, lv.dx, lv.gamma, signature=True)[3] for _ in range(2)]
    assert same[0] == same[1]


def test_box_rollout_equals_level_rollout():
    """The box form (no ghost refill, shrinking margin) gives the level
    rollout's values bitwise on the cells it determines."""
    lv, _ = W.smooth_wave(32, smooth_vp=0.01)
    dt = 0.2 * lv.dx
    ref, _, _ = oracle.rollout(lv.U, lv.ng, 3, lv.bc, 2, lv.dx, lv.gamma, dt=dt)
    grid, rgrid = W.groups_to_grid(lv.U, lv.ng), W.groups_to_grid(ref, lv.ng)
    c = (3, 30, 17)
    out, _, _, _ = oracle.rollout_box(box_around(grid, c, 12), 2, dt, lv.dx, lv.gamma)
    np.testing.assert_array_equal(out, box_around(rgrid, c, 8))
