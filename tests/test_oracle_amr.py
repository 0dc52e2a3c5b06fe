"""Pins of the oracle's coarse-fine coupling (Sec. 2.1 W-cycle, Sec. 2.2
restriction and flux fix-up, Sec. 3.2 ghost zones from siblings or coarse
interpolation) against what the mathematics fixes.

* conservation: in a periodic domain the composite sum (uncovered cells of
  every level times their volume) is conserved to round-off over a coarse
  step -- only if the fine fluxes across the interface replace the coarse
  ones (fix-up), the registers average them correctly over time and area,
  and the restriction is volume-weighted
* a uniform flow stays uniform on every level, bitwise
* a fine level covering the whole domain advances exactly as a uniform fine
  grid does in two steps of dt/2, and the coarse level becomes its
  restriction (bitwise)
* ghost interpolation reproduces linear data exactly, in space and in time
* a hierarchy symmetric about the domain centre keeps a centred blast
  mirror-symmetric
"""

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W
from tests.oracle_runs import field_scale_error

G53 = 5.0 / 3.0
# n0 = 2 groups per axis (32^3 coarse cells); level 1 refines the central 2^3
# coarse patches, level 2 the central 2^3 level-1 patches
SMALL3 = (((1, 3), (1, 3), (1, 3)), ((3, 5), (3, 5), (3, 5)))


def composite_sum(h, states):
    """sum over the uncovered cells of every level of U dx_l^3 (per field)."""
    total = np.zeros(5)
    for l, U in enumerate(states):
        dv = (h.dx0 / 2 ** l) ** 3
        covered = np.zeros(U.shape[0:1] + (16, 16, 16), bool)
        if l + 1 < h.n_levels:
            m = {tuple(p): g for g, p in enumerate(h.positions[l])}
            for px, py, pz in h.positions[l + 1]:
                g = m[(px >> 1, py >> 1, pz >> 1)]
                covered[g, (pz & 1) * 8:(pz & 1) * 8 + 8, (py & 1) * 8:(py & 1) * 8 + 8,
                        (px & 1) * 8:(px & 1) * 8 + 8] = True
        for q in range(5):
            total[q] += U[:, q][~covered].sum() * dv
    return total


def test_composite_conservation_periodic():
    h = W.sedov_hierarchy(n0=2, boxes=SMALL3)
    # add a flow so every field crosses the interfaces
    rng = np.random.default_rng(2)
    for l in range(h.n_levels):
        X, Y, Z = W._level_cells(h.positions[l], h.dx0 / 2 ** l)
        h.states[l][:, 1] += 0.3 * np.sin(2 * np.pi * Y)
        h.states[l][:, 2] += 0.2 * np.cos(2 * np.pi * Z)
        h.states[l][:, 3] += 0.1 * np.sin(2 * np.pi * X)
        h.states[l][:, 4] += 0.5
    del rng
    W.restrict_states(h)
    s0 = composite_sum(h, h.states)
    states = h.states
    for _ in range(2):
        states, nb = oracle.amr_step(h.n0, h.positions, states, h.bc, 2e-4, h.dx0, h.gamma)
        assert nb == 0
    s1 = composite_sum(h, states)
    mag = sum(np.abs(U).sum(axis=(0, 2, 3, 4)) * (h.dx0 / 2 ** l) ** 3 for l, U in enumerate(h.states))
    n_cells = sum(U[:, 0].size for U in h.states)
    tol = 20 * n_cells * np.finfo(float).eps * mag
    assert np.all(np.abs(s1 - s0) <= tol), (s1 - s0, tol)
    assert not np.array_equal(states[2], h.states[2])


def test_uniform_flow_stays_uniform_on_every_level():
    h = W.sedov_hierarchy(n0=2, boxes=SMALL3)
    u = W.conserved(1.3, 0.7, -0.4, 0.25, 0.8, G53)
    states = [np.broadcast_to(u[None, :, None, None, None], s.shape).copy() for s in h.states]
    out, _ = oracle.amr_step(h.n0, h.positions, states, h.bc, 1e-3, h.dx0, G53)
    for a, b in zip(out, states):
        assert np.array_equal(a, b)


def test_full_refinement_equals_uniform_fine_grid():
    lv = W.white_noise(32)                      # the fine grid: 2^3 groups of the fine level
    fine_grid = W.groups_to_grid(lv.U, lv.ng)
    coarse = fine_grid.reshape(5, 16, 2, 16, 2, 16, 2).mean(axis=(2, 4, 6))
    pos = W.nested_positions(1, (((0, 2), (0, 2), (0, 2)),))
    states = [W.grid_to_groups(coarse), lv.U.copy()]
    h = W.AmrHierarchy((1, 1, 1), pos, states, 1.0 / 16, G53)
    W.restrict_states(h)
    dt = 1e-3
    out, nb = oracle.amr_step(h.n0, h.positions, h.states, h.bc, dt, h.dx0, G53)
    ref = lv.U
    for _ in range(2):
        ref, _ = oracle.level_step_any(ref, lv.ng, 3, lv.bc, 0.5 * dt, lv.dx, G53)
    assert np.array_equal(out[1], ref)
    fg = W.groups_to_grid(ref, lv.ng)
    c = lambda dx, dy, dz: fg[:, dz::2, dy::2, dx::2]
    r = ((c(0, 0, 0) + c(1, 0, 0)) + (c(0, 1, 0) + c(1, 1, 0))) + ((c(0, 0, 1) + c(1, 0, 1)) + (c(0, 1, 1) + c(1, 1, 1)))
    assert np.array_equal(out[0][0], 0.125 * r)


def test_ghost_interpolation_linear_in_space_and_time():
    pos = W.nested_positions(2, (((1, 3), (1, 3), (1, 3)),))
    N = 32
    x = (np.arange(N) + 0.5) / N
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    coef = np.array([[1.0, 0.5, -0.25, 0.125], [0.3, -0.5, 0.25, 0.75], [0.1, 0.25, 1.0, -0.5],
                     [0.2, -0.125, 0.5, 0.25], [3.0, 1.0, 0.5, -0.75]])
    lin = lambda c, X, Y, Z: c[0] + c[1] * X + c[2] * Y + c[3] * Z
    old = np.stack([lin(c, X, Y, Z) for c in coef])
    new = np.stack([lin(c[::-1], X, Y, Z) for c in coef])
    co, cn = W.grid_to_groups(old), W.grid_to_groups(new)
    fine = np.zeros((8, 5, 16, 16, 16))
    h = W.AmrHierarchy((2, 2, 2), pos, [co, fine], 1.0 / 32, G53)
    for a in (0.0, 0.5):
        pad = oracle.amr_fill(h.n0, h.positions, h.states, h.bc, 1, co, cn, a, ghost=3)
        for g, (px, py, pz) in enumerate(pos[1]):
            i = (np.arange(-3, 19) + 0.5) / 64
            fz, fy, fx = np.meshgrid(pz * 16 / 64 + i, py * 16 / 64 + i, px * 16 / 64 + i, indexing="ij")
            inside = (np.abs(fx - 0.5) < 0.25) & (np.abs(fy - 0.5) < 0.25) & (np.abs(fz - 0.5) < 0.25)
            for q, c in enumerate(coef):
                want = (1 - a) * lin(c, fx, fy, fz) + a * lin(c[::-1], fx, fy, fz)
                got = pad[g, q]
                # ghost cells outside the fine region are interpolated; inside it they are
                # sibling copies (zeros here)
                np.testing.assert_allclose(got[~inside], want[~inside], rtol=1e-13, atol=1e-13)


def test_centred_blast_stays_mirror_symmetric():
    h = W.sedov_hierarchy(n0=2, boxes=SMALL3)
    out, nb = oracle.amr_step(h.n0, h.positions, h.states, h.bc, 2e-6, h.dx0, h.gamma)
    assert nb == 0
    for l in range(h.n_levels):
        n = [v << l for v in h.n0]
        m = h.dense_map(l)
        grid_pos = h.positions[l]
        for g, (px, py, pz) in enumerate(grid_pos):
            gm = m[pz, py, n[0] - 1 - px]                 # the mirror group across x = 1/2
            a = out[l][g]
            b = out[l][gm][:, :, :, ::-1].copy()
            b[1] *= -1
            assert field_scale_error(a, b) < 1e-13 or np.abs(a - b).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("scheme", [oracle.SCHEME_MHM_PLM_HLLC, oracle.SCHEME_CTU | oracle.PPM | oracle.RIEMANN_ROE])
def test_patch_boundary_fluxes_balance_each_patch(scheme):
    """The fluxes step_any_flux reports on the patch-boundary faces are the
    ones the update used: for every 8^3 patch of every group, the change of
    the patch's sum of U equals -dt/dx times the net flux through its six
    faces (to round-off).  A wrong plane, a transposed (a, b) pair or a
    flipped orientation breaks the balance of some patch."""
    lv = W.white_noise(32)
    pad = oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc)
    dt = 1e-3
    out, ff, nb = oracle.step_any_flux(pad, dt, lv.dx, lv.gamma, 1.5, scheme)
    ref, _ = oracle.step_any(pad, dt, lv.dx, lv.gamma, 1.5, scheme)
    assert nb == 0 and np.array_equal(out, ref)
    dU = out - lv.U
    dtdx = dt / lv.dx
    for g in range(lv.n_groups):
        for pz in range(2):
            for py in range(2):
                for px in range(2):
                    zs, ys, xs = (slice(8 * v, 8 * v + 8) for v in (pz, py, px))
                    lhs = dU[g][:, zs, ys, xs].sum(axis=(1, 2, 3))
                    fx = ff[g, px + 1][:, zs, ys].sum(axis=(1, 2)) - ff[g, px][:, zs, ys].sum(axis=(1, 2))
                    fy = ff[g, 3 + py + 1][:, xs, zs].sum(axis=(1, 2)) - ff[g, 3 + py][:, xs, zs].sum(axis=(1, 2))
                    fz = ff[g, 6 + pz + 1][:, ys, xs].sum(axis=(1, 2)) - ff[g, 6 + pz][:, ys, xs].sum(axis=(1, 2))
                    rhs = -dtdx * (fx + fy + fz)
                    scale = np.abs(dU[g][:, zs, ys, xs]).sum(axis=(1, 2, 3)) + 1e-300
                    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale + 1e-15), (g, px, py, pz, lhs, rhs)
