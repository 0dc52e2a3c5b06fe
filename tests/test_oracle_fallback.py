"""Pins of the oracle's procedure for unphysical results (Sec. 2.2, steps
(ii)-(v)): cells whose update gives rho <= 0 or p <= 0 are recomputed
first-order unsplit, then first-order split, then the level is retried with
dt * 0.8 down to a minimum.

* a state with no unphysical cell: the procedure returns the plain step bitwise
* first-order split == first-order unsplit bitwise on 1D data (the transverse
  flux differences are exact zeros)
* a repaired (unsplit) cell equals the first-order scheme's value there (a
  second code path: zero slopes through the whole MHM step), every other cell
  the plain step's bitwise, and no cell is left unphysical
* a split repair equals three first-order sweeps computed here from the
  Riemann solver alone (brute force on the 3x3x3 block)
* retries: the accepted dt is dt0 * 0.8^k with k the retry count, the result
  equals the procedure started at that dt with no retry, and a minimum dt
  above it stops the retries with cells still unphysical
"""

import numpy as np

import oracle
from paper_1712_07070_amd import workloads as W

G53 = 5.0 / 3.0


def noisy_state(seed=0, n=32):
    """White noise with low pressures: MHM's update fails on some hundred cells."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.05, 2, (n, n, n))
    p = np.exp(rng.uniform(np.log(1e-3), np.log(2.0), (n, n, n)))
    v = rng.normal(0, 0.5, (3, n, n, n))
    U = W.grid_to_groups(W.conserved(rho, v[0], v[1], v[2], p, G53))
    ng = (n // 16,) * 3
    dx = 1.0 / n
    dt = float(oracle.dt_patch(oracle.fill_ghosts(U, ng, 3, (0,) * 6), dx, G53, 0.5).min())
    return U, ng, dx, dt


def octant_state(n=32, s=2.0, p=0.01):
    """Cold gas streaming out of the box centre along every axis: a first-order
    unsplit update empties the central cells at dt = 0.3 dx."""
    x = (np.arange(n) + 0.5) / n - 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    U = W.grid_to_groups(W.conserved(np.ones((n, n, n)), s * np.sign(X), s * np.sign(Y), s * np.sign(Z),
                                     np.full((n, n, n), p), G53))
    return U, (n // 16,) * 3, 1.0 / n


def unphysical(U):
    r = U[:, 0]
    p = (G53 - 1) * (U[:, 4] - 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2 + U[:, 3] ** 2) / r)
    return ~((r > 0) & (p > 0))


def test_no_unphysical_cell_gives_the_plain_step():
    lv = W.white_noise(32)
    dt = float(oracle.dt_patch(oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc), lv.dx, lv.gamma, 0.5).min())
    a, nb = oracle.level_step_any(lv.U, lv.ng, 3, lv.bc, dt, lv.dx, lv.gamma)
    b, left, info = oracle.level_step_fallback(lv.U, lv.ng, 3, lv.bc, dt, lv.dx, lv.gamma)
    assert nb == 0 and left == 0
    assert info == {"dt": dt, "retries": 0, "unsplit": 0, "split": 0}
    assert np.array_equal(a, b)


def test_split_equals_unsplit_on_1d_data():
    lv = W.sod_tube(64)
    rng = np.random.default_rng(1)
    for X in rng.integers(0, 64, 12):
        Y, Z = rng.integers(0, 16, 2)
        a = oracle.first_order_cell(lv.U, lv.ng, lv.bc, int(X), int(Y), int(Z), 0.3, G53, split=False)
        b = oracle.first_order_cell(lv.U, lv.ng, lv.bc, int(X), int(Y), int(Z), 0.3, G53, split=True)
        assert np.array_equal(a, b)


def test_unsplit_repair_is_the_first_order_scheme():
    U, ng, dx, dt = noisy_state()
    plain, nb = oracle.level_step_any(U, ng, 3, (0,) * 6, dt, dx, G53)
    bad = unphysical(plain)
    assert bad.sum() > 100 and nb > 0
    out, left, info = oracle.level_step_fallback(U, ng, 3, (0,) * 6, dt, dx, G53)
    assert left == 0 and info["retries"] == 0 and info["split"] == 0
    assert info["unsplit"] == int(bad.sum())
    assert not unphysical(out).any()
    fo, _ = oracle.level_step_any(U, ng, 3, (0,) * 6, dt, dx, G53, scheme=oracle.SCHEME_MHM | oracle.FIRST_ORDER)
    m = np.broadcast_to(bad[:, None], out.shape)
    assert np.array_equal(out[~m], plain[~m])
    np.testing.assert_allclose(out[m], fo[m], rtol=1e-12, atol=1e-14)


def test_split_repair_is_three_first_order_sweeps():
    U, ng, dx = octant_state()
    dt = 0.3 * dx
    plain, _ = oracle.level_step_any(U, ng, 3, (0,) * 6, dt, dx, G53)
    out, left, info = oracle.level_step_fallback(U, ng, 3, (0,) * 6, dt, dx, G53)
    assert left == 0 and info["retries"] == 0 and info["split"] > 0
    assert not unphysical(out).any()
    grid = W.groups_to_grid(U, ng)
    og = W.groups_to_grid(out, ng)
    bad = W.groups_to_grid(unphysical(plain)[:, None].astype(float), ng)[0] > 0
    n = grid.shape[1]
    dtdx = dt / dx
    cells = np.argwhere(bad)[:10]
    for z, y, x in cells:
        B = np.stack([[[grid[:, (z + k) % n, (y + j) % n, (x + i) % n] for i in (-1, 0, 1)] for j in (-1, 0, 1)]
                      for k in (-1, 0, 1)])          # [k][j][i][5]
        fo = oracle.SCHEME_MHM | oracle.FIRST_ORDER

        def sweep(Um, U0, Up, d):
            Fm, _ = oracle.riemann(Um, U0, d, G53, fo)
            Fp, _ = oracle.riemann(U0, Up, d, G53, fo)
            return U0 - dtdx * (Fp - Fm)

        C = {(k, j): sweep(B[k, j, 0], B[k, j, 1], B[k, j, 2], 0) for k in range(3) for j in range(3)}
        D = [sweep(C[(k, 0)], C[(k, 1)], C[(k, 2)], 1) for k in range(3)]
        ref = sweep(D[0], D[1], D[2], 2)
        unsplit_ref = oracle.first_order_cell(U, ng, (0,) * 6, int(x), int(y), int(z), dtdx, G53, split=False)
        assert unphysical(unsplit_ref[None])[0]       # the unsplit recomputation failed here
        np.testing.assert_array_equal(og[:, z, y, x], ref)


def test_retries_reduce_dt_by_the_ratio():
    U, ng, dx = octant_state()
    dt0 = 0.5 * dx
    out, left, info = oracle.level_step_fallback(U, ng, 3, (0,) * 6, dt0, dx, G53)
    k = info["retries"]
    assert left == 0 and k >= 1
    assert info["dt"] == dt0 * 0.8 ** k or abs(info["dt"] / (dt0 * 0.8 ** k) - 1) < 1e-15
    again, left2, info2 = oracle.level_step_fallback(U, ng, 3, (0,) * 6, info["dt"], dx, G53)
    assert left2 == 0 and info2["retries"] == 0 and np.array_equal(again, out)
    stuck, left3, info3 = oracle.level_step_fallback(U, ng, 3, (0,) * 6, dt0, dx, G53, dt_min=info["dt"] * 1.01)
    assert left3 > 0 and info3["retries"] == k - 1
