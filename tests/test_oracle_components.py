"""Pins of the oracle's building blocks: limiter, HLLC flux, Hancock predictor.

Each test checks a property the mathematics fixes (special cases that reduce to
a textbook limiter, consistency and upwinding of the Riemann flux, exact
resolution of contacts, symmetry, agreement with the exact Riemann solver's
Godunov flux for weak waves), so that a dropped term, a wrong sign or a
swapped operand in the oracle fails one of them."""

import numpy as np
import pytest

import oracle

G53 = 5.0 / 3.0


def prim2cons(r, u, v, w, p, g):
    return np.array([r, r * u, r * v, r * w, p / (g - 1) + 0.5 * r * (u * u + v * v + w * w)])


def phys_flux(U, d, g):
    """Euler flux along axis d from conserved variables (definition)."""
    r = U[0]
    vel = U[1:4] / r
    p = (g - 1) * (U[4] - 0.5 * r * np.dot(vel, vel))
    F = U * vel[d]
    F[1 + d] += p
    F[4] = (U[4] + p) * vel[d]
    return F


# ------------------------------------------------------------------ limiter --

def _dyadic(rng, n):
    return rng.integers(-64, 65, n) / 16.0


def test_limiter_theta1_is_minmod():
    rng = np.random.default_rng(0)
    for qm, q0, qp in zip(_dyadic(rng, 400), _dyadic(rng, 400), _dyadic(rng, 400)):
        dm, dp = q0 - qm, qp - q0
        mm = 0.0 if dm * dp <= 0 else np.sign(dm) * min(abs(dm), abs(dp))
        assert oracle.limited_slope(qm, q0, qp, 1.0) == mm


def test_limiter_theta2_is_monotonized_central():
    rng = np.random.default_rng(1)
    for qm, q0, qp in zip(_dyadic(rng, 400), _dyadic(rng, 400), _dyadic(rng, 400)):
        dm, dp = q0 - qm, qp - q0
        mc = 0.0 if dm * dp <= 0 else np.sign(dm) * min(2 * abs(dm), 2 * abs(dp), 0.5 * abs(dm + dp))
        assert oracle.limited_slope(qm, q0, qp, 2.0) == mc


@pytest.mark.parametrize("theta", [1.0, 1.3, 1.5, 2.0])
def test_limiter_tvd_and_linear_exactness(theta):
    rng = np.random.default_rng(2)
    q = rng.normal(size=(2000, 3))
    for qm, q0, qp in q:
        s = oracle.limited_slope(qm, q0, qp, theta)
        lo, hi = min(qm, q0, qp), max(qm, q0, qp)
        # face values stay inside the neighbour range (TVD for theta <= 2)
        assert lo - 1e-15 <= q0 - 0.5 * s <= hi + 1e-15
        assert lo - 1e-15 <= q0 + 0.5 * s <= hi + 1e-15
        if (q0 - qm) * (qp - q0) <= 0:
            assert s == 0.0  # extrema are flattened
    # linear data: the central difference is returned exactly
    for a, b in rng.integers(-50, 50, (200, 2)) / 8.0:
        if b == 0:
            continue
        assert oracle.limited_slope(a - b, a, a + b, theta) == b


# --------------------------------------------------------------------- HLLC --

@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("ws", [0, 1])
def test_hllc_consistency(d, ws):
    rng = np.random.default_rng(10 + d)
    for _ in range(50):
        U = prim2cons(rng.uniform(0.2, 3), *rng.normal(0, 2, 3), rng.uniform(0.2, 3), G53)
        F, bad = oracle.hllc(U, U, d, G53, ws)
        assert not bad
        ref = phys_flux(U, d, G53)
        assert np.all(np.abs(F - ref) <= 8 * np.finfo(float).eps * (np.abs(ref) + np.abs(U).max()))


@pytest.mark.parametrize("ws", [0, 1])
def test_hllc_supersonic_upwinding(ws):
    g = G53
    UL = prim2cons(1.0, 5.0, 0.3, -0.2, 1.0, g)   # u - c > 0 on both sides
    UR = prim2cons(0.5, 4.5, 0.1, 0.4, 0.7, g)
    F, _ = oracle.hllc(UL, UR, 0, g, ws)
    np.testing.assert_allclose(F, phys_flux(UL, 0, g), rtol=1e-15, atol=1e-15)
    UL2 = prim2cons(1.0, -5.0, 0.3, -0.2, 1.0, g)
    UR2 = prim2cons(0.5, -4.5, 0.1, 0.4, 0.7, g)
    F2, _ = oracle.hllc(UL2, UR2, 0, g, ws)
    np.testing.assert_allclose(F2, phys_flux(UR2, 0, g), rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("u", [0.4, -0.4])
def test_hllc_resolves_isolated_contact(u):
    g = G53
    UL = prim2cons(2.0, u, 0.3, -0.1, 1.5, g)
    UR = prim2cons(0.3, u, -0.7, 0.2, 1.5, g)
    F, _ = oracle.hllc(UL, UR, 0, g, 0)
    up = UL if u > 0 else UR
    np.testing.assert_allclose(F, phys_flux(up, 0, g), rtol=1e-13, atol=1e-14)


def test_hllc_stationary_contact_exact():
    g = G53
    UL = prim2cons(2.0, 0.0, 0.0, 0.0, 1.0, g)
    UR = prim2cons(0.25, 0.0, 0.0, 0.0, 1.0, g)
    for d in range(3):
        F, _ = oracle.hllc(UL, UR, d, g, 0)
        p = (g - 1) * UL[4]
        expect = np.zeros(5)
        expect[1 + d] = p
        assert np.array_equal(F, expect)


@pytest.mark.parametrize("ws", [0, 1])
def test_hllc_rotation_and_mirror(ws):
    # both wave-speed estimates map to their mirror image (S_L <-> -S_R), so
    # the mirrored problem's flux is the mirrored flux; a wrong term in either
    # speed breaks it
    g = G53
    rng = np.random.default_rng(3)
    for _ in range(40):
        UL = prim2cons(rng.uniform(0.2, 3), *rng.normal(0, 1, 3), rng.uniform(0.2, 3), g)
        UR = prim2cons(rng.uniform(0.2, 3), *rng.normal(0, 1, 3), rng.uniform(0.2, 3), g)
        Fx, _ = oracle.hllc(UL, UR, 0, g, ws)
        # rotate (x, y, z) -> (y, z, x): the y-face flux of the rotated states
        rot = [0, 3, 1, 2, 4]
        Fy, _ = oracle.hllc(UL[rot], UR[rot], 1, g, ws)
        assert np.array_equal(Fy, Fx[rot])
        # mirror x -> -x swaps the sides and flips normal momentum
        M = np.array([1, -1, 1, 1, 1.0])
        Fm, _ = oracle.hllc(UR * M, UL * M, 0, g, ws)
        np.testing.assert_allclose(Fm, -Fx * M, rtol=1e-12, atol=1e-13)


def test_hllc_davis_and_roe_agree_when_supersonic():
    g = G53
    UL = prim2cons(1.0, 6.0, 0.0, 0.0, 1.0, g)
    UR = prim2cons(0.9, 5.5, 0.2, 0.0, 0.8, g)
    assert np.array_equal(oracle.hllc(UL, UR, 0, g, 0)[0], oracle.hllc(UL, UR, 0, g, 1)[0])


@pytest.mark.parametrize("ws", [0, 1])
def test_hllc_close_to_exact_godunov_flux_for_weak_waves(ws):
    g = 1.4
    for eps in (1e-2, 1e-3):
        left, right = (1.0, 0.2, 1.0), (1.0 - eps, 0.2 + 0.5 * eps, 1.0 - 1.3 * eps)
        r, u, p = oracle.exact_sample(left, right, g, np.array([0.0]))
        Fex = phys_flux(prim2cons(r[0], u[0], 0, 0, p[0], g), 0, g)
        F, _ = oracle.hllc(prim2cons(left[0], left[1], 0, 0, left[2], g),
                           prim2cons(right[0], right[1], 0, 0, right[2], g), 0, g, ws)
        assert np.abs(F - Fex).max() < 5 * eps ** 2


def test_hllc_flags_unphysical_states():
    g = G53
    good = prim2cons(1.0, 0.1, 0, 0, 1.0, g)
    bad_rho = good.copy()
    bad_rho[0] = -0.1
    bad_p = prim2cons(1.0, 0.1, 0, 0, 1.0, g)
    bad_p[4] = 0.001
    assert not oracle.hllc(good, good, 0, g, 0)[1]
    assert oracle.hllc(bad_rho, good, 0, g, 0)[1]
    assert oracle.hllc(good, bad_p, 0, g, 0)[1]


# ------------------------------------------------------------------ Hancock --

def test_hancock_first_order_and_uniform():
    g = G53
    rng = np.random.default_rng(4)
    Wc = np.array([1.2, 0.3, -0.2, 0.1, 0.9])
    Wm = rng.normal(0, 0.1, (3, 5)) + Wc
    Wp = rng.normal(0, 0.1, (3, 5)) + Wc
    Ut = oracle.hancock_cell(Wc, Wm, Wp, g, 1.5, 0.2, first_order=True)
    U = oracle.prim_to_cons(Wc, g)
    assert np.array_equal(Ut, np.broadcast_to(U, (3, 2, 5)))
    # uniform neighbours: no slope, no evolution
    Ut = oracle.hancock_cell(Wc, np.tile(Wc, (3, 1)), np.tile(Wc, (3, 1)), g, 1.5, 0.2)
    assert np.array_equal(Ut, np.broadcast_to(U, (3, 2, 5)))


def test_hancock_predictor_matches_conservative_half_step():
    """Linear data in x only: face states W -+ s/2 advanced by
    dt/(2dx) [F(U_-) - F(U_+)], independent of theta (slope = central)."""
    g = G53
    Wc = np.array([1.0, 0.5, 0.0, 0.0, 1.0])
    dW = np.array([0.05, 0.01, 0.0, 0.0, 0.04])
    Wm = np.tile(Wc, (3, 1))
    Wp = np.tile(Wc, (3, 1))
    Wm[0], Wp[0] = Wc - dW, Wc + dW
    h = 0.3
    Ut = oracle.hancock_cell(Wc, Wm, Wp, g, 1.5, h)
    Um = prim2cons(*(Wc - 0.5 * dW), g)
    Up = prim2cons(*(Wc + 0.5 * dW), g)
    dU = h * (phys_flux(Um, 0, g) - phys_flux(Up, 0, g))
    np.testing.assert_allclose(Ut[0, 0], Um + dU, rtol=1e-14)
    np.testing.assert_allclose(Ut[0, 1], Up + dU, rtol=1e-14)
    np.testing.assert_allclose(Ut[1, 0], prim2cons(*Wc, g) + dU, rtol=1e-14)
    # the half step moves mass against the gradient of the flux
    assert dU[0] < 0


def test_prim_cons_roundtrip():
    g = G53
    rng = np.random.default_rng(5)
    for _ in range(100):
        W = np.array([rng.uniform(0.1, 5), *rng.normal(0, 2, 3), rng.uniform(0.1, 5)])
        np.testing.assert_allclose(oracle.cons_to_prim(oracle.prim_to_cons(W, g), g), W, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(oracle.prim_to_cons(W, g), prim2cons(*W, g), rtol=1e-15)


def _shock_pair(r0, p0, mach, g):
    """Pre-shock state at rest-frame speed 0 with a 1-shock (left-facing)
    moving at speed S: Rankine-Hugoniot from the normal Mach number."""
    c0 = np.sqrt(g * p0 / r0)
    w0 = mach * c0                                        # upstream speed in the shock frame
    r1 = r0 * (g + 1) * mach ** 2 / ((g - 1) * mach ** 2 + 2)
    p1 = p0 * (2 * g * mach ** 2 - (g - 1)) / (g + 1)
    w1 = w0 * r0 / r1
    return (r0, w0, p0), (r1, w1, p1)


@pytest.mark.parametrize("S", [0.0, -0.3, 0.25])
@pytest.mark.parametrize("mach", [1.5, 3.0])
def test_hllc_resolves_isolated_shock(S, mach):
    """For two states joined by one shock, the Roe-averaged speed equals the
    shock speed, so HLLC with Einfeldt/Roe speeds returns the exact Godunov
    flux (F_R if the shock moves left, F_L if it moves right)."""
    g = 1.4
    (r0, w0, p0), (r1, w1, p1) = _shock_pair(1.0, 1.0, mach, g)
    UL = prim2cons(r0, w0 + S, 0.2, -0.1, p0, g)      # upstream on the left: a 1-shock
    UR = prim2cons(r1, w1 + S, 0.2, -0.1, p1, g)
    FL, FR = phys_flux(UL, 0, g), phys_flux(UR, 0, g)
    np.testing.assert_allclose(FR - FL, S * (UR - UL), rtol=1e-12, atol=1e-12)   # R-H check of the pair
    F, _ = oracle.hllc(UL, UR, 0, g, 0)
    np.testing.assert_allclose(F, FR if S <= 0 else FL, rtol=1e-12, atol=1e-12)


def _brute_fill(level, ng, ghost, bc):
    ngx, ngy, ngz = ng
    N = 16
    grid = np.zeros((5, ngz * N, ngy * N, ngx * N))
    for g in range(ngx * ngy * ngz):
        gx, gy, gz = g % ngx, (g // ngx) % ngy, g // (ngx * ngy)
        grid[:, gz * N:(gz + 1) * N, gy * N:(gy + 1) * N, gx * N:(gx + 1) * N] = level[g]
    P = N + 2 * ghost
    out = np.zeros((ngx * ngy * ngz, 5, P, P, P))
    dims = grid.shape[1:][::-1]

    def src(i, n, lo, hi):
        if i < 0:
            return i + n if lo == 0 else 0
        if i >= n:
            return i - n if hi == 0 else n - 1
        return i
    for g in range(ngx * ngy * ngz):
        gx, gy, gz = g % ngx, (g // ngx) % ngy, g // (ngx * ngy)
        for z in range(P):
            Z = src(gz * N + z - ghost, dims[2], bc[4], bc[5])
            for y in range(P):
                Y = src(gy * N + y - ghost, dims[1], bc[2], bc[3])
                for x in range(P):
                    X = src(gx * N + x - ghost, dims[0], bc[0], bc[1])
                    out[g, :, z, y, x] = grid[:, Z, Y, X]
    return out


@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 0, 0), (1, 1, 0, 0, 1, 1), (1, 0, 1, 1, 0, 1)])
def test_ghost_fill_definition(bc):
    rng = np.random.default_rng(sum(bc))
    ng = (2, 1, 2)
    level = rng.normal(size=(4, 5, 16, 16, 16))
    np.testing.assert_array_equal(oracle.fill_ghosts(level, ng, 3, bc), _brute_fill(level, ng, 3, bc))
