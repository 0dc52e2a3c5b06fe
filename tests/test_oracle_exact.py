"""Pins of the oracle's exact Riemann solver (used to pin the MHM scheme on Sod).

The solver finds p* from the pressure functions; these tests check its output
against relations it does not evaluate itself: the Rankine-Hugoniot jump
conditions of the Euler equations across the shock, the isentrope and the
Riemann invariant across the rarefaction, the two-rarefaction closed form, the
mirror symmetry of the problem, and tabulated star values (tests/golden)."""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sod_star.txt")
SOD_L, SOD_R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def _euler_flux_1d(r, u, p, g):
    E = p / (g - 1.0) + 0.5 * r * u * u
    return np.array([r * u, r * u * u + p, (E + p) * u]), np.array([r, r * u, E])


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        rows.append((float(Fraction(tok[0])), *[float(t) for t in tok[1:]]))
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_sod_star_values_golden(row):
    g, ps, us, rl, rr, s_shock, atol = row
    p, u, a, b, _ = oracle.exact_star(SOD_L, SOD_R, g)
    np.testing.assert_allclose([p, u, a, b], [ps, us, rl, rr], rtol=0, atol=atol)
    if not np.isnan(s_shock):
        cR = np.sqrt(g * SOD_R[2] / SOD_R[0])
        S = SOD_R[1] + cR * np.sqrt((g + 1) / (2 * g) * p / SOD_R[2] + (g - 1) / (2 * g))
        np.testing.assert_allclose(S, s_shock, rtol=0, atol=atol)


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_sod_rankine_hugoniot_and_isentrope(g):
    p, u, rl, rr, _ = oracle.exact_star(SOD_L, SOD_R, g)
    # right-moving shock: speed from mass conservation, then momentum and energy jumps
    r0, u0, p0 = SOD_R
    S = (rr * u - r0 * u0) / (rr - r0)
    F1, U1 = _euler_flux_1d(rr, u, p, g)
    F0, U0 = _euler_flux_1d(r0, u0, p0, g)
    np.testing.assert_allclose(F1 - S * U1, F0 - S * U0, rtol=0, atol=1e-13)
    # left rarefaction: isentropic, Riemann invariant u + 2c/(g-1) conserved
    rL, uL, pL = SOD_L
    np.testing.assert_allclose(p / rl ** g, pL / rL ** g, rtol=1e-13)
    cL, cs = np.sqrt(g * pL / rL), np.sqrt(g * p / rl)
    np.testing.assert_allclose(u + 2 * cs / (g - 1), uL + 2 * cL / (g - 1), rtol=1e-13)


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_residual_vanishes_at_root(g):
    p = oracle.exact_star(SOD_L, SOD_R, g)[0]
    assert abs(oracle.exact_residual(SOD_L, SOD_R, g, p)) < 1e-14
    # and it is not trivially zero elsewhere
    assert abs(oracle.exact_residual(SOD_L, SOD_R, g, 1.5 * p)) > 1e-3


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_two_rarefaction_closed_form(g):
    # two rarefactions: both states at p_K > p*; p* then has a closed form
    left, right = (1.0, -0.8, 0.7), (0.6, 0.9, 0.4)
    p, u, _, _, _ = oracle.exact_star(left, right, g)
    assert p < min(left[2], right[2])
    z = (g - 1) / (2 * g)
    cL, cR = np.sqrt(g * left[2] / left[0]), np.sqrt(g * right[2] / right[0])
    closed = ((cL + cR - 0.5 * (g - 1) * (right[1] - left[1])) /
              (cL * left[2] ** -z + cR * right[2] ** -z)) ** (1 / z)
    np.testing.assert_allclose(p, closed, rtol=1e-13)
    # each side on its isentrope with its Riemann invariant
    _, _, rl, rr, _ = oracle.exact_star(left, right, g)
    np.testing.assert_allclose(u + 2 * np.sqrt(g * p / rl) / (g - 1), left[1] + 2 * cL / (g - 1), rtol=1e-12)
    np.testing.assert_allclose(u - 2 * np.sqrt(g * p / rr) / (g - 1), right[1] - 2 * cR / (g - 1), rtol=1e-12)


def test_mirror_symmetry_of_riemann_problem():
    g = 1.4
    left, right = (1.0, 0.3, 2.0), (0.4, -0.2, 0.5)
    p, u, rl, rr, _ = oracle.exact_star(left, right, g)
    mp, mu, mrl, mrr, _ = oracle.exact_star((right[0], -right[1], right[2]), (left[0], -left[1], left[2]), g)
    np.testing.assert_allclose([mp, -mu, mrr, mrl], [p, u, rl, rr], rtol=1e-13)


def test_sampled_profile_structure():
    g = 5.0 / 3.0
    p, u, rl, rr, _ = oracle.exact_star(SOD_L, SOD_R, g)
    xi = np.linspace(-3, 3, 6001)
    r, uu, pp = oracle.exact_sample(SOD_L, SOD_R, g, xi)
    cL = np.sqrt(g)
    assert np.all(r[xi < -cL] == 1.0) and np.all(pp[xi < -cL] == 1.0)
    # inside the fan: isentropic and constant left Riemann invariant
    fan = (xi > -cL + 1e-9) & (xi < u - np.sqrt(g * p / rl) - 1e-9)
    assert fan.sum() > 100
    np.testing.assert_allclose(pp[fan] / r[fan] ** g, 1.0, rtol=1e-12)
    np.testing.assert_allclose(uu[fan] + 2 * np.sqrt(g * pp[fan] / r[fan]) / (g - 1), 2 * cL / (g - 1), rtol=1e-12)
    # star region: pressure and velocity constant across the contact
    star = (xi > u - np.sqrt(g * p / rl) + 1e-9) & (xi < 1.8)
    np.testing.assert_allclose(pp[star], p, rtol=1e-14)
    np.testing.assert_allclose(uu[star], u, rtol=1e-14)
    assert np.all(r[(xi > u + 1e-9) & (xi < 1.8)] == rr)
    assert np.all(r[xi > 1.9] == 0.125)
