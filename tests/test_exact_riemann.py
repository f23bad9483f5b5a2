"""Self-checks of the exact Riemann solver used as a reference for the oracle:
its solution must satisfy the Rankine-Hugoniot conditions across shocks, keep
the Riemann invariants constant through rarefactions and have continuous
pressure and velocity across the contact."""
import numpy as np

from tests.refsol import exact_riemann as er


def rh_residual(W1, W2, S, g):
    r1, u1, p1 = W1
    r2, u2, p2 = W2
    E1 = p1 / (g - 1) + 0.5 * r1 * u1 * u1
    E2 = p2 / (g - 1) + 0.5 * r2 * u2 * u2
    f1 = np.array([r1 * u1, r1 * u1 * u1 + p1, u1 * (E1 + p1)])
    f2 = np.array([r2 * u2, r2 * u2 * u2 + p2, u2 * (E2 + p2)])
    U1 = np.array([r1, r1 * u1, E1])
    U2 = np.array([r2, r2 * u2, E2])
    return (f2 - f1) - S * (U2 - U1)


def shock_speed_from_samples(xi, rho):
    j = np.argmax(np.abs(np.diff(rho)))
    return 0.5 * (xi[j] + xi[j + 1]), j


def test_sod_right_shock_rankine_hugoniot():
    g = 1.4
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = er.star_state(WL, WR, g)
    rs = WR[0] * (ps / WR[2] + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / WR[2] + 1)
    S = (rs * us - WR[0] * WR[1]) / (rs - WR[0])  # mass conservation fixes the speed
    res = rh_residual((rs, us, ps), WR, S, g)
    assert np.all(np.abs(res) < 1e-12)
    # the sampled solution jumps at that speed
    xi = np.linspace(S - 1e-3, S + 1e-3, 3)
    r, u, p = er.sample(WL, WR, g, xi)
    assert abs(r[0] - rs) < 1e-12 and abs(r[2] - WR[0]) < 1e-15


def test_left_rarefaction_invariants_and_contact():
    g = 1.4
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = er.star_state(WL, WR, g)
    cL = np.sqrt(g * WL[2] / WL[0])
    xi = np.linspace(-cL, us - np.sqrt(g * ps / (WL[0] * (ps / WL[2]) ** (1 / g))), 50)
    r, u, p = er.sample(WL, WR, g, xi)
    c = np.sqrt(g * p / r)
    assert np.allclose(u + 2 * c / (g - 1), 2 * cL / (g - 1), rtol=1e-12)
    assert np.allclose(p / r ** g, WL[2] / WL[0] ** g, rtol=1e-12)
    r2, u2, p2 = er.sample(WL, WR, g, np.array([us - 1e-9, us + 1e-9]))
    assert abs(p2[0] - p2[1]) < 1e-12 and abs(u2[0] - u2[1]) < 1e-12 and r2[0] != r2[1]


def test_symmetric_rarefactions_have_zero_star_velocity():
    g = 1.4
    ps, us = er.star_state((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), g)
    assert abs(us) < 1e-14 and 0 < ps < 0.4


def test_timmes_tube_two_shock_free_structure():
    """Large pressure ratio: left rarefaction, contact, right shock; both
    Rankine-Hugoniot and the pressure-function root hold."""
    g = 1.4
    WL, WR = (10.0, 0.0, 100.0), (1.0, 0.0, 1.0)
    ps, us = er.star_state(WL, WR, g)
    assert WR[2] < ps < WL[2]
    rs = WR[0] * (ps / WR[2] + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / WR[2] + 1)
    S = (rs * us) / (rs - WR[0])
    assert np.all(np.abs(rh_residual((rs, us, ps), WR, S, g)) < 1e-10 * ps)
