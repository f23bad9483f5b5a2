"""Pins of the oracle's building blocks (reconstruction, Riemann solvers,
closure) against textbook facts and independent derivations (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import inputs
from paper_2110_01792_amd.inputs import rad_params
from tests.refsol import exact_riemann as er


# ------------------------------------------------------------------ PPM
def test_ppm_exact_on_linear_data():
    """Linear cell averages: the interface value is exact and no limiter fires,
    so the reconstruction is the line itself."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, s = rng.normal(), rng.normal()
        q = a + s * np.arange(-2, 3)
        aL, aR = oracle.ppm_cell(q)
        assert abs(aL - (a - 0.5 * s)) <= 1e-14 * (1 + abs(a) + abs(s))
        assert abs(aR - (a + 0.5 * s)) <= 1e-14 * (1 + abs(a) + abs(s))


def test_ppm_interface_value_fourth_order_on_cubics():
    """The unlimited interface value equals the point value of the cubic whose
    cell averages are the data (fourth-order formula of Section 2.2.1).  A
    monotone cubic with small curvature keeps every limiter inactive."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        c0, c1 = rng.normal(), 1.0 + rng.uniform()
        c2, c3 = 0.02 * rng.normal(), 0.01 * rng.normal()
        poly = lambda x: c0 + c1 * x + c2 * x * x + c3 * x ** 3
        prim = lambda x: c0 * x + c1 * x * x / 2 + c2 * x ** 3 / 3 + c3 * x ** 4 / 4
        q = np.array([prim(j + 0.5) - prim(j - 0.5) for j in range(-2, 3)])
        aL, aR = oracle.ppm_cell(q)
        assert abs(aR - poly(0.5)) < 1e-13 and abs(aL - poly(-0.5)) < 1e-13


def test_ppm_extremum_of_cell_averages_is_flat():
    """At a local extremum of the cell averages the linear fallback has zero
    monotonized-central slope, so both interface states equal the average."""
    assert oracle.ppm_cell([0.0, 1.0, 2.0, 1.0, 0.0]) == (2.0, 2.0)
    assert oracle.ppm_cell([3.0, 1.0, -1.0, 1.0, 3.0]) == (-1.0, -1.0)


def test_ppm_extremum_inside_cell_uses_mc_slope():
    """Monotone averages whose interface values make the parabola turn inside the
    cell: linear profile with the MC slope min(2|dr|, 2|dl|, |dc|/2)."""
    aL, aR = oracle.ppm_cell([0.0, 0.0, 1.0, 1.01, 5.0])
    assert abs(aL - 0.99) < 1e-15 and abs(aR - 1.01) < 1e-15


def test_ppm_profiles_are_monotone_and_conservative():
    """Properties of the CW84 construction on random data: the parabola through
    (aL, aR) with mean q0 is monotone inside the cell (|a6| <= |aR - aL|) and the
    interface states bracket q0 unless the profile is flat."""
    rng = np.random.default_rng(2)
    for _ in range(5000):
        q = rng.normal(size=5) * rng.choice([1e-3, 1.0, 1e3])
        aL, aR = oracle.ppm_cell(q)
        q0 = q[2]
        d = aR - aL
        a6 = 6.0 * (q0 - 0.5 * (aL + aR))
        assert abs(a6) <= abs(d) * (1 + 1e-12) + 1e-12 * abs(q0)
        assert (aL - q0) * (aR - q0) <= 1e-24 * max(1.0, q0 * q0)


# ------------------------------------------------------------------ HLLC
def rand_state(rng, g):
    return np.array([rng.uniform(0.1, 3), rng.normal(), rng.normal(), rng.normal(), rng.uniform(0.1, 3)])


def phys_flux(W, g):
    r, u, v, w, p = W
    E = p / (g - 1) + 0.5 * r * (u * u + v * v + w * w)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])


def test_hllc_consistency():
    g = 1.4
    rng = np.random.default_rng(3)
    for _ in range(500):
        W = rand_state(rng, g)
        F = oracle.hllc(W, W, g)
        assert np.allclose(F, phys_flux(W, g), rtol=1e-13, atol=1e-13)


def test_hllc_supersonic_upwinding():
    g = 1.4
    WL = np.array([1.0, 5.0, 0.2, -0.1, 1.0])
    WR = np.array([0.5, 4.0, 0.0, 0.3, 0.8])
    assert np.array_equal(oracle.hllc(WL, WR, g), phys_flux(WL, g))
    WL2 = WL * np.array([1, -1, 1, 1, 1])
    WR2 = WR * np.array([1, -1, 1, 1, 1])
    assert np.array_equal(oracle.hllc(WR2, WL2, g), phys_flux(WL2, g))


def test_hllc_mirror_symmetry():
    """Reflecting x -> -x (swap sides, flip normal velocity) flips the mass and
    energy fluxes and keeps the normal-momentum flux."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(4)
    m = np.array([1, -1, 1, 1, 1])
    for _ in range(500):
        WL, WR = rand_state(rng, g), rand_state(rng, g)
        F = oracle.hllc(WL, WR, g)
        Fm = oracle.hllc(WR * m, WL * m, g)
        assert np.allclose(F * np.array([-1, 1, -1, -1, -1]), Fm, rtol=1e-12, atol=1e-12)


def test_hllc_resolves_contacts_exactly():
    """HLLC resolves isolated contacts (Section 3.1.2): stationary gives (0, p, 0,
    0, 0) exactly; a moving contact gives the upwind physical flux."""
    g = 1.4
    F = oracle.hllc([1.4, 0, 0, 0, 1.0], [1.0, 0, 0, 0, 1.0], g)
    assert np.array_equal(F, np.array([0.0, 1.0, 0.0, 0.0, 0.0]))
    WL, WR = np.array([1.0, 0.3, 0.1, 0.0, 1.0]), np.array([0.4, 0.3, -0.2, 0.5, 1.0])
    F = oracle.hllc(WL, WR, g)
    assert np.allclose(F, phys_flux(WL, g), rtol=1e-14, atol=1e-14)


def test_hllc_close_to_godunov_flux_for_weak_waves():
    """For small jumps the PVRS-based HLLC flux agrees with the exact Godunov flux
    to second order in the jump amplitude."""
    g = 1.4
    rng = np.random.default_rng(5)
    for _ in range(50):
        W0 = np.array([1.0, rng.uniform(-0.3, 0.3), 0.0, 0.0, 1.0])
        for amp in (1e-3, 1e-4):
            d = amp * rng.normal(size=5) * np.array([1, 1, 0, 0, 1])
            WL, WR = W0 - d, W0 + d
            rs, us, ps = er.sample((WL[0], WL[1], WL[4]), (WR[0], WR[1], WR[4]), g, np.array([0.0]))
            Fg = phys_flux(np.array([rs[0], us[0], 0, 0, ps[0]]), g)
            Fh = oracle.hllc(WL, WR, g)
            assert np.max(np.abs(Fh - Fg)) < 50 * amp * amp


# ---------------------------------------------------------------- closure
def test_closure_limits():
    """Section 2.2.2: chi(0) = 1/3 and chi(1) = 1 exactly; tr P = E_r; f = 1 gives
    P = E n n; F = 0 gives P = E/3 I."""
    assert oracle.closure_chi(0.0) == 1.0 / 3.0
    assert oracle.closure_chi(1.0) == 1.0
    c = 10.0
    P = oracle.closure_pressure(2.0, [0.0, 0.0, 0.0], c)
    assert np.allclose(P, 2.0 / 3.0 * np.eye(3), rtol=1e-15)
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    P = oracle.closure_pressure(2.0, c * 2.0 * n, c)
    assert np.allclose(P, 2.0 * np.outer(n, n), atol=1e-15)
    rng = np.random.default_rng(6)
    for _ in range(200):
        F = rng.normal(size=3)
        E = rng.uniform(0.1, 2.0)
        P = oracle.closure_pressure(E, F, c)
        assert abs(np.trace(P) - E) < 1e-14 * E
        assert np.allclose(P, P.T, rtol=0, atol=1e-15)


def test_levermore_chi_matches_boosted_isotropic_field():
    """Levermore's closure is the Eddington factor of radiation that is isotropic
    in a frame moving at speed beta: f = 4 beta/(3 + beta^2) and
    chi = (1 + 3 beta^2)/(3 + beta^2) (moments of a boosted isotropic field)."""
    for beta in np.linspace(0.0, 0.999, 41):
        f = 4 * beta / (3 + beta * beta)
        chi = (1 + 3 * beta * beta) / (3 + beta * beta)
        assert abs(oracle.closure_chi(f) - chi) < 1e-14


def test_eddington_closure_is_isotropic():
    assert oracle.closure_chi(0.7, 1) == 1.0 / 3.0


def _minerbo_max_entropy(f):
    """Minerbo's maximum-entropy Eddington factor from its implicit definition:
    f = coth Z - 1/Z (Langevin function), chi = 1 - 2 f / Z (bisection on Z)."""
    if f < 1e-8:
        return 1.0 / 3.0
    lo, hi = 1e-9, 1e4
    for _ in range(200):
        Z = 0.5 * (lo + hi)
        if 1.0 / np.tanh(Z) - 1.0 / Z < f:
            lo = Z
        else:
            hi = Z
    return 1.0 - 2.0 * f / Z


def test_minerbo_closure():
    """Closure 2 (the Minerbo closure the paper offers beside Levermore's):
    exact limits 1/3 and 1, monotone, and within 0.006 of the maximum-entropy
    closure it approximates."""
    assert oracle.closure_chi(0.0, 2) == 1.0 / 3.0
    assert abs(oracle.closure_chi(1.0, 2) - 1.0) <= 2e-16
    fs = np.linspace(0.0, 0.999, 200)
    chi = np.array([oracle.closure_chi(f, 2) for f in fs])
    assert np.all(np.diff(chi) > 0)
    assert max(abs(c - _minerbo_max_entropy(f)) for f, c in zip(fs, chi)) < 6e-3
    # distinct from Levermore's in between
    assert abs(oracle.closure_chi(0.5, 2) - oracle.closure_chi(0.5, 0)) > 1e-2


# -------------------------------------------------------------- HLL (rad)
def test_hll_free_streaming_is_exact_upwind():
    """F = c E along +x: the Eddington tensor is E x x, both wave speeds are chat,
    and the HLL flux reduces to chat (E_L, c E_L) (free-streaming limit)."""
    p = rad_params(chat=30.0)
    c, ch = p["c"], p["chat"]
    EL, ER = 2.0, 0.5
    f = oracle.hll_rad(EL, [c * EL, 0, 0], ER, [c * ER, 0, 0], 0, p)
    assert np.allclose(f, [ch * EL, c * ch * EL, 0.0, 0.0], rtol=1e-14)


def test_hll_diffusion_limit_speed():
    """F = 0: isotropic tensor, wave speed chat/sqrt(3), flux is the central
    pressure term minus (chat/sqrt 3)/2 times the jump."""
    p = rad_params(chat=30.0)
    c, ch = p["c"], p["chat"]
    EL, ER = 2.0, 0.5
    f = oracle.hll_rad(EL, [0, 0, 0], ER, [0, 0, 0], 1, p)
    S = ch / np.sqrt(3.0)
    assert np.allclose(f, [-0.5 * S * (ER - EL), 0.0, c * ch * (EL + ER) / 6.0, 0.0], rtol=1e-14)


# ------------------------------------------------------------------ PLM
def test_plm_mc_slope():
    """PLM with the monotonized-central limiter (van Leer 1977): exact on lines,
    zero slope at an extremum, slope min(2|dr|, 2|dl|, |dc|/2) otherwise."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        a, s = rng.normal(), rng.normal()
        aL, aR = oracle.plm_cell([a - s, a, a + s])
        assert abs(aL - (a - 0.5 * s)) < 1e-14 * (1 + abs(a) + abs(s))
        assert abs(aR - (a + 0.5 * s)) < 1e-14 * (1 + abs(a) + abs(s))
    assert oracle.plm_cell([0.0, 1.0, 0.5]) == (1.0, 1.0)
    aL, aR = oracle.plm_cell([0.0, 1.0, 1.1])  # dl = 1, dr = 0.1: slope 2 dr = 0.2
    assert abs(aL - 0.9) < 1e-15 and abs(aR - 1.1) < 1e-15
    aL, aR = oracle.plm_cell([0.0, 0.45, 1.0])  # slope |dc|/2 = 0.5
    assert abs(aL - 0.2) < 1e-15 and abs(aR - 0.7) < 1e-15


# ----------------------------------------------------------- shock flattening
def _flat_state(A, ux, B, uy, gamma=1.4, n=12):
    """Box n x n x 1 (z inactive), rho = 1, P(i, j) = A[i] + B[j] - 1,
    velocity (ux[i], uy[j], 0); A, B, ux, uy are dicts over interior indices
    (missing entries: the nearest given value).  Ghost cells are filled."""
    b = inputs.make_box((n, n, 1))
    g = b.ng

    def full(d):
        ks = sorted(d)
        return np.array([d[min(ks, key=lambda k: (abs(k - i), k))] for i in range(-g, n + g)])
    Ai, Bj, ui, vj = full(A), full(B), full(ux), full(uy)
    P = Ai[None, :] + Bj[:, None] - 1.0
    vx = np.broadcast_to(ui[None, :], P.shape)
    vy = np.broadcast_to(vj[:, None], P.shape)
    U = np.zeros((5,) + b.shape)
    U[0] = 1.0
    U[1] = vx[None]
    U[2] = vy[None]
    U[4] = (P / (gamma - 1.0) + 0.5 * (vx * vx + vy * vy))[None]
    oracle.fill_ghosts(b, U)
    return b, U, gamma


# profile with a compression at cell 6 whose jump ratio is z = dp1/dp2 = 0.8
# (CW84 ramp: chi_tilde = 1 - (0.8 - 0.75)/0.1 = 0.5) and whose higher-pressure
# neighbour (cell 7, expanding: du = u8 - u6 > 0) is not a shock
PROF_05 = ({3: 1.0, 4: 1.0, 5: 1.1, 6: 1.5, 7: 1.9, 8: 2.0}, {4: 0.0, 5: 0.1, 6: 0.0, 7: -0.1, 8: 0.2})
# the same with z = 0.82: chi_tilde = 1 - (0.82 - 0.75)/0.1 = 0.3
PROF_03 = ({3: 1.0, 4: 1.0, 5: 1.09, 6: 1.5, 7: 1.91, 8: 2.0}, {4: 0.0, 5: 0.1, 6: 0.0, 7: -0.1, 8: 0.2})
FLAT = ({0: 1.0}, {0: 0.0})


@pytest.mark.parametrize("px,py,want", [(PROF_05, FLAT, 0.5), (FLAT, PROF_03, 0.3), (PROF_05, PROF_03, 0.3),
                                        (PROF_03, PROF_05, 0.3)])
def test_flattening_multidimensional_minimum(px, py, want):
    """Section 2.2.1 flattening (CW84 coefficient, Miller & Colella's
    multidimensional form): at a cell compressed along x with chi_tilde_x =
    0.5 and along y with chi_tilde_y = 0.3 (values evaluated by hand from the
    jump ratios), chi is the minimum over the axes, 0.3, whichever axis
    carries which profile.  Other combinations give other values: the mean
    0.4, the product 0.15, x alone 0.5 or 0.3 depending on the case.  A single
    axis gives its own 1-D value."""
    b, U, gamma = _flat_state(px[0], px[1], py[0], py[1])
    chi = oracle.flatten_chi(b, U, gamma)
    g = b.ng
    assert chi[g, g + 6, g + 6] == pytest.approx(want, abs=1e-12)
    # away from both profiles (and from the compression where the periodic
    # box wraps the profile around, at cells 0 and 11) nothing is flattened
    assert chi[g, g + 3, g + 3] == 1.0


def test_flattening_takes_the_neighbour_toward_higher_pressure():
    """The coefficient of a cell is the minimum of its own chi_tilde and that
    of its neighbour toward the higher pressure.  Here cell 6 itself expands
    (chi_tilde = 1), its high-pressure neighbour 7 has z = 0.8 (chi_tilde =
    0.5) and its low-pressure neighbour 5 has z = 0.7/0.8536585 = 0.82
    (chi_tilde = 0.3): chi(6) = 0.5, while taking both neighbours (or the
    low one) would give 0.3 and taking none 1."""
    A = {3: 1.6 - 0.7 / 0.82, 4: 0.5, 5: 1.0, 6: 1.2, 7: 1.6, 8: 2.0, 9: 2.0}
    u = {3: 0.0, 4: 0.1, 5: -0.1, 6: 0.0, 7: 0.0, 8: -0.1, 9: 0.0}
    b, U, gamma = _flat_state(A, u, *FLAT)
    chi = oracle.flatten_chi(b, U, gamma)
    g = b.ng
    assert chi[g, g + 6, g + 6] == pytest.approx(0.5, abs=1e-12)
    assert chi[g, g + 5, g + 5] == pytest.approx(0.3, abs=1e-9)  # cell 5's own coefficient shows
