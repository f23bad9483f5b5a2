"""Pins of the oracle's hydrodynamics against what the paper and the
mathematics fix (no GPU).  Each test names the passage it checks."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import inputs
from paper_2110_01792_amd.inputs import OUTFLOW, PERIODIC, Box
from tests.oracle_runs import box1d, evolve, line, prim_to_cons, set_line
from tests.refsol import exact_riemann as er

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- P1 contact
def test_stationary_contact_exact_zero():
    """Section 3.1.2: an isolated stationary contact stays exactly unchanged with
    HLLC; the error at t = 2 is exactly zero."""
    gd = gold("contact.json")
    N = 64
    b = box1d(N, bc=OUTFLOW)
    U = np.zeros((5,) + b.shape)
    x = (np.arange(N) + 0.5) / N
    rho = np.where(x < gd["x0"], gd["rhoL"], gd["rhoR"])
    p = np.where(x < gd["x0"], gd["pL"], gd["pR"])
    U0 = prim_to_cons(rho, np.zeros(N), p, gd["gamma"])
    set_line(b, U, U0)
    evolve(b, U, gd["gamma"], 0.3, gd["t_end"])
    assert np.array_equal(line(b, U), U0)


# ------------------------------------------------------------- P2 sound wave
def sound_wave_error(N, gd):
    g = gd["gamma"]
    b = box1d(N)
    x = (np.arange(N) + 0.5) / N
    rho0, P0 = 1.0, 1.0 / g
    U0 = np.array([rho0, 0.0, 0.0, 0.0, P0 / (g - 1.0)])[:, None] * np.ones(N)
    U0 = U0 + gd["amplitude"] * np.array(gd["eigenvector"])[:, None] * np.sin(2 * np.pi * x)[None, :]
    U = np.zeros((5,) + b.shape)
    set_line(b, U, U0)
    evolve(b, U, g, gd["cfl"], gd["t_end"])
    dU = np.abs(line(b, U) - U0).mean(axis=1)  # eq. convergence_error, per component
    # The norm over components: the printed values match the root-sum-square
    # over the five components (the convention of the Athena test the paper
    # follows), not the mean-square root; that reading is used here.
    return float(np.sqrt(np.sum(dU ** 2)))


def test_sound_wave_second_order_and_magnitude():
    """Section 3.1.1: a linear sound wave returns after one period with an error
    norm of 1.0e-7 at N = 16 and 1.6e-9 at N = 128, scaling as N^-2.  The
    paper prints two significant digits; agreement is required to 10 %."""
    gd = gold("sound_wave.json")
    errs = {N: sound_wave_error(N, gd) for N in (16, 32, 64, 128)}
    ref = gd["error_norm"]
    for N in (16, 128):
        assert 0.9 < errs[N] / ref[str(N)] < 1.1, (N, errs[N], ref[str(N)])
    slope = np.log(errs[128] / errs[32]) / np.log(4.0)
    assert -2.3 < slope < -1.7, (errs, slope)


def test_sound_wave_plm_second_order_and_less_accurate_than_ppm():
    """PLM (MC limiter) option of Section 2.2.1: still second order on the sound
    wave, with a larger error than PPM at the same resolution."""
    gd = gold("sound_wave.json")
    g = gd["gamma"]

    def err(N, recon):
        b = box1d(N)
        x = (np.arange(N) + 0.5) / N
        U0 = np.array([1.0, 0.0, 0.0, 0.0, (1.0 / g) / (g - 1.0)])[:, None] * np.ones(N)
        U0 = U0 + gd["amplitude"] * np.array(gd["eigenvector"])[:, None] * np.sin(2 * np.pi * x)[None, :]
        U = np.zeros((5,) + b.shape)
        set_line(b, U, U0)
        t, n = 0.0, 0
        while t < 1.0 * (1 - 1e-14):
            oracle.fill_ghosts(b, U)
            dt = gd["cfl"] * (1.0 / N) / oracle.hydro_max_signal(b, U, g)
            dt = min(dt, 1.0 - t)
            oracle.hydro_step(b, U, g, gd["cfl"], dt, recon=recon)
            t += dt
        return float(np.sqrt(np.sum(np.abs(line(b, U) - U0).mean(axis=1) ** 2)))

    e32, e128 = err(32, 1), err(128, 1)
    slope = np.log(e128 / e32) / np.log(4.0)
    assert -2.4 < slope < -1.6, (e32, e128, slope)
    assert e128 > err(128, 0)


# -------------------------------------------------------- P3 shock capturing
def run_tube(WL, WR, g, N, L, x0, cfl, t_end):
    b = box1d(N, L=L, bc=OUTFLOW)
    x = (np.arange(N) + 0.5) * (L / N)
    left = x < x0
    rho = np.where(left, WL[0], WR[0])
    u = np.where(left, WL[1], WR[1])
    p = np.where(left, WL[2], WR[2])
    U = np.zeros((5,) + b.shape)
    set_line(b, U, prim_to_cons(rho, u, p, g))
    evolve(b, U, g, cfl, t_end)
    re, ue, pe = er.sample(WL, WR, g, (x - x0) / t_end)
    return line(b, U), er.conserved(re, ue, pe, g), x


def rel_rms_l1(Un, Ue):
    l1 = np.abs(Un - Ue).mean(axis=1)
    ln = np.abs(Ue).mean(axis=1)
    keep = [0, 1, 4]  # the transverse momenta are identically zero on both sides
    return float(np.sqrt(np.mean(l1[keep] ** 2)) / np.sqrt(np.mean(ln[keep] ** 2)))


def test_timmes_shock_tube_against_exact_solution():
    """Section 3.1.3: rms L1 error over rms exact is 1.12e-3 at N = 1000 (t = 0.4)."""
    gd = gold("shock_tube.json")
    g = gd["gamma"]
    Un, Ue, _ = run_tube((gd["rhoL"], 0.0, gd["pL"]), (gd["rhoR"], 0.0, gd["pR"]), g, gd["N"], gd["L"], gd["x0"],
                         gd["cfl"], gd["t_end"])
    e = rel_rms_l1(Un, Ue)
    assert 0.9 * gd["rel_rms_L1"] < e < 1.1 * gd["rel_rms_L1"], e


def test_sod_converges_to_exact_solution():
    """Axis-aligned version of the benchmark's planar discontinuity (rho 1/0.125,
    P 1/0.1, gamma 1.4): L1 error against the exact Riemann solution falls
    roughly as 1/N and the shock sits where the exact solution puts it."""
    WL, WR, g = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4
    errs = []
    for N in (100, 200, 400):
        Un, Ue, x = run_tube(WL, WR, g, N, 1.0, 0.5, 0.3, 0.2)
        errs.append(rel_rms_l1(Un, Ue))
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs
    assert errs[2] < 1e-2


@pytest.mark.parametrize("axis", [1, 2])
def test_sod_along_other_axes_matches_x(axis):
    """The same tube along y or z gives the x result bitwise (axis-independence
    of the unsplit scheme)."""
    WL, WR, g = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4
    N = 64
    out = []
    for ax in (0, axis):
        b = box1d(N, bc=OUTFLOW, axis=ax)
        x = (np.arange(N) + 0.5) / N
        left = x < 0.5
        U0 = prim_to_cons(np.where(left, 1.0, 0.125), np.zeros(N), np.where(left, 1.0, 0.1), g)
        if ax != 0:
            U0[[1, 1 + ax]] = U0[[1 + ax, 1]]
        U = np.zeros((5,) + b.shape)
        set_line(b, U, U0, axis=ax)
        for _ in range(10):
            oracle.hydro_step(b, U, g, 0.3, 1e-3)
        r = line(b, U, axis=ax).copy()
        if ax != 0:
            r[[1, 1 + ax]] = r[[1 + ax, 1]]
        out.append(r)
    assert np.array_equal(out[0], out[1])


def test_123_rarefaction_stable_and_close_to_exact():
    """Section 3.1.6 (Einfeldt 1-2-3 problem): stable, positive, and the density
    close to the exact solution except near the centre."""
    gd = gold("rarefaction_123.json")
    g = gd["gamma"]
    p = (g - 1.0) * (gd["E"] - 0.5 * gd["mom"] ** 2 / gd["rho"])
    WL, WR = (gd["rho"], -gd["mom"] / gd["rho"], p), (gd["rho"], gd["mom"] / gd["rho"], p)
    Un, Ue, x = run_tube(WL, WR, g, gd["N"], gd["L"], gd["x0"], gd["cfl"], gd["t_end"])
    assert np.all(Un[0] > 0.0)
    ekin = 0.5 * Un[1] ** 2 / Un[0]
    assert np.all(Un[4] - ekin > 0.0)
    far = np.abs(x - 0.5) > 0.1
    assert np.mean(np.abs(Un[0][far] - Ue[0][far])) < 0.03
    assert 0.5 * Ue[0].min() < Un[0].min() < 2.0 * Ue[0].min()


# ------------------------------------------------ P4-P7 invariants (3D box)
def test_conservation_periodic():
    """Flux form (Section 2.2.1): on a periodic box the sums of mass, momentum
    and energy change only by round-off over 10 steps of the 32^3 workload."""
    b, U, p = inputs.hydro_smooth()
    oracle.fill_ghosts(b, U)
    s0 = U[b.interior()].sum(axis=(1, 2, 3))
    a0 = np.abs(U[b.interior()]).sum(axis=(1, 2, 3))
    for _ in range(10):
        oracle.hydro_step(b, U, p["gamma"], p["cfl"])
    s1 = U[b.interior()].sum(axis=(1, 2, 3))
    assert np.all(np.abs(s1 - s0) / a0 < 1e-13), (s1 - s0) / a0


def test_uniform_state_unchanged_bitwise():
    b = inputs.make_box(12)
    U = np.zeros((5,) + b.shape)
    U[b.interior()] = np.array([1.3, 0.2, -0.1, 0.05, 2.7])[:, None, None, None]
    U0 = U.copy()
    for _ in range(3):
        oracle.hydro_step(b, U, 1.4, 0.3)
    assert np.array_equal(U[b.interior()], U0[b.interior()])


def test_periodic_shift_equivariance_bitwise():
    b, U, p = inputs.hydro_smooth(n=16)
    V = U.copy()
    Vi = np.roll(U[b.interior()], shift=(3, -5, 7), axis=(1, 2, 3))
    V[b.interior()] = Vi
    for _ in range(2):
        oracle.hydro_step(b, U, p["gamma"], p["cfl"], 1e-2)
        oracle.hydro_step(b, V, p["gamma"], p["cfl"], 1e-2)
    assert np.array_equal(np.roll(U[b.interior()], shift=(3, -5, 7), axis=(1, 2, 3)), V[b.interior()])


def test_xy_swap_symmetry_bitwise():
    """Section 3.1.8 (implosion): x and y fluxes are summed symmetrically so that
    swapping the x and y axes of the input swaps the output bitwise."""
    b, U, p = inputs.hydro_shock(n=24)
    V = np.ascontiguousarray(np.swapaxes(U, 2, 3)[[0, 2, 1, 3, 4]])
    for _ in range(3):
        oracle.hydro_step(b, U, p["gamma"], p["cfl"], 2e-3)
        oracle.hydro_step(b, V, p["gamma"], p["cfl"], 2e-3)
    W = np.swapaxes(V, 2, 3)[[0, 2, 1, 3, 4]]
    assert np.array_equal(U[b.interior()], W[b.interior()])


def test_cyclic_axis_permutation_round_off():
    """A cyclic x->y->z relabelling gives the same result to round-off (the sum
    ((x + y) + z) is not invariant under it bitwise)."""
    b, U, p = inputs.hydro_shock(n=20)
    # new axes: (x', y', z') = (y, z, x) => array axes (z,y,x) -> (x,z,y)
    V = np.ascontiguousarray(np.transpose(U, (0, 3, 1, 2))[[0, 2, 3, 1, 4]])
    for _ in range(2):
        oracle.hydro_step(b, U, p["gamma"], p["cfl"], 2e-3)
        oracle.hydro_step(b, V, p["gamma"], p["cfl"], 2e-3)
    W = np.transpose(V, (0, 2, 3, 1))[[0, 3, 1, 2, 4]]
    d = np.abs(U[b.interior()] - W[b.interior()]).max(axis=(1, 2, 3))
    s = np.abs(U[b.interior()]).max(axis=(1, 2, 3))
    assert np.all(d <= 1e-13 * s), d / s


def test_cfl_timestep_definition():
    """Section 2.2.1: dt = CFL * dx / max(|v| + c_s), with |v| the vector magnitude."""
    b = inputs.make_box(8)
    U = np.zeros((5,) + b.shape)
    g = 1.4
    rho, v, P = 2.0, np.array([0.3, -0.4, 1.2]), 0.5
    U[b.interior()] = np.array([rho, rho * v[0], rho * v[1], rho * v[2],
                                P / (g - 1) + 0.5 * rho * v.dot(v)])[:, None, None, None]
    s = oracle.hydro_max_signal(b, U, g)
    assert abs(s - (1.3 + np.sqrt(g * P / rho))) < 1e-14
    st = oracle.hydro_step(b, U, g, 0.3)
    assert abs(st["dt"] - 0.3 * (1 / 8) / s) < 1e-16


def test_outflow_and_periodic_ghosts():
    """Boundary fill: periodic wraps, outflow copies the nearest interior cell,
    fixed leaves ghosts untouched; corners follow the axis-by-axis fill."""
    b = Box((5, 4, 3), 4, (1.0, 1.0, 1.0), ((PERIODIC, PERIODIC), (OUTFLOW, OUTFLOW), (2, 2)))
    U = np.full((1,) + b.shape, -7.0)
    rng = np.random.default_rng(0)
    U[b.interior()] = rng.normal(size=(1, 3, 4, 5))
    oracle.fill_ghosts(b, U)
    g = 4
    for k in range(3):
        for j in range(-4, 8):
            for i in range(-4, 9):
                jj = min(max(j, 0), 3)
                ii = i % 5
                assert U[0, k + g, j + g, i + g] == U[0, k + g, jj + g, ii + g]
    assert np.all(U[0, :g] == -7.0) and np.all(U[0, g + 3:] == -7.0)
