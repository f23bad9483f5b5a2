"""Seeded synthetic inputs for the per-cell update (shared by the GPU path's
tests and benchmark and by the oracle's tests).

This module holds workload recipes only: grid geometry, seeded random fields
and the initial-condition definitions (ideal-gas energy E = P/(gamma-1) +
rho v^2/2, E_r = a_r T_r^4).  It contains none of the update's arithmetic and
imports neither the GPU binding nor the oracle.

Every array is float64, C-contiguous, shape (nvar, nz+2ng, ny+2ng, nx+2ng),
x fastest.  Ghost cells are left at zero unless a recipe defines them (the
batched level, whose ghosts are fixed data); the path under test fills them.

Draw order is fixed per recipe and documented in each function, so a seed
fixes the input exactly.
"""
from __future__ import annotations

from typing import NamedTuple, Optional, Sequence, Tuple

import numpy as np

# FIXED_FREE_FLUX: Dirichlet ghosts except the radiation flux of a radiation
# state, which is zero-gradient (see rad_pressure_tube)
PERIODIC, OUTFLOW, FIXED, FIXED_FREE_FLUX = 0, 1, 2, 3


class Box(NamedTuple):
    n: Tuple[int, int, int]
    ng: int
    dx: Tuple[float, float, float]
    bc: Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, int]]
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def shape(self):
        return (self.n[2] + 2 * self.ng, self.n[1] + 2 * self.ng, self.n[0] + 2 * self.ng)

    def interior(self):
        g = self.ng
        return (slice(None), slice(g, g + self.n[2]), slice(g, g + self.n[1]), slice(g, g + self.n[0]))

    @property
    def ncells(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def make_box(n, ng=4, L=1.0, bc=PERIODIC, origin=(0.0, 0.0, 0.0)) -> Box:
    if isinstance(n, int):
        n = (n, n, n)
    if isinstance(L, (int, float)):
        L = (float(L),) * 3
    if isinstance(bc, int):
        bc = ((bc, bc),) * 3
    dx = tuple(float(L[d]) / n[d] for d in range(3))
    return Box(tuple(int(v) for v in n), int(ng), dx, tuple(tuple(int(v) for v in p) for p in bc),
               tuple(float(o) for o in origin))


def cell_centres(b: Box, with_ghosts: bool = False):
    """Cell-centre coordinates (z, y, x broadcastable), x_i = origin + (i + 1/2) dx."""
    out = []
    for d in (2, 1, 0):
        if with_ghosts:
            idx = np.arange(-b.ng, b.n[d] + b.ng, dtype=np.float64)
        else:
            idx = np.arange(b.n[d], dtype=np.float64)
        out.append(b.origin[d] + (idx + 0.5) * b.dx[d])
    z, y, x = out
    return z[:, None, None], y[None, :, None], x[None, None, :]


def _conserved(rho, vx, vy, vz, P, gamma):
    E = P / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, E])


def _modes(rng, nmodes=4):
    """Wave vectors drawn uniformly from {-2..2}^3 without 0, then phases in [0, 2 pi)."""
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-2, 3, size=3)
        if np.any(k != 0):
            ks.append(k)
    phis = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    return np.array(ks, dtype=np.float64), phis


def _mode_sum(ks, phis, z, y, x):
    s = 0.0
    for k, ph in zip(ks, phis):
        s = s + np.sin(2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
    return s


def _alloc(b: Box, nvar: int):
    return np.zeros((nvar,) + b.shape, dtype=np.float64)


# ---------------------------------------------------------------------------
# Plain hydro, 32^3 periodic, gamma 5/3 (smooth density, random velocities).
# Draws: 4 wave vectors + 4 phases, then vx, vy, vz per cell U[-0.1, 0.1].
# ---------------------------------------------------------------------------
def hydro_smooth(n=32, seed=1, gamma=5.0 / 3.0, ng=4):
    b = make_box(n, ng=ng, bc=PERIODIC)
    rng = np.random.default_rng(seed)
    ks, phis = _modes(rng)
    z, y, x = cell_centres(b)
    rho = 1.0 + 0.1 * _mode_sum(ks, phis, z, y, x) * np.ones((b.n[2], b.n[1], b.n[0]))
    v = rng.uniform(-0.1, 0.1, size=(3, b.n[2], b.n[1], b.n[0]))
    P = np.ones_like(rho)
    U = _alloc(b, 5)
    U[b.interior()] = _conserved(rho, v[0], v[1], v[2], P, gamma)
    return b, U, {"gamma": gamma, "cfl": 0.3}


# ---------------------------------------------------------------------------
# Plain hydro, one box n^3 (256 by default) with outflow boundaries, gamma 1.4:
# planar discontinuity of seeded orientation through the centre
# (rho 1 / 0.125, P 1 / 0.1, v = 0), density times (1 + 0.01 xi), xi U[-1,1].
# Draws: normal = 3 standard normals (normalised), then xi per cell.
# ---------------------------------------------------------------------------
def hydro_shock(n=256, seed=2, gamma=1.4, ng=4):
    b = make_box(n, ng=ng, bc=OUTFLOW)
    rng = np.random.default_rng(seed)
    nh = rng.normal(size=3)
    nh = nh / np.sqrt(np.sum(nh * nh))
    xi = rng.uniform(-1.0, 1.0, size=(b.n[2], b.n[1], b.n[0]))
    z, y, x = cell_centres(b)
    s = nh[0] * (x - 0.5) + nh[1] * (y - 0.5) + nh[2] * (z - 0.5)
    left = s < 0.0
    rho = np.where(left, 1.0, 0.125) * (1.0 + 0.01 * xi)
    P = np.where(left, 1.0, 0.1) * np.ones_like(rho)
    zero = np.zeros_like(rho)
    U = _alloc(b, 5)
    U[b.interior()] = _conserved(rho, zero, zero, zero, P, gamma)
    return b, U, {"gamma": gamma, "cfl": 0.3, "normal": nh}


# ---------------------------------------------------------------------------
# Sedov-Taylor blast in [-1, 1]^3, periodic, rho 1, P 10 inside r < 0.1 else
# 0.1, v = 0, gamma 5/3, CFL 0.25 (the paper's hydro performance workload).
# No random draws.
# ---------------------------------------------------------------------------
def sedov(n=256, gamma=5.0 / 3.0, ng=4):
    b = make_box(n, ng=ng, L=2.0, bc=PERIODIC, origin=(-1.0, -1.0, -1.0))
    z, y, x = cell_centres(b)
    r2 = x * x + y * y + z * z
    P = np.where(r2 < 0.01, 10.0, 0.1) * np.ones((b.n[2], b.n[1], b.n[0]))
    rho = np.ones_like(P)
    zero = np.zeros_like(P)
    U = _alloc(b, 5)
    U[b.interior()] = _conserved(rho, zero, zero, zero, P, gamma)
    return b, U, {"gamma": gamma, "cfl": 0.25}


# ---------------------------------------------------------------------------
# Radiation hydrodynamics, n^3 periodic, dimensionless units (P = rho T,
# a_r = 1, c = 1000, gamma 5/3), constant grey opacity 1.
# rho = exp(0.5 xi - 0.125), xi ~ N(0,1); T_gas, T_rad ~ U[0.5, 2] independent;
# v = 0; E = rho T/(gamma-1); E_r = a_r T_rad^4; F = 0;
# chat = 10 x max over cells of sqrt(gamma T).
# Draws: xi per cell, then T_gas per cell, then T_rad per cell.
# ---------------------------------------------------------------------------
def rad_params(chat, gamma=5.0 / 3.0, **kw):
    p = {"c": 1000.0, "chat": float(chat), "a_r": 1.0, "kappa_P": 1.0, "kappa_R": 1.0, "gamma": gamma,
         "alpha_cv": 4.0, "cfl": 0.3, "newton_tol": 1e-12, "newton_max_iter": 400, "nsub_max": 10,
         "closure": 0, "tau_correction": 1, "eos": 0, "recon": 0}
    p.update(kw)
    return p


def rhd_lognormal(n=128, seed=3, gamma=5.0 / 3.0, ng=4):
    b = make_box(n, ng=ng, bc=PERIODIC)
    rng = np.random.default_rng(seed)
    shape = (b.n[2], b.n[1], b.n[0])
    xi = rng.normal(size=shape)
    rho = np.exp(0.5 * xi - 0.125)
    Tg = rng.uniform(0.5, 2.0, size=shape)
    Tr = rng.uniform(0.5, 2.0, size=shape)
    a_r = 1.0
    zero = np.zeros(shape)
    Ug = _alloc(b, 5)
    Ug[b.interior()] = _conserved(rho, zero, zero, zero, rho * Tg, gamma)
    Ur = _alloc(b, 4)
    Ur[(0,) + b.interior()[1:]] = a_r * Tr ** 4
    chat = 10.0 * float(np.sqrt(gamma * Tg.max()))
    return b, Ug, Ur, rad_params(chat, gamma)


# ---------------------------------------------------------------------------
# Batched AMR-like level: nbox boxes, each axis edge i.i.d. from
# {8,16,24,32,48,64}, dx = 1/256, origin U[0,1)^3, RHD with probability 1/2.
# Interior and the 4 ghost layers are filled from smooth seeded fields:
# rho = 1 + 0.1 s1, P = 1 + 0.05 s2, v_d = 0.05 s_{3+d}; RHD boxes also get
# T_r = (P/rho)(1 + 0.05 s6), E_r = a_r T_r^4, F = 0 (s_i = sum of 4 modes).
# Ghosts are fixed data (the boundary kind of every face is FIXED).
# Draws: 6 mode sets, then per box: 3 edges, 3 origin coordinates, 1 type draw.
# ---------------------------------------------------------------------------
EDGES = (8, 16, 24, 32, 48, 64)


def batch_level(nbox=600, seed=5, gamma=5.0 / 3.0, ng=4, edges: Optional[Sequence[int]] = None,
                rad_fraction=0.5):
    rng = np.random.default_rng(seed)
    modes = [_modes(rng) for _ in range(6)]
    edges = EDGES if edges is None else tuple(edges)
    boxes, Ugs, Urs = [], [], []
    dx = 1.0 / 256.0
    cmax = 0.0
    for _ in range(nbox):
        n = tuple(int(edges[i]) for i in rng.integers(0, len(edges), size=3))
        origin = tuple(float(o) for o in rng.uniform(0.0, 1.0, size=3))
        is_rad = bool(rng.uniform() < rad_fraction)
        b = Box(n, ng, (dx, dx, dx), ((FIXED, FIXED),) * 3, origin)
        z, y, x = cell_centres(b, with_ghosts=True)
        full = np.ones(b.shape)
        s = [_mode_sum(k, p, z, y, x) * full for (k, p) in modes]
        rho = 1.0 + 0.1 * s[0]
        P = 1.0 + 0.05 * s[1]
        vx, vy, vz = 0.05 * s[2], 0.05 * s[3], 0.05 * s[4]
        Ug = np.ascontiguousarray(_conserved(rho, vx, vy, vz, P, gamma))
        Ur = None
        if is_rad:
            T = P / rho
            Tr = T * (1.0 + 0.05 * s[5])
            Ur = np.zeros((4,) + b.shape)
            Ur[0] = Tr ** 4
            cmax = max(cmax, float(np.sqrt(gamma * T.max())))
        boxes.append(b)
        Ugs.append(Ug)
        Urs.append(Ur)
    chat = 10.0 * cmax if cmax > 0 else 10.0
    return boxes, Ugs, Urs, rad_params(chat, gamma), {"gamma": gamma, "cfl": 0.3}


# ---------------------------------------------------------------------------
# Radiation pressure tube (Section 3.3.1; Krumholz et al. 2007): a 1-D column
# [0, 128] cm, 128 cells, in which radiation and gas pressure gradients balance
# in the equilibrium-diffusion regime (tau_cell ~ 100).  cgs, mu = 2.33 m_H,
# gamma 5/3, kappa_P = kappa_R = 100, T_0 = 2.75e7 K, rho_0 = 1,
# drho/dx(0) = 0.005; chat = 10 c_s(0).  Dirichlet ends hold what the ODE
# solution fixes (rho, v = 0, T and so E_gas and E_r = a_r T^4); the radiation
# flux in the ghost cells is not given by it and is extrapolated with zero
# gradient (boundary kind FIXED_FREE_FLUX).
#
# The update's EOS is P = rho T, so temperature is carried as T' = k_B T / mu
# (erg/g) with a_r' = a_r (mu / k_B)^4, which leaves a_r T^4 and P unchanged.
# The steady state solves the two ODEs the paper gives (hydrostatic total
# pressure, and constant diffusive flux F = -(c / (3 rho kappa_R)) dE_r/dx),
# integrated with classical RK4 from x = 0 in both directions; cell values are
# point values at cell centres, the ghosts included.  No random draws.
# ---------------------------------------------------------------------------
CGS = {"a_r": 7.5657e-15, "c": 2.99792458e10, "k_B": 1.380649e-16, "m_H": 1.6735575e-24}


def _tube_rhs(y, a_r):
    rho, T, dT = y
    drho = -(rho + (4.0 / 3.0) * a_r * T ** 3) * dT / T
    d2T = -3.0 * dT * dT / T + drho * dT / rho
    return np.array([drho, dT, d2T])


def _rk4_to(y, x0, x1, a_r, h=1e-3):
    n = max(1, int(np.ceil(abs(x1 - x0) / h)))
    hh = (x1 - x0) / n
    for _ in range(n):
        k1 = _tube_rhs(y, a_r)
        k2 = _tube_rhs(y + 0.5 * hh * k1, a_r)
        k3 = _tube_rhs(y + 0.5 * hh * k2, a_r)
        k4 = _tube_rhs(y + hh * k3, a_r)
        y = y + (hh / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def rad_pressure_tube(n=128, ng=4, L=128.0):
    mu = 2.33 * CGS["m_H"]
    kB_mu = CGS["k_B"] / mu
    a_r = CGS["a_r"] / kB_mu ** 4
    gamma, kappa = 5.0 / 3.0, 100.0
    T0, rho0, drho0 = 2.75e7 * kB_mu, 1.0, 0.005
    dT0 = -drho0 * T0 / (rho0 + (4.0 / 3.0) * a_r * T0 ** 3)
    dx = L / n
    b = Box((n, 1, 1), ng, (dx, dx, dx), ((FIXED_FREE_FLUX, FIXED_FREE_FLUX), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    xs = (np.arange(-ng, n + ng) + 0.5) * dx
    prof = np.zeros((len(xs), 3))
    y0 = np.array([rho0, T0, dT0])
    order = np.argsort(np.abs(xs))  # march outwards from x = 0 on each side
    for side in (xs < 0, xs >= 0):
        idx = [i for i in order if side[i]]
        y, x = y0.copy(), 0.0
        for i in idx:
            y = _rk4_to(y, x, xs[i], a_r)
            x = xs[i]
            prof[i] = y
    rho, T, dT = prof[:, 0], prof[:, 1], prof[:, 2]
    Er = a_r * T ** 4
    F = -(CGS["c"] / (3.0 * rho * kappa)) * 4.0 * a_r * T ** 3 * dT
    Ug = np.zeros((5,) + b.shape)
    Ur = np.zeros((4,) + b.shape)
    Ug[0] = rho[None, None, :]
    Ug[4] = (rho * T / (gamma - 1.0))[None, None, :]
    Ur[0] = Er[None, None, :]
    Ur[1] = F[None, None, :]
    cs0 = np.sqrt(gamma * T0)
    p = rad_params(10.0 * cs0, gamma=gamma, c=CGS["c"], a_r=a_r, kappa_P=kappa, kappa_R=kappa, cfl=0.4,
                   newton_tol=1e-12, tau_correction=1)
    return b, Ug, Ur, p, {"T": T, "rho": rho, "t_end": L / cs0, "cfl": 0.4, "cs0": cs0}


# ---------------------------------------------------------------------------
# Streaming radiation entering an optically thick slab (Section 2.2.2: the
# optical-depth correction can give |F| > c E_r where a streaming flux meets
# a discontinuity between optically thin and thick cells).  Box n (x outflow,
# y and z periodic), [0,1] along x, cubic cells; dimensionless units (c =
# 1000, chat = 100, a_r = 1, kappa_R = 1 and kappa_P = 0 (a purely scattering
# slab keeps its low E_r), gamma 5/3, P = rho T).
# Thin cells (x below the interface) have rho dx = tau_thin, E_r = 1 and a
# beam F = f_beam c E_r along a direction tilted in x-y by a seeded angle in
# [-0.2, 0.2] rad; thick cells have rho dx = tau_thick, E_r = e_thick, F = 0.
# The interface is x = 1/2 + 0.1 sin(2 pi (y + phi_y)) sin(2 pi (z + phi_z))
# with seeded phases (so y and z faces also join thin and thick cells); v = 0
# and the gas pressure uniform (T = 1 in thin cells, tau_thin/tau_thick in
# thick ones).  Draws: angle, phi_y, phi_z.
# ---------------------------------------------------------------------------
def rad_thick_streaming(n=(32, 1, 1), seed=9, tau_thin=0.01, tau_thick=100.0, e_thick=1e-3, f_beam=0.99, ng=4):
    if isinstance(n, int):
        n = (n, n, n)
    dx = 1.0 / n[0]
    b = Box(tuple(int(v) for v in n), ng, (dx, dx, dx), ((OUTFLOW, OUTFLOW), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    rng = np.random.default_rng(seed)
    ang = rng.uniform(-0.2, 0.2)
    phy, phz = rng.uniform(0.0, 1.0, 2)
    z, y, x = cell_centres(b, with_ghosts=True)
    xs = 0.5 + 0.1 * np.sin(2 * np.pi * (y + phy)) * np.sin(2 * np.pi * (z + phz))
    thick = np.broadcast_to(x >= xs, b.shape)
    p = rad_params(100.0, c=1000.0, kappa_P=0.0, kappa_R=1.0, cfl=0.3)
    gamma = p["gamma"]
    rho = np.where(thick, tau_thick, tau_thin) / (p["kappa_R"] * dx)
    E = np.where(thick, e_thick, 1.0)
    F = np.where(thick, 0.0, f_beam * p["c"] * E)
    Ug = _alloc(b, 5)
    Ur = _alloc(b, 4)
    Ug[0] = rho
    Ug[4] = rho * np.where(thick, tau_thin / tau_thick, 1.0) / (gamma - 1.0)
    Ur[0] = E
    Ur[1] = F * np.cos(ang)
    Ur[2] = F * np.sin(ang)
    return b, Ug, Ur, p


def to_f32_and_back(U):
    """FP32-rounded copy promoted exactly back to float64 (mixed-precision reference start)."""
    return U.astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Two AMR levels (refinement ratio 2) for the level-synchronisation tests: a
# periodic coarse box of n^3 cells on [0,1]^3 and one fine box of m^3 fine
# cells whose lowest cell lies in coarse cell `off` (fine ghosts are FIXED:
# the caller fills them from the coarse level).  Both levels hold point
# values of the same smooth seeded field at their cell centres:
# rho = 1 + 0.2 s1, P = 1 + 0.1 s2, v_d = 0.2 s_{3+d} (s_i = sum of 4 modes),
# gamma 5/3.  Draws: 5 mode sets.
# ---------------------------------------------------------------------------
def two_level(n=16, m=16, off=(4, 4, 4), seed=61, gamma=5.0 / 3.0, ng=4, rad=False):
    """With rad=True also radiation states on both levels (E_r = (1 + 0.2 s6)^4,
    F = 0.2 c E_r (s7, s8, s9) / 4 with c = 1000; two more draws of 4 mode sets)
    and radiation parameters (chat 50, kappa 0: transport only) are returned."""
    rng = np.random.default_rng(seed)
    modes = [_modes(rng) for _ in range(5)]
    rmodes = [_modes(rng) for _ in range(4)] if rad else []
    cb = make_box(n, ng=ng, bc=PERIODIC)
    dxf = cb.dx[0] / 2.0
    fo = tuple(off[d] * cb.dx[d] for d in range(3))
    fb = Box((m, m, m), ng, (dxf, dxf, dxf), ((FIXED, FIXED),) * 3, fo)

    def fill(b):
        z, y, x = cell_centres(b)
        full = np.ones((b.n[2], b.n[1], b.n[0]))
        s = [_mode_sum(k, p, z, y, x) * full for (k, p) in modes]
        U = _alloc(b, 5)
        U[b.interior()] = _conserved(1.0 + 0.2 * s[0], 0.2 * s[2], 0.2 * s[3], 0.2 * s[4], 1.0 + 0.1 * s[1], gamma)
        return U

    def fill_rad(b, c):
        z, y, x = cell_centres(b)
        full = np.ones((b.n[2], b.n[1], b.n[0]))
        s = [_mode_sum(k, p, z, y, x) * full for (k, p) in rmodes]
        E = (1.0 + 0.2 * s[0]) ** 4
        U = _alloc(b, 4)
        I = b.interior()
        U[(0,) + I[1:]] = E
        for d in range(3):
            U[(1 + d,) + I[1:]] = 0.2 * c * E * s[1 + d] / 4.0
        return U

    hp = {"gamma": gamma, "cfl": 0.3}
    if not rad:
        return cb, fill(cb), fb, fill(fb), tuple(off), hp
    p = rad_params(50.0, gamma=gamma, kappa_P=0.0, kappa_R=0.0)
    return (cb, fill(cb), fill_rad(cb, p["c"]), fb, fill(fb), fill_rad(fb, p["c"]), tuple(off), hp, p)
