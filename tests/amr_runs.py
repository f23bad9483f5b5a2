"""Two-level (refinement ratio 2) step sequencing shared by the oracle and
GPU level-synchronisation tests.  `A` supplies fill_ghosts, max_signal,
hydro_step_reg, prolong, average_down and reflux with the oracle's
signatures; this module only calls them in order (Section 2.2: coarse step, two
fine steps with ghosts interpolated in space and time from the coarse level,
average-down, reflux)."""
import numpy as np


def region_size(lo, hi, nvar=5):
    m = [hi[d] - lo[d] for d in range(3)]
    return nvar * 2 * (m[1] * m[2] + m[0] * m[2] + m[0] * m[1])


def two_level_step(A, cb, Uc, fb, Uf, off, gamma, cfl, reflux=True):
    lo = tuple(off)
    hi = tuple(off[d] + fb.n[d] // 2 for d in range(3))
    A.fill_ghosts(cb, Uc)
    A.prolong(cb, Uc, Uc, 0.0, fb, Uf, off)  # fine ghosts at the old time, for the fine CFL limit
    dt = min(cfl * min(cb.dx) / A.max_signal(cb, Uc, gamma), 2.0 * cfl * min(fb.dx) / A.max_signal(fb, Uf, gamma))
    Uc_old = A.copy(Uc)
    reg_c = A.zeros(region_size(lo, hi))
    A.hydro_step_reg(cb, Uc, gamma, cfl, dt, lo, hi, reg_c)
    reg_f = A.zeros(region_size((0, 0, 0), fb.n))
    for alpha in (0.0, 0.5):
        A.prolong(cb, Uc_old, Uc, alpha, fb, Uf, off)
        A.hydro_step_reg(fb, Uf, gamma, cfl, 0.5 * dt, (0, 0, 0), fb.n, reg_f)
    A.average_down(fb, Uf, cb, Uc, off)
    if reflux:
        A.reflux(cb, Uc, lo, hi, reg_c, fb, reg_f)
    return dt, reg_c, reg_f


def composite_totals(cb, Uc, fb, Uf, off):
    """Sum of U x cell volume over the coarse cells outside the fine footprint
    and the fine cells (per variable)."""
    g = cb.ng
    I = cb.interior()
    vc = cb.dx[0] * cb.dx[1] * cb.dx[2]
    mask = np.ones((cb.n[2], cb.n[1], cb.n[0]), dtype=bool)
    mask[off[2]:off[2] + fb.n[2] // 2, off[1]:off[1] + fb.n[1] // 2, off[0]:off[0] + fb.n[0] // 2] = False
    tc = (Uc[I] * mask).reshape(5, -1).sum(axis=1) * vc
    tf = Uf[fb.interior()].reshape(5, -1).sum(axis=1) * (fb.dx[0] * fb.dx[1] * fb.dx[2])
    return tc + tf


def coarse_totals(cb, Uc):
    return Uc[cb.interior()].reshape(5, -1).sum(axis=1) * (cb.dx[0] * cb.dx[1] * cb.dx[2])


def two_level_rad_step(A, cb, Gc, Rc, fb, Gf, Rf, off, p, reflux=True):
    """Radiation on two levels over one coarse step dt_c = 1.8 dt_r (two
    substeps on each level): coarse radiation step with a register over the
    footprint, two fine radiation steps of dt_c/2 with radiation ghosts
    interpolated from the coarse level in space and time (gas ghosts once),
    average-down of both states, reflux of the radiation register."""
    lo = tuple(off)
    hi = tuple(off[d] + fb.n[d] // 2 for d in range(3))
    A.fill_ghosts(cb, Gc)
    A.fill_ghosts(cb, Rc)
    A.prolong(cb, Gc, Gc, 0.0, fb, Gf, off, nvar=5)
    dt = 1.8 * p["cfl"] * min(cb.dx) / p["chat"]
    Rc_old = A.copy(Rc)
    reg_c = A.zeros(region_size(lo, hi, 4))
    A.rad_step_reg(cb, Gc, Rc, p, dt, lo, hi, reg_c)
    reg_f = A.zeros(region_size((0, 0, 0), fb.n, 4))
    for alpha in (0.0, 0.5):
        A.prolong(cb, Rc_old, Rc, alpha, fb, Rf, off, nvar=4)
        A.rad_step_reg(fb, Gf, Rf, p, 0.5 * dt, (0, 0, 0), fb.n, reg_f)
    A.average_down(fb, Gf, cb, Gc, off, nvar=5)
    A.average_down(fb, Rf, cb, Rc, off, nvar=4)
    if reflux:
        A.reflux(cb, Rc, lo, hi, reg_c, fb, reg_f, nvar=4)
    return dt


def composite_totals_n(cb, Uc, fb, Uf, off):
    nv = Uc.shape[0]
    I = cb.interior()
    mask = np.ones((cb.n[2], cb.n[1], cb.n[0]), dtype=bool)
    mask[off[2]:off[2] + fb.n[2] // 2, off[1]:off[1] + fb.n[1] // 2, off[0]:off[0] + fb.n[0] // 2] = False
    tc = (Uc[(slice(None),) + I[1:]] * mask).reshape(nv, -1).sum(axis=1) * (cb.dx[0] * cb.dx[1] * cb.dx[2])
    tf = Uf[(slice(None),) + fb.interior()[1:]].reshape(nv, -1).sum(axis=1) * (fb.dx[0] * fb.dx[1] * fb.dx[2])
    return tc + tf


def coarse_totals_n(cb, Uc):
    nv = Uc.shape[0]
    return Uc[(slice(None),) + cb.interior()[1:]].reshape(nv, -1).sum(axis=1) * (cb.dx[0] * cb.dx[1] * cb.dx[2])
