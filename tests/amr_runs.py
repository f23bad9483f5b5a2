"""Two-level (refinement ratio 2) step driver shared by the oracle and GPU
level-synchronisation tests.  `A` supplies fill_ghosts, max_signal,
hydro_step_reg, prolong, average_down and reflux with the oracle's
signatures; the driver only sequences them (Section 2.2: coarse step, two
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
