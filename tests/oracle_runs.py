"""Small drivers that run the oracle on one-dimensional test problems of the
paper (used by the oracle pin tests)."""
import numpy as np

import oracle
from paper_2110_01792_amd.inputs import Box, OUTFLOW, PERIODIC


def box1d(N, L=1.0, bc=PERIODIC, ng=4, axis=0):
    n = [1, 1, 1]
    n[axis] = N
    dx = L / N
    bcs = [(PERIODIC, PERIODIC)] * 3
    bcs[axis] = (bc, bc)
    return Box(tuple(n), ng, (dx, dx, dx), tuple(bcs))


def line(b, U, axis=0):
    """Interior values along the active axis, shape (nvar, N)."""
    Ui = U[b.interior()]
    if axis == 0:
        return Ui[:, 0, 0, :]
    if axis == 1:
        return Ui[:, 0, :, 0]
    return Ui[:, :, 0, 0]


def set_line(b, U, vals, axis=0):
    g = b.ng
    idx = [slice(None), slice(g, g + 1), slice(g, g + 1), slice(g, g + 1)]
    idx[3 - axis] = slice(g, g + b.n[axis])
    shape = [vals.shape[0], 1, 1, 1]
    shape[3 - axis] = b.n[axis]
    U[tuple(idx)] = vals.reshape(shape)


def evolve(b, U, gamma, cfl, t_end, max_steps=10 ** 7):
    t, n = 0.0, 0
    while t < t_end * (1.0 - 1e-14) and n < max_steps:
        oracle.fill_ghosts(b, U)
        dt = cfl * min(b.dx[d] for d in range(3) if b.n[d] > 1) / oracle.hydro_max_signal(b, U, gamma)
        if t + dt > t_end:
            dt = t_end - t
        oracle.hydro_step(b, U, gamma, cfl, dt)
        t += dt
        n += 1
    return n


def prim_to_cons(rho, u, p, gamma):
    return np.stack([rho, rho * u, np.zeros_like(rho), np.zeros_like(rho), p / (gamma - 1.0) + 0.5 * rho * u * u])
