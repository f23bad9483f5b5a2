"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal
gas (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4),
written from the mathematics: the star-region pressure is the root of the
pressure function f(p) = f_L(p) + f_R(p) + (u_R - u_L), where f_K is the
shock (Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction
branch otherwise; the solution is then sampled on x/t.

Used by the tests as an independent reference for the oracle's shock tubes.
Its own correctness is checked in tests/test_exact_riemann.py against the jump
conditions and Riemann invariants it must satisfy.
"""
import numpy as np
from scipy.optimize import brentq


def _fK(p, rho, pK, g):
    c = np.sqrt(g * pK / rho)
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        return (p - pK) * np.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(WL, WR, g):
    """(p*, u*) for primitive states (rho, u, p)."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    f = lambda p: _fK(p, rL, pL, g) + _fK(p, rR, pR, g) + (uR - uL)
    lo, hi = 1e-14 * min(pL, pR), 10.0 * max(pL, pR)
    while f(hi) < 0.0:
        hi *= 10.0
    if f(lo) > 0.0:
        raise ValueError("vacuum generated; no star state")
    ps = brentq(f, lo, hi, xtol=1e-15 * max(pL, pR), rtol=1e-15, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (_fK(ps, rR, pR, g) - _fK(ps, rL, pL, g))
    return ps, us


def sample(WL, WR, g, xi):
    """Primitive (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    ps, us = star_state(WL, WR, g)
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.ravel()):
        if s <= us:  # left of contact
            if ps > pL:  # left shock
                SL = uL - cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                if s <= SL:
                    w = (rL, uL, pL)
                else:
                    w = (rL * (ps / pL + gm) / (gm * ps / pL + 1.0), us, ps)
            else:  # left rarefaction
                SHL = uL - cL
                csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
                STL = us - csL
                if s <= SHL:
                    w = (rL, uL, pL)
                elif s >= STL:
                    w = (rL * (ps / pL) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    w = (rL * (c / cL) ** (2.0 / (g - 1)), 2.0 / (g + 1) * (cL + (g - 1) / 2 * uL + s),
                         pL * (c / cL) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pR:
                SR = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                if s >= SR:
                    w = (rR, uR, pR)
                else:
                    w = (rR * (ps / pR + gm) / (gm * ps / pR + 1.0), us, ps)
            else:
                SHR = uR + cR
                csR = cR * (ps / pR) ** ((g - 1) / (2 * g))
                STR = us + csR
                if s >= SHR:
                    w = (rR, uR, pR)
                elif s <= STR:
                    w = (rR * (ps / pR) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    w = (rR * (c / cR) ** (2.0 / (g - 1)), 2.0 / (g + 1) * (-cR + (g - 1) / 2 * uR + s),
                         pR * (c / cR) ** (2 * g / (g - 1)))
        rho.flat[n], u.flat[n], p.flat[n] = w
    return rho, u, p


def conserved(rho, u, p, g):
    return np.stack([rho, rho * u, np.zeros_like(rho), np.zeros_like(rho), p / (g - 1.0) + 0.5 * rho * u * u])
