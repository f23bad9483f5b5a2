"""Plain FP64 CPU oracle of the QUOKKA per-cell update (arXiv:2110.01792).

TEST INFRASTRUCTURE ONLY.  This is the slow reference that the GPU library is
checked against.  Only tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does.  It shares no code with the
GPU path: the C source is oracle/quokka_oracle.c, loaded here with ctypes.

Arrays are numpy float64, C-contiguous, shape (nvar, nz+2ng, ny+2ng, nx+2ng).
A box is any object with attributes n (nx, ny, nz), ng, dx (3 floats) and
bc ((lo, hi) per axis, 0 periodic, 1 outflow, 2 fixed, 3 fixed with a
zero-gradient radiation flux).

A function that no independent check fixes would be marked "parity
unpinned" in its docstring; every function here has pins (tests/test_oracle_*.py).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("dx", ctypes.c_double * 3),
                ("bc", (ctypes.c_int32 * 2) * 3)]


class _Rad(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("chat", ctypes.c_double), ("a_r", ctypes.c_double),
                ("kappa_P", ctypes.c_double), ("kappa_R", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha_cv", ctypes.c_double), ("cfl", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("newton_max_iter", ctypes.c_int32), ("nsub_max", ctypes.c_int32), ("closure", ctypes.c_int32),
                ("tau_correction", ctypes.c_int32), ("eos", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("src", ctypes.POINTER(ctypes.c_double))]


class _Region(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


class _Stats(ctypes.Structure):
    _fields_ = [("neg_cells", ctypes.c_int64), ("newton_fail", ctypes.c_int64),
                ("newton_iter_max", ctypes.c_int64), ("nsub", ctypes.c_int32), ("dt", ctypes.c_double),
                ("causal_cells", ctypes.c_int64)]


_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "oracle_fill_ghosts": (None, [P(_Box), _D, ctypes.c_int]),
        "oracle_hydro_max_signal": (ctypes.c_double, [P(_Box), _D, ctypes.c_double]),
        "oracle_hydro_rhs": (None, [P(_Box), _D, ctypes.c_double, ctypes.c_int, _D, P(_Stats)]),
        "oracle_hydro_step": (None, [P(_Box), _D, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     P(_Stats)]),
        "oracle_flatten_chi": (None, [P(_Box), _D, ctypes.c_double, _D]),
        "oracle_rad_rhs": (None, [P(_Box), _D, _D, P(_Rad), _D, P(_Stats)]),
        "oracle_rad_transport_substep": (None, [P(_Box), _D, _D, P(_Rad), ctypes.c_double, P(_Stats)]),
        "oracle_rad_stage": (None, [P(_Box), _D, _D, _D, P(_Rad), ctypes.c_double, _D, P(_Stats)]),
        "oracle_exchange_cell": (ctypes.c_int, [P(_Rad), ctypes.c_double, ctypes.c_double, _D, _D, P(ctypes.c_int)]),
        "oracle_exchange_all": (None, [P(_Box), _D, _D, P(_Rad), ctypes.c_double, P(_Stats)]),
        "oracle_hydro_step_reg": (None, [P(_Box), _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, P(_Region), _D, ctypes.c_double, P(_Stats)]),
        "oracle_average_down": (None, [P(_Box), _D, P(_Box), _D, P(ctypes.c_int32), ctypes.c_int]),
        "oracle_prolong": (None, [P(_Box), _D, _D, ctypes.c_double, P(_Box), _D, P(ctypes.c_int32), ctypes.c_int,
                                  ctypes.c_int]),
        "oracle_reflux": (None, [P(_Box), _D, P(_Region), _D, P(_Box), _D, ctypes.c_int]),
        "oracle_rad_transport_substep_reg": (None, [P(_Box), _D, _D, P(_Rad), ctypes.c_double, P(_Region), _D,
                                                     ctypes.c_double, P(_Stats)]),
        "oracle_exchange_series": (ctypes.c_double, [P(_Rad), ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                                     _D, _D, _D, ctypes.c_int64]),
        "oracle_rhd_step": (None, [P(_Box), _D, _D, P(_Rad), ctypes.c_double, P(_Stats)]),
        "oracle_batch_step": (None, [ctypes.c_int32, P(_Box), P(_D), P(_D), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, P(_Rad), P(_Stats)]),
        "oracle_closure_chi": (ctypes.c_double, [ctypes.c_double, ctypes.c_int]),
        "oracle_closure_pressure": (None, [ctypes.c_double, _D, ctypes.c_double, ctypes.c_int, _D]),
        "oracle_ppm_cell": (None, [_D, _D]),
        "oracle_plm_cell": (None, [_D, _D]),
        "oracle_hllc": (None, [_D, _D, ctypes.c_double, _D]),
        "oracle_hll_rad": (None, [ctypes.c_double, _D, ctypes.c_double, _D, ctypes.c_int, P(_Rad),
                                  ctypes.c_double, _D]),
        "oracle_set_threads": (ctypes.c_int, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _box(b):
    cb = _Box()
    for d in range(3):
        cb.n[d] = int(b.n[d])
        cb.dx[d] = float(b.dx[d])
        cb.bc[d][0] = int(b.bc[d][0])
        cb.bc[d][1] = int(b.bc[d][1])
    cb.ng = int(b.ng)
    return cb


def _rad(p):
    r = _Rad()
    for k in ("c", "chat", "a_r", "kappa_P", "kappa_R", "gamma", "alpha_cv", "cfl", "newton_tol"):
        setattr(r, k, float(p[k]))
    for k in ("newton_max_iter", "nsub_max", "closure", "tau_correction", "eos"):
        setattr(r, k, int(p[k]))
    r.recon = int(p.get("recon", 0))
    src = p.get("source")  # per-cell source rate j, one variable in the box layout (the dict keeps it alive)
    r.src = _ptr(src) if src is not None else ctypes.cast(None, _D)
    return r


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _check(b, a, nvar):
    shape = (nvar, b.n[2] + 2 * b.ng, b.n[1] + 2 * b.ng, b.n[0] + 2 * b.ng)
    if a.shape != shape:
        raise ValueError(f"array shape {a.shape} != {shape}")


def _stats(st):
    return {"neg_cells": st.neg_cells, "newton_fail": st.newton_fail, "newton_iter_max": st.newton_iter_max,
            "nsub": st.nsub, "dt": st.dt, "causal_cells": st.causal_cells}


def set_threads(n=0):
    return _load().oracle_set_threads(int(n))


def fill_ghosts(b, U):
    """Periodic wrap / zero-gradient outflow / fixed ghost cells, axis by axis."""
    _check(b, U, U.shape[0])
    _load().oracle_fill_ghosts(ctypes.byref(_box(b)), _ptr(U), U.shape[0])


def hydro_max_signal(b, U, gamma):
    _check(b, U, 5)
    return _load().oracle_hydro_max_signal(ctypes.byref(_box(b)), _ptr(U), float(gamma))


def hydro_rhs(b, U, gamma, recon=0):
    """L(U) of the hydrodynamic subsystem over interior cells (ghosts of U must be filled).
    recon: 0 PPM, 1 PLM."""
    _check(b, U, 5)
    L = np.zeros_like(U)
    st = _Stats()
    _load().oracle_hydro_rhs(ctypes.byref(_box(b)), _ptr(U), float(gamma), int(recon), _ptr(L), ctypes.byref(st))
    return L, _stats(st)


def flatten_chi(b, U, gamma):
    """Flattening coefficient chi (one variable, box layout) of every cell of
    the box grown by one cell along each active axis (ghosts of U must be filled)."""
    _check(b, U, 5)
    chi = np.zeros(U.shape[1:])
    _load().oracle_flatten_chi(ctypes.byref(_box(b)), _ptr(U), float(gamma), _ptr(chi))
    return chi


def hydro_step(b, U, gamma, cfl, dt=0.0, recon=0):
    """One SSP-RK2 hydro step in place; dt <= 0 takes the CFL step; recon: 0 PPM, 1 PLM."""
    _check(b, U, 5)
    st = _Stats()
    _load().oracle_hydro_step(ctypes.byref(_box(b)), _ptr(U), float(gamma), float(cfl), float(dt), int(recon),
                              ctypes.byref(st))
    return _stats(st)


def rad_rhs(b, Ur, Ug, p):
    _check(b, Ur, 4)
    _check(b, Ug, 5)
    L = np.zeros_like(Ur)
    st = _Stats()
    _load().oracle_rad_rhs(ctypes.byref(_box(b)), _ptr(Ur), _ptr(Ug), ctypes.byref(_rad(p)), _ptr(L),
                           ctypes.byref(st))
    return L, _stats(st)


def rad_transport_substep(b, Ur, Ug, p, dt):
    """One RK2 radiation transport substep (no coupling) in place."""
    _check(b, Ur, 4)
    _check(b, Ug, 5)
    st = _Stats()
    _load().oracle_rad_transport_substep(ctypes.byref(_box(b)), _ptr(Ur), _ptr(Ug), ctypes.byref(_rad(p)),
                                         float(dt), ctypes.byref(st))
    return _stats(st)


def rad_stage(b, Uin, Ug, p, dt, Ubase=None):
    """One radiation RK stage: Uin + dt L(Uin) (first stage) or, given Ubase,
    Ubase/2 + (Uin + dt L(Uin))/2; returns (Uout, stats).  Uout's ghosts are
    those of Ubase (else Uin).  tau_correction 1 applies the causality rule of
    Section 2.2.2, 2 the optical-depth factor without it."""
    _check(b, Uin, 4)
    _check(b, Ug, 5)
    out = (Ubase if Ubase is not None else Uin).copy()
    st = _Stats()
    _load().oracle_rad_stage(ctypes.byref(_box(b)), _ptr(Uin), _ptr(Ubase) if Ubase is not None else ctypes.cast(None, _D),
                             _ptr(Ug), ctypes.byref(_rad(p)), float(dt), _ptr(out), ctypes.byref(st))
    return out, _stats(st)


def exchange_cell(p, dt, gas, rad, S=0.0):
    """Coupling update of one cell with radiation source S (energy density
    added over dt); returns (gas, rad, converged, iterations)."""
    g = np.ascontiguousarray(gas, dtype=np.float64).copy()
    r = np.ascontiguousarray(rad, dtype=np.float64).copy()
    it = ctypes.c_int(0)
    fail = _load().oracle_exchange_cell(ctypes.byref(_rad(p)), float(dt), float(S), _ptr(g), _ptr(r),
                                        ctypes.byref(it))
    return g, r, fail == 0, it.value


def exchange_all(b, Ug, Ur, p, dt):
    st = _Stats()
    _load().oracle_exchange_all(ctypes.byref(_box(b)), _ptr(Ug), _ptr(Ur), ctypes.byref(_rad(p)), float(dt),
                                ctypes.byref(st))
    return _stats(st)


def exchange_series(p, dt, nsteps, gas, rad, every, S=0.0):
    g = np.ascontiguousarray(gas, dtype=np.float64).copy()
    r = np.ascontiguousarray(rad, dtype=np.float64).copy()
    out = np.zeros(int(nsteps) // int(every), dtype=np.float64)
    _load().oracle_exchange_series(ctypes.byref(_rad(p)), float(dt), float(S), int(nsteps), _ptr(g), _ptr(r),
                                   _ptr(out), int(every))
    return out, g, r


def rhd_step(b, Ug, Ur, p, dt=0.0):
    """One radiation-hydrodynamics step in place (hydro RK2, then N_sub x (radiation RK2 + coupling))."""
    _check(b, Ug, 5)
    _check(b, Ur, 4)
    st = _Stats()
    _load().oracle_rhd_step(ctypes.byref(_box(b)), _ptr(Ug), _ptr(Ur), ctypes.byref(_rad(p)), float(dt),
                            ctypes.byref(st))
    return _stats(st)


def batch_step(boxes, Ugs, Urs, gamma_h, cfl, p, recon_h=0):
    """One level step over boxes with fixed ghosts; Urs[i] None marks a hydro-only box."""
    nb = len(boxes)
    cboxes = (_Box * nb)(*[_box(b) for b in boxes])
    gp = (_D * nb)(*[_ptr(u) for u in Ugs])
    rp = (_D * nb)(*[(_ptr(u) if u is not None else ctypes.cast(None, _D)) for u in Urs])
    st = _Stats()
    _load().oracle_batch_step(nb, cboxes, gp, rp, float(gamma_h), float(cfl), int(recon_h), ctypes.byref(_rad(p)),
                              ctypes.byref(st))
    return _stats(st)


def closure_chi(f, closure=0):
    return _load().oracle_closure_chi(float(f), int(closure))


def closure_pressure(E, F, c, closure=0):
    Fa = np.ascontiguousarray(F, dtype=np.float64)
    P = np.zeros(9)
    _load().oracle_closure_pressure(float(E), _ptr(Fa), float(c), int(closure), _ptr(P))
    return P.reshape(3, 3)


def plm_cell(q3):
    q = np.ascontiguousarray(q3, dtype=np.float64)
    out = np.zeros(2)
    _load().oracle_plm_cell(_ptr(q), _ptr(out))
    return out[0], out[1]


def ppm_cell(q5):
    q = np.ascontiguousarray(q5, dtype=np.float64)
    out = np.zeros(2)
    _load().oracle_ppm_cell(_ptr(q), _ptr(out))
    return out[0], out[1]


def hllc(WL, WR, gamma):
    a = np.ascontiguousarray(WL, dtype=np.float64)
    b = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    _load().oracle_hllc(_ptr(a), _ptr(b), float(gamma), _ptr(F))
    return F


def hll_rad(EL, FL, ER, FR, direction, p, eps=1.0):
    a = np.ascontiguousarray(FL, dtype=np.float64)
    b = np.ascontiguousarray(FR, dtype=np.float64)
    out = np.zeros(4)
    _load().oracle_hll_rad(float(EL), _ptr(a), float(ER), _ptr(b), int(direction), ctypes.byref(_rad(p)),
                           float(eps), _ptr(out))
    return out


# ------------------------------------------------------------ AMR (ratio 2)
def region_size(lo, hi, nvar=5):
    """Doubles in a flux register over region [lo, hi)."""
    m = [hi[d] - lo[d] for d in range(3)]
    return nvar * 2 * (m[1] * m[2] + m[0] * m[2] + m[0] * m[1])


def _region(lo, hi):
    r = _Region()
    for d in range(3):
        r.lo[d] = int(lo[d])
        r.hi[d] = int(hi[d])
    return r


def _i3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def hydro_step_reg(b, U, gamma, cfl, dt, lo, hi, reg, weight=1.0, recon=0):
    """Hydro step that adds weight * dt/2 * F of both RK stages at the faces
    bounding region [lo, hi) to the FP64 register `reg`."""
    _check(b, U, 5)
    assert reg.dtype == np.float64 and reg.size == region_size(lo, hi)
    st = _Stats()
    _load().oracle_hydro_step_reg(ctypes.byref(_box(b)), _ptr(U), float(gamma), float(cfl), float(dt), int(recon),
                                  ctypes.byref(_region(lo, hi)), _ptr(reg), float(weight), ctypes.byref(st))
    return _stats(st)


def average_down(fine, Uf, coarse, Uc, off, nvar=5):
    _load().oracle_average_down(ctypes.byref(_box(fine)), _ptr(Uf), ctypes.byref(_box(coarse)), _ptr(Uc), _i3(off),
                                int(nvar))


def prolong(coarse, Uc0, Uc1, alpha, fine, Uf, off, nvar=5, interior=False):
    _load().oracle_prolong(ctypes.byref(_box(coarse)), _ptr(Uc0), _ptr(Uc1), float(alpha), ctypes.byref(_box(fine)),
                           _ptr(Uf), _i3(off), int(nvar), int(bool(interior)))


def reflux(coarse, Uc, lo, hi, reg_c, fine, reg_f, nvar=5):
    _load().oracle_reflux(ctypes.byref(_box(coarse)), _ptr(Uc), ctypes.byref(_region(lo, hi)), _ptr(reg_c),
                          ctypes.byref(_box(fine)), _ptr(reg_f), int(nvar))


def rad_transport_substep_reg(b, Ur, Ug, p, dt, lo, hi, reg, weight=1.0):
    """Radiation RK2 transport substep adding weight * dt/2 * F of both stages
    at the faces bounding [lo, hi) to `reg` (4 variables)."""
    _check(b, Ur, 4)
    _check(b, Ug, 5)
    assert reg.dtype == np.float64 and reg.size == region_size(lo, hi, 4)
    st = _Stats()
    _load().oracle_rad_transport_substep_reg(ctypes.byref(_box(b)), _ptr(Ur), _ptr(Ug), ctypes.byref(_rad(p)),
                                             float(dt), ctypes.byref(_region(lo, hi)), _ptr(reg), float(weight),
                                             ctypes.byref(st))
    return _stats(st)
