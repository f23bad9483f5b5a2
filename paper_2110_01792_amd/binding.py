"""ctypes binding of libquokka_mi355x.so (C ABI in include/quokka.h).

Argument marshalling only: every step of the update runs in the HIP library.
State arguments are torch tensors on a ROCm device (float64 for F64, float32
for MIXED), shape (nvar, nz+2ng, ny+2ng, nx+2ng), contiguous or a padded view
with x contiguous (its strides become the box pitches); PyTorch supplies
device memory and streams, nothing else.  If the library is missing this
module raises; there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libquokka_mi355x.so")

QK_OK, QK_EINVAL, QK_ENOMEM, QK_EHIP, QK_ENEGATIVE, QK_ENEWTON = range(6)
F64, MIXED = 0, 1
STATUS_NAMES = {0: "QK_OK", 1: "QK_EINVAL", 2: "QK_ENOMEM", 3: "QK_EHIP", 4: "QK_ENEGATIVE", 5: "QK_ENEWTON"}

EXPORTED = ("quokka_ctx_create", "quokka_ctx_destroy", "quokka_last_error", "quokka_fill_ghosts",
            "quokka_compute_dt", "quokka_hydro_step", "quokka_rad_step", "quokka_rhd_step", "quokka_batch_step",
            "quokka_sync_status", "quokka_newton_iter_max", "quokka_timing", "quokka_kernel_time", "quokka_batch_config",
            "quokka_hydro_step_reg", "quokka_average_down", "quokka_prolong", "quokka_reflux",
            "quokka_rad_step_reg", "quokka_hydro_step_noalloc")
K_HYDRO_STAGE, K_FLATTEN, K_RAD_STAGE, K_RAD_COUPLE, K_GHOST, K_BATCH = range(6)


class QkBox(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("pitch_y", ctypes.c_int64),
                ("pitch_z", ctypes.c_int64), ("var_stride", ctypes.c_int64), ("dx", ctypes.c_double * 3),
                ("bc", (ctypes.c_int32 * 2) * 3)]


class QkRegion(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


def make_region(lo, hi):
    r = QkRegion()
    for d in range(3):
        r.lo[d] = int(lo[d])
        r.hi[d] = int(hi[d])
    return r


def region_size(lo, hi, nvar=5):
    """Doubles in a flux register over region [lo, hi)."""
    m = [int(hi[d]) - int(lo[d]) for d in range(3)]
    return nvar * 2 * (m[1] * m[2] + m[0] * m[2] + m[0] * m[1])


class QkHydroParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("reconstruction", ctypes.c_int32)]


class QkRadParams(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("chat", ctypes.c_double), ("a_r", ctypes.c_double),
                ("kappa_P", ctypes.c_double), ("kappa_R", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha_cv", ctypes.c_double), ("cfl", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("newton_max_iter", ctypes.c_int32), ("nsub_max", ctypes.c_int32), ("closure", ctypes.c_int32),
                ("tau_correction", ctypes.c_int32), ("eos", ctypes.c_int32), ("reconstruction", ctypes.c_int32),
                ("source", ctypes.c_void_p)]


class QuokkaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2110_01792_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    # torch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes the library bind to that already-loaded copy,
    # so the process has one HIP runtime and torch's memory and streams are
    # valid in library calls (loading the library first would bring up a
    # second runtime, which then cannot see the device).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I32, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sigs = {
        "quokka_ctx_create": (ctypes.c_int, [ctypes.c_int, P(V)]),
        "quokka_ctx_destroy": (None, [V]),
        "quokka_last_error": (ctypes.c_char_p, [V]),
        "quokka_fill_ghosts": (ctypes.c_int, [V, P(QkBox), V, I32, ctypes.c_int, V]),
        "quokka_compute_dt": (ctypes.c_int, [V, P(QkBox), V, ctypes.c_int, P(QkHydroParams), P(QkRadParams), V, V,
                                             P(D), V]),
        "quokka_hydro_step": (ctypes.c_int, [V, P(QkBox), V, ctypes.c_int, P(QkHydroParams), V, D, V, V]),
        "quokka_hydro_step_noalloc": (ctypes.c_int, [V, P(QkBox), V, ctypes.c_int, P(QkHydroParams), V, D, V, V]),
        "quokka_rad_step": (ctypes.c_int, [V, P(QkBox), V, V, ctypes.c_int, P(QkRadParams), V, V, D, V]),
        "quokka_rhd_step": (ctypes.c_int, [V, P(QkBox), V, V, ctypes.c_int, P(QkRadParams), P(D), V]),
        "quokka_batch_step": (ctypes.c_int, [V, P(QkBox), I32, P(V), P(V), ctypes.c_int, P(QkHydroParams),
                                             P(QkRadParams), P(D), V]),
        "quokka_sync_status": (ctypes.c_int, [V, V]),
        "quokka_newton_iter_max": (I32, [V, V]),
        "quokka_timing": (ctypes.c_int, [V, I32]),
        "quokka_kernel_time": (ctypes.c_int, [V, I32, P(D), P(ctypes.c_int64)]),
        "quokka_batch_config": (ctypes.c_int, [V, P(I32), P(I32), P(D)]),
        "quokka_hydro_step_reg": (ctypes.c_int, [V, P(QkBox), V, ctypes.c_int, P(QkHydroParams), V, D, P(QkRegion), V,
                                                 D, V]),
        "quokka_average_down": (ctypes.c_int, [V, P(QkBox), V, P(QkBox), V, P(I32), I32, ctypes.c_int, V]),
        "quokka_prolong": (ctypes.c_int, [V, P(QkBox), V, V, D, P(QkBox), V, P(I32), I32, I32, ctypes.c_int, V]),
        "quokka_reflux": (ctypes.c_int, [V, P(QkBox), V, P(QkRegion), V, P(QkBox), V, I32, ctypes.c_int, V]),
        "quokka_rad_step_reg": (ctypes.c_int, [V, P(QkBox), V, V, ctypes.c_int, P(QkRadParams), V, V, D,
                                               P(QkRegion), V, D, V]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def make_box(b, layout=(0, 0, 0)):
    """QkBox from any object with n, ng, dx, bc; layout = (pitch_y, pitch_z,
    var_stride) in elements, (0, 0, 0) for the contiguous layout."""
    q = QkBox()
    for d in range(3):
        q.n[d] = int(b.n[d])
        q.dx[d] = float(b.dx[d])
        q.bc[d][0] = int(b.bc[d][0])
        q.bc[d][1] = int(b.bc[d][1])
    q.ng = int(b.ng)
    q.pitch_y, q.pitch_z, q.var_stride = (int(x) for x in layout)
    return q


def hydro_params(gamma, cfl, recon=0):
    """recon: 0 PPM, 1 PLM."""
    return QkHydroParams(float(gamma), float(cfl), int(recon))


def rad_params(p, source=None):
    """Radiation parameters from a dict; `source` is None or a device tensor of
    the per-cell radiation source rate (box shape, state dtype), which the
    caller keeps alive while the library uses it."""
    r = QkRadParams()
    for k in ("c", "chat", "a_r", "kappa_P", "kappa_R", "gamma", "alpha_cv", "cfl", "newton_tol"):
        setattr(r, k, float(p[k]))
    for k in ("newton_max_iter", "nsub_max", "closure", "tau_correction", "eos"):
        setattr(r, k, int(p[k]))
    r.reconstruction = int(p.get("recon", 0))
    r.source = None if source is None else source.data_ptr()
    return r


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _prec_of(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return MIXED
    raise TypeError(f"state dtype {t.dtype} is neither float64 nor float32")


def _check_state(t, b, nvar):
    """Check a device state tensor of shape (nvar, NZ, NY, NX) and return its
    layout (pitch_y, pitch_z, var_stride): (0, 0, 0) when contiguous, else
    the strides of a padded view (x contiguous, each outer stride at least the
    extent it spans), which the library addresses through the box pitches."""
    shape = (nvar, b.n[2] + 2 * b.ng, b.n[1] + 2 * b.ng, b.n[0] + 2 * b.ng)
    if tuple(t.shape) != shape:
        raise ValueError(f"state shape {tuple(t.shape)} != {shape}")
    if t.device.type != "cuda":
        raise ValueError("state must be a device tensor")
    if t.is_contiguous():
        return (0, 0, 0)
    sv, sz, sy, sx = t.stride()
    if sx != 1 or sy < shape[3] or sz < sy * shape[2] or sv < sz * shape[1]:
        raise ValueError(f"state strides {t.stride()} are not a padded x-contiguous layout")
    return (sy, sz, sv)


def _same_layout(*layouts):
    """Gas and radiation states of one call share the box's pitches."""
    if any(l != layouts[0] for l in layouts[1:]):
        raise ValueError(f"states of one box must share one layout, got {layouts}")
    return layouts[0]


class Context:
    """One library context on one device."""

    def __init__(self, device=0):
        self.lib = load()
        h = ctypes.c_void_p()
        st = self.lib.quokka_ctx_create(int(device), ctypes.byref(h))
        if st != QK_OK:
            raise QuokkaError(st, f"cannot create a context on device {device}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.quokka_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, st):
        if st != QK_OK:
            raise QuokkaError(st, self.lib.quokka_last_error(self.h).decode())

    def fill_ghosts(self, b, U, stream=None):
        lay = _check_state(U, b, U.shape[0])
        self._ok(self.lib.quokka_fill_ghosts(self.h, ctypes.byref(make_box(b, lay)), _ptr(U), int(U.shape[0]),
                                             _prec_of(U), _stream(stream)))

    def compute_dt(self, b, Ug, hp=None, rp=None, dt_dev=None, nsub_dev=None, host=True, stream=None):
        lay = _check_state(Ug, b, 5)
        out = ctypes.c_double(0.0)
        self._ok(self.lib.quokka_compute_dt(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _prec_of(Ug),
                                            ctypes.byref(hp) if hp is not None else None,
                                            ctypes.byref(rp) if rp is not None else None, _ptr(dt_dev),
                                            _ptr(nsub_dev), ctypes.byref(out) if host else None, _stream(stream)))
        return out.value if host else None

    def hydro_step(self, b, Ug, hp, dt_dev=None, dt=0.0, dt_next_dev=None, stream=None):
        lay = _check_state(Ug, b, 5)
        self._ok(self.lib.quokka_hydro_step(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _prec_of(Ug),
                                            ctypes.byref(hp), _ptr(dt_dev), float(dt), _ptr(dt_next_dev),
                                            _stream(stream)))

    def hydro_step_noalloc(self, b, Ug, hp, dt_dev=None, dt=0.0, dt_next_dev=None, stream=None):
        """quokka_hydro_step with the library's static scratch (allocates nothing)."""
        lay = _check_state(Ug, b, 5)
        self._ok(self.lib.quokka_hydro_step_noalloc(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _prec_of(Ug),
                                                    ctypes.byref(hp), _ptr(dt_dev), float(dt), _ptr(dt_next_dev),
                                                    _stream(stream)))

    # ---------------------------------------------------- AMR (ratio 2)
    def hydro_step_reg(self, b, Ug, hp, lo, hi, reg, dt=0.0, dt_dev=None, weight=1.0, stream=None):
        """Hydro step adding weight * dt/2 * F of both stages at the faces
        bounding region [lo, hi) to the FP64 device register `reg`."""
        import torch
        lay = _check_state(Ug, b, 5)
        if reg.dtype != torch.float64 or reg.numel() != region_size(lo, hi) or not reg.is_cuda:
            raise ValueError("register must be a float64 device tensor of region_size(lo, hi) elements")
        self._ok(self.lib.quokka_hydro_step_reg(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _prec_of(Ug),
                                                ctypes.byref(hp), _ptr(dt_dev), float(dt),
                                                ctypes.byref(make_region(lo, hi)), _ptr(reg), float(weight),
                                                _stream(stream)))

    def rad_step_reg(self, b, Ug, Ur, rp, lo, hi, reg, dt, weight=1.0, stream=None):
        """Radiation step over host dt (ceil(dt / dt_r) substeps) adding
        weight * dt_sub/2 * F of every stage at the faces bounding [lo, hi)
        to the FP64 device register `reg` (4 variables)."""
        import torch
        lay = _same_layout(_check_state(Ug, b, 5), _check_state(Ur, b, 4))
        if reg.dtype != torch.float64 or reg.numel() != region_size(lo, hi, 4) or not reg.is_cuda:
            raise ValueError("register must be a float64 device tensor of region_size(lo, hi, 4) elements")
        self._ok(self.lib.quokka_rad_step_reg(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _ptr(Ur), _prec_of(Ug),
                                              ctypes.byref(rp), None, None, float(dt),
                                              ctypes.byref(make_region(lo, hi)), _ptr(reg), float(weight),
                                              _stream(stream)))

    def average_down(self, fb, Uf, cb, Uc, off, nvar=5, stream=None):
        lf = _check_state(Uf, fb, nvar)
        lc = _check_state(Uc, cb, nvar)
        o = (ctypes.c_int32 * 3)(*[int(x) for x in off])
        self._ok(self.lib.quokka_average_down(self.h, ctypes.byref(make_box(fb, lf)), _ptr(Uf),
                                              ctypes.byref(make_box(cb, lc)), _ptr(Uc), o, int(nvar), _prec_of(Uf),
                                              _stream(stream)))

    def prolong(self, cb, Uc0, Uc1, alpha, fb, Uf, off, nvar=5, interior=False, stream=None):
        lc = _same_layout(_check_state(Uc0, cb, nvar), _check_state(Uc1, cb, nvar))
        lf = _check_state(Uf, fb, nvar)
        o = (ctypes.c_int32 * 3)(*[int(x) for x in off])
        self._ok(self.lib.quokka_prolong(self.h, ctypes.byref(make_box(cb, lc)), _ptr(Uc0), _ptr(Uc1), float(alpha),
                                         ctypes.byref(make_box(fb, lf)), _ptr(Uf), o, int(nvar), int(bool(interior)),
                                         _prec_of(Uf), _stream(stream)))

    def reflux(self, cb, Uc, lo, hi, reg_c, fb, reg_f, nvar=5, stream=None):
        lc = _check_state(Uc, cb, nvar)
        self._ok(self.lib.quokka_reflux(self.h, ctypes.byref(make_box(cb, lc)), _ptr(Uc),
                                        ctypes.byref(make_region(lo, hi)), _ptr(reg_c), ctypes.byref(make_box(fb)),
                                        _ptr(reg_f), int(nvar), _prec_of(Uc), _stream(stream)))

    def rad_step(self, b, Ug, Ur, rp, dt_dev=None, nsub_dev=None, dt=0.0, stream=None):
        lay = _same_layout(_check_state(Ug, b, 5), _check_state(Ur, b, 4))
        self._ok(self.lib.quokka_rad_step(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _ptr(Ur), _prec_of(Ug),
                                          ctypes.byref(rp), _ptr(dt_dev), _ptr(nsub_dev), float(dt),
                                          _stream(stream)))

    def rhd_step(self, b, Ug, Ur, rp, host_dt=False, stream=None):
        lay = _same_layout(_check_state(Ug, b, 5), _check_state(Ur, b, 4))
        out = ctypes.c_double(0.0)
        self._ok(self.lib.quokka_rhd_step(self.h, ctypes.byref(make_box(b, lay)), _ptr(Ug), _ptr(Ur), _prec_of(Ug),
                                          ctypes.byref(rp), ctypes.byref(out) if host_dt else None,
                                          _stream(stream)))
        return out.value if host_dt else None

    def batch_step(self, boxes, Ugs, Urs, hp, rp, host_dt=True, stream=None):
        n = len(boxes)
        lays = [_check_state(g, b, 5) if r is None else _same_layout(_check_state(g, b, 5), _check_state(r, b, 4))
                for b, g, r in zip(boxes, Ugs, Urs)]
        arr = (QkBox * n)(*[make_box(b, l) for b, l in zip(boxes, lays)])
        gp = (ctypes.c_void_p * n)(*[u.data_ptr() for u in Ugs])
        rpp = (ctypes.c_void_p * n)(*[(u.data_ptr() if u is not None else None) for u in Urs])
        out = ctypes.c_double(0.0)
        self._ok(self.lib.quokka_batch_step(self.h, arr, n, gp, rpp, _prec_of(Ugs[0]), ctypes.byref(hp),
                                            ctypes.byref(rp) if rp is not None else None,
                                            ctypes.byref(out) if host_dt else None, _stream(stream)))
        return out.value if host_dt else None

    def sync_status(self, stream=None):
        return self.lib.quokka_sync_status(self.h, _stream(stream))

    def newton_iter_max(self, stream=None):
        return self.lib.quokka_newton_iter_max(self.h, _stream(stream))

    def batch_config(self):
        """(tile, zc, tune_ms) chosen for the last batch step."""
        t, z, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
        self._ok(self.lib.quokka_batch_config(self.h, ctypes.byref(t), ctypes.byref(z), ctypes.byref(ms)))
        return t.value, z.value, ms.value

    def timing(self, enable):
        self._ok(self.lib.quokka_timing(self.h, 1 if enable else 0))

    def kernel_time(self, kclass):
        """(total ms, launches) of a kernel class since timing was enabled."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        self._ok(self.lib.quokka_kernel_time(self.h, int(kclass), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
