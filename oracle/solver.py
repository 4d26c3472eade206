"""ctypes wrapper over the FP64 C oracle (``oracle.c``).

Test infrastructure only: see ``oracle/__init__.py``.  The parameter record
is this module's own; it mirrors nothing from the HIP library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
EPS0 = 8.8541878128e-12

X, VX, VY, SRC, SEE, SELF = 1, 2, 4, 8, 16, 32
ALL = X | VX | VY | SRC | SEE | SELF
BGK = 64   # electron-electron collisions (Eq 3-5); not part of ALL
NOSC = 128  # with SELF: E_x from sigma alone, no electron space charge


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("nvx", C.c_int), ("nvy", C.c_int),
        ("length", C.c_double), ("vmax_x", C.c_double), ("vmax_y", C.c_double),
        ("dt", C.c_double), ("cfl", C.c_double), ("ey", C.c_double),
        ("delta_max", C.c_double), ("a_max_ev", C.c_double), ("ks", C.c_double),
        ("t_se_ev", C.c_double), ("j_src", C.c_double), ("x_src_lo", C.c_double),
        ("x_src_hi", C.c_double), ("t_src_ev", C.c_double),
        ("emission_norm", C.c_int), ("physics_mask", C.c_uint),
        ("ex_external", C.c_double), ("t_e_ev", C.c_double), ("ln_lambda", C.c_double),
        ("r_refl", C.c_double), ("r_inel", C.c_double), ("scheme", C.c_int),
    ]


class Record(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("t", C.c_double), ("sigma", C.c_double),
        ("g_pe", C.c_double), ("g_see", C.c_double), ("g_top", C.c_double),
        ("emitted", C.c_double), ("loss_v", C.c_double), ("n_total", C.c_double),
        ("resid", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_native = False


def use_native_build():
    """Load the host-tuned build (-march=native, compiled on this machine)
    instead of the portable one; only before the first oracle call (the
    benchmark's CPU baseline)."""
    global _native
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _native = True


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=_native, native=_native)
        L = C.CDLL(path)
        P = C.POINTER
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [P(_Params)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p, P(C.c_double), C.c_double, C.c_int64]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64, P(Record)]
        L.orc_get_record.argtypes = [C.c_void_p, P(Record)]
        L.orc_get_f.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_get_field.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        L.orc_get_tables.argtypes = [C.c_void_p] + [P(C.c_double)] * 7
        L.orc_get_ghost.argtypes = [C.c_void_p, P(C.c_double)]
        L.orc_cfl_max_vx.restype = C.c_double
        L.orc_cfl_max_vx.argtypes = [C.c_void_p]
        L.orc_sey.restype = C.c_double
        L.orc_sey.argtypes = [C.c_double] * 5
        L.orc_fn_current.restype = C.c_double
        L.orc_fn_current.argtypes = [C.c_double] * 3
        L.orc_nu_ee.restype = C.c_double
        L.orc_nu_ee.argtypes = [C.c_double] * 3
        L.orc_nu_dt_max.restype = C.c_double
        L.orc_nu_dt_max.argtypes = [C.c_void_p]
        L.orc_get_feq.argtypes = [C.c_void_p, P(C.c_double)]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def sey(delta_max, a_max_ev, ks, a_in_ev, alpha):
    """Eq 8-9 evaluated by the C oracle at one (energy, angle)."""
    return lib().orc_sey(delta_max, a_max_ev, ks, a_in_ev, alpha)


def fn_current(e_field, phi_ev, beta=1.0):
    """Eq 6 evaluated by the C oracle (A/m^2)."""
    return lib().orc_fn_current(float(e_field), float(phi_ev), float(beta))


def nu_ee(n_e, t_e_ev, ln_lambda):
    """Eq 4 evaluated by the C oracle: collision frequency (1/s) at density
    n_e (1/m^3) and temperature t_e_ev (eV)."""
    return lib().orc_nu_ee(float(n_e), float(t_e_ev), float(ln_lambda))


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


class Oracle:
    """One FP64 CPU simulation.  ``cfg`` is a dict of the parameter names above."""

    def __init__(self, cfg):
        c = dict(cfg)
        missing = [n for n, _ in _Params._fields_ if n not in c]
        if missing:
            raise KeyError(f"oracle parameters missing: {missing}")
        self.cfg = c
        p = _Params()
        for name, _ in _Params._fields_:
            setattr(p, name, c[name])
        self._p = p
        self._h = lib().orc_create(C.byref(p))
        if not self._h:
            raise MemoryError("oracle allocation failed")
        self.nx, self.nvx, self.nvy = c["nx"], c["nvx"], c["nvy"]
        self.shape = (self.nx, self.nvx, self.nvy)
        self.dt = lib().orc_dt(self._h)
        self.dx = c["length"] / self.nx
        self.dvx = 2 * c["vmax_x"] / self.nvx
        self.dvy = 2 * c["vmax_y"] / self.nvy

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, f=None, sigma=0.0, step=0):
        if f is None:
            lib().orc_set_state(self._h, None, float(sigma), int(step))
        else:
            a = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape)
            lib().orc_set_state(self._h, _ptr(a), float(sigma), int(step))

    def step(self, n=1, trace=False):
        if trace:
            recs = (Record * n)()
            lib().orc_step(self._h, int(n), recs)
            return [r.as_dict() for r in recs]
        lib().orc_step(self._h, int(n), None)
        return None

    def record(self):
        r = Record()
        lib().orc_get_record(self._h, C.byref(r))
        return r.as_dict()

    def f(self):
        out = np.empty(self.shape, dtype=np.float64)
        lib().orc_get_f(self._h, _ptr(out))
        return out

    def field(self):
        ex = np.empty(self.nx)
        ne = np.empty(self.nx)
        lib().orc_get_field(self._h, _ptr(ex), _ptr(ne))
        return ex, ne

    def tables(self):
        vx = np.empty(self.nvx)
        vy = np.empty(self.nvy)
        delta = np.empty((self.nvx, self.nvy))
        ghat = np.empty((self.nvx, self.nvy))
        fsrc = np.empty((self.nvx, self.nvy))
        w = np.empty(self.nx)
        z = np.empty(1)
        lib().orc_get_tables(self._h, _ptr(vx), _ptr(vy), _ptr(delta), _ptr(ghat), _ptr(fsrc),
                             _ptr(w), _ptr(z))
        return dict(vx=vx, vy=vy, delta=delta, ghat=ghat, fsrc=fsrc, wband=w, zsum=float(z[0]))

    def ghost(self):
        g = np.empty((self.nvx, self.nvy))
        lib().orc_get_ghost(self._h, _ptr(g))
        return g

    def cfl_max_vx(self):
        return lib().orc_cfl_max_vx(self._h)

    def nu_dt_max(self):
        """Largest nu_ee dt of the collision steps so far."""
        return lib().orc_nu_dt_max(self._h)

    def feq(self):
        """The collisional equilibrium of Eq 5 on the grid, normalised."""
        out = np.empty((self.nvx, self.nvy))
        lib().orc_get_feq(self._h, _ptr(out))
        return out
