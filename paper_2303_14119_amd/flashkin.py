"""ctypes binding of ``libflashkin.so`` (declared in ``include/flashkin.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
Importing this module loads the library and raises ``ImportError`` if it has
not been built (``python -m paper_2303_14119_amd.build``); there is no other
code path.  torch is optional and used only to hand device pointers and
streams to the library.
"""
import ctypes as C
import os

import numpy as np

# One HIP runtime per process.  torch's HIP libraries ask for the runtime
# under a different file name than this library does, so whichever loads
# second would otherwise bring in a second runtime, and only one of the two
# can open the device.  Loading torch first lets the library bind to torch's
# runtime, the one that owns the device memory and streams handed over.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflashkin.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_14119_amd.build`")
_lib = C.CDLL(LIB_PATH)

ABI_VERSION = 5
F32, F64 = 0, 1
EMIT_DISCRETE, EMIT_ANALYTIC = 0, 1
PHYS_X, PHYS_VX, PHYS_VY, PHYS_SRC, PHYS_SEE, PHYS_SELF_FIELD, PHYS_ALL = 1, 2, 4, 8, 16, 32, 63
PHYS_BGK = 64   # electron-electron collisions (Eq 3-5); opt-in
PHYS_NO_SPACE_CHARGE = 128   # with PHYS_SELF_FIELD: the surface charge's field alone; opt-in
SCHEME_UPWIND, SCHEME_LIMITED2 = 0, 1
OK, E_INVALID, E_OOM, E_HIP, E_CFL, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5, -6


class fk_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("abi_version", C.c_uint32),
        ("nx", C.c_int32), ("nvx", C.c_int32), ("nvy", C.c_int32), ("dtype", C.c_int32),
        ("length_m", C.c_double), ("vmax_x", C.c_double), ("vmax_y", C.c_double),
        ("dt", C.c_double), ("cfl", C.c_double), ("ey", C.c_double),
        ("delta_max", C.c_double), ("a_max_ev", C.c_double), ("ks", C.c_double),
        ("t_se_ev", C.c_double), ("j_src", C.c_double), ("x_src_lo", C.c_double),
        ("x_src_hi", C.c_double), ("t_src_ev", C.c_double),
        ("emission_norm", C.c_int32), ("physics_mask", C.c_uint32),
        ("ex_external", C.c_double), ("trace_stride", C.c_int32), ("trace_cap", C.c_int32),
        ("tile_rows", C.c_int32), ("tile_planes", C.c_int32),
        ("t_e_ev", C.c_double), ("ln_lambda", C.c_double), ("r_refl", C.c_double),
        ("r_inel", C.c_double), ("scheme", C.c_int32), ("reserved0", C.c_int32),
    ]


class fk_state(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("t", C.c_double), ("sigma", C.c_double), ("sigma_lo", C.c_double),
        ("g_pe", C.c_double), ("g_see", C.c_double), ("g_top", C.c_double),
        ("emitted", C.c_double), ("loss_v", C.c_double), ("n_total", C.c_double),
        ("resid", C.c_double),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class fk_info(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("dvx", C.c_double), ("dvy", C.c_double), ("dt", C.c_double),
        ("courant_x", C.c_double), ("courant_vy", C.c_double), ("cells", C.c_int64),
        ("tile_rows", C.c_int32), ("tile_planes", C.c_int32), ("block", C.c_int32),
        ("n_tiles", C.c_int32), ("bytes_device", C.c_uint64),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class fk_batch_info_t(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("tile_rows", C.c_int32), ("tile_planes", C.c_int32),
        ("grid", C.c_int32), ("items", C.c_int32), ("lds_bytes", C.c_int64), ("cells", C.c_int64),
        ("schedule", C.c_int32), ("sweep_launches", C.c_int32), ("single_threads", C.c_int32),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_P = C.POINTER
_vp = C.c_void_p
_ctx = C.c_void_p
SIGNATURES = {
    "fk_error_string": (C.c_char_p, [C.c_int]),
    "fk_last_error": (C.c_char_p, [_ctx]),
    "fk_validate": (C.c_int, [_P(fk_params), _P(fk_info)]),
    "fk_create": (C.c_int, [_P(fk_params), _vp, _P(_ctx)]),
    "fk_create_borrowed": (C.c_int, [_P(fk_params), _vp, _vp, _vp, _P(_ctx)]),
    "fk_destroy": (C.c_int, [_ctx]),
    "fk_query": (C.c_int, [_ctx, _P(fk_info)]),
    "fk_step": (C.c_int, [_ctx, C.c_int64]),
    "fk_sync": (C.c_int, [_ctx]),
    "fk_read_f": (C.c_int, [_ctx, _vp, C.c_size_t, C.c_int]),
    "fk_read_state": (C.c_int, [_ctx, _P(fk_state)]),
    "fk_read_field": (C.c_int, [_ctx, _vp, _vp, C.c_int]),
    "fk_read_tables": (C.c_int, [_ctx, _vp, _vp, _vp, _vp]),
    "fk_read_trace": (C.c_int, [_ctx, _P(fk_state), C.c_size_t, _P(C.c_size_t)]),
    "fk_write_state": (C.c_int, [_ctx, _vp, C.c_int, C.c_double, C.c_double, C.c_int64]),
    "fk_saturated": (C.c_int, [_ctx, C.c_double, C.c_double, _P(C.c_int)]),
    "fk_saturation_check": (C.c_int, [_P(fk_state), C.c_size_t, C.c_double, C.c_double, _P(C.c_int)]),
    "fk_fn_current": (C.c_int, [C.c_double, C.c_double, C.c_double, _P(C.c_double)]),
    "fk_sigma_along": (C.c_int, [_P(fk_state), C.c_size_t, C.c_double, C.c_double, _P(C.c_double), C.c_size_t,
                                 _P(C.c_double)]),
    "fk_set_profiling": (C.c_int, [_ctx, C.c_int]),
    "fk_kernel_times": (C.c_int, [_ctx, _P(C.c_double), _P(C.c_int64), _P(C.c_double), _P(C.c_int64)]),
    "fk_autotune": (C.c_int, [_ctx, C.c_int, _P(fk_info)]),
    "fk_step_noalloc": (C.c_int, [_P(fk_params), _vp, _vp, _vp, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                  _vp, _vp]),
    "fk_batch_create": (C.c_int, [_P(fk_params), C.c_int, _vp, C.c_int, _P(_vp)]),
    "fk_batch_destroy": (C.c_int, [_vp]),
    "fk_batch_step": (C.c_int, [_vp, C.c_int64]),
    "fk_batch_sync": (C.c_int, [_vp, _P(C.c_int)]),
    "fk_batch_get": (C.c_int, [_vp, C.c_int, _P(_ctx)]),
    "fk_batch_info": (C.c_int, [_vp, _P(fk_batch_info_t)]),
    "fk_batch_last_error": (C.c_char_p, [_vp]),
    "fk_read_profile": (C.c_int, [_ctx, C.c_int, _vp, C.c_int]),
    "fk_warm_start": (C.c_int, [_ctx, _vp, C.c_int, C.c_int, C.c_double, C.c_int64]),
    "fk_batch_retire": (C.c_int, [_vp, _P(C.c_int), C.c_int]),
    "fk_mlp_create": (C.c_int, [C.c_int, _P(C.c_int32), C.c_int, _vp, _P(_vp)]),
    "fk_mlp_destroy": (C.c_int, [_vp]),
    "fk_mlp_last_error": (C.c_char_p, [_vp]),
    "fk_mlp_num_params": (C.c_int, [_vp, _P(C.c_int64)]),
    "fk_mlp_set_params": (C.c_int, [_vp, _vp, C.c_int]),
    "fk_mlp_get_params": (C.c_int, [_vp, _vp, C.c_int]),
    "fk_mlp_get_grads": (C.c_int, [_vp, _vp, C.c_int]),
    "fk_mlp_forward": (C.c_int, [_vp, _vp, C.c_int, _vp]),
    "fk_mlp_backward": (C.c_int, [_vp, _vp, C.c_int, _P(C.c_float)]),
    "fk_mlp_adamw": (C.c_int, [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64]),
    "fk_mlp_train_step": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int64]),
    "fk_mlp_take_loss": (C.c_int, [_vp, _P(C.c_double), _P(C.c_int64)]),
    "fk_mlp_sync": (C.c_int, [_vp]),
}
for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


class FlashkinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{fk_error_string(code).decode()} ({code}): {msg}")
        self.code = code


def check(code, ctx=None):
    if code != OK:
        raise FlashkinError(code, (fk_last_error(ctx) or b"").decode())
    return code


PARAM_KEYS = ("nx", "nvx", "nvy", "length", "vmax_x", "vmax_y", "dt", "cfl", "ey", "delta_max",
              "a_max_ev", "ks", "t_se_ev", "j_src", "x_src_lo", "x_src_hi", "t_src_ev",
              "emission_norm", "physics_mask", "ex_external", "t_e_ev", "ln_lambda", "r_refl", "r_inel",
              "scheme")
# keys a dictionary may leave out: the paper's values (collision parameters),
# no reflection, the paper's first-order scheme
OPTIONAL_KEYS = {"t_e_ev": 2.0, "ln_lambda": 10.0, "r_refl": 0.0, "r_inel": 0.0, "scheme": 0}


def make_params(cfg, dtype="f32", trace_stride=1, trace_cap=4096, tile_rows=0, tile_planes=0):
    """fk_params from a workload dictionary (keys as in ``workloads``)."""
    p = fk_params()
    p.struct_size = C.sizeof(fk_params)
    p.abi_version = ABI_VERSION
    for k in PARAM_KEYS:
        setattr(p, "length_m" if k == "length" else k, cfg[k] if k in cfg else OPTIONAL_KEYS[k])
    p.dtype = F32 if dtype in ("f32", F32) else F64
    p.trace_stride = trace_stride
    p.trace_cap = trace_cap
    p.tile_rows = tile_rows
    p.tile_planes = tile_planes
    return p


def validate(params):
    info = fk_info()
    check(fk_validate(C.byref(params), C.byref(info)))
    return info.as_dict()


def saturation_check(records, window_s, rtol):
    arr = (fk_state * len(records))(*records)
    out = C.c_int(0)
    check(fk_saturation_check(arr, len(records), window_s, rtol, C.byref(out)))
    return bool(out.value)


def fn_current(e_field, phi_ev, beta=1.0):
    """Eq 6: field-emission current density (A/m^2) at junction field
    beta * |e_field| and work function phi_ev (eV)."""
    out = C.c_double(0.0)
    check(fk_fn_current(float(e_field), float(phi_ev), float(beta), C.byref(out)))
    return out.value


def _as_states(records):
    out = (fk_state * len(records))()
    for m, r in enumerate(records):
        if isinstance(r, fk_state):
            out[m] = r
        else:
            for name, _ in fk_state._fields_:
                setattr(out[m], name, r.get(name, 0))
    return out


def sigma_along(records, v_seea, t, y):
    """sigma(y, t) along the insulator from a 1D trace (fk_sigma_along):
    records are fk_state or dictionaries of its fields, y positions in m."""
    arr = _as_states(records)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty_like(y)
    P = C.POINTER(C.c_double)
    check(fk_sigma_along(arr, len(records), float(v_seea), float(t), y.ctypes.data_as(P), y.size,
                         out.ctypes.data_as(P)))
    return out


class Solver:
    """One context.  ``stream`` is a hipStream_t as an int (e.g.
    ``torch.cuda.current_stream().cuda_stream``) or None for the null stream."""

    def __init__(self, cfg, dtype="f32", stream=None, borrowed=None, **kw):
        self.params = make_params(cfg, dtype, **kw)
        self.np_dtype = np.float32 if self.params.dtype == F32 else np.float64
        h = _ctx()
        if borrowed is None:
            check(fk_create(C.byref(self.params), stream, C.byref(h)))
        else:
            check(fk_create_borrowed(C.byref(self.params), stream, borrowed[0], borrowed[1], C.byref(h)))
        self._h = h
        info = fk_info()
        check(fk_query(self._h, C.byref(info)), self._h)
        self.info = info.as_dict()
        self.shape = (cfg["nx"], cfg["nvx"], cfg["nvy"])
        self.dt = self.info["dt"]

    def close(self):
        if getattr(self, "_h", None):
            fk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _chk(self, code):
        return check(code, self._h)

    def step(self, n=1):
        self._chk(fk_step(self._h, int(n)))

    def sync(self):
        self._chk(fk_sync(self._h))

    def f(self):
        out = np.empty(self.shape, dtype=self.np_dtype)
        self._chk(fk_read_f(self._h, out.ctypes.data, out.nbytes, 0))
        return out

    def f_to_device(self, ptr, nbytes):
        self._chk(fk_read_f(self._h, ptr, nbytes, 1))

    def state(self):
        s = fk_state()
        self._chk(fk_read_state(self._h, C.byref(s)))
        return s.as_dict()

    def field(self):
        ex = np.empty(self.shape[0])
        ne = np.empty(self.shape[0])
        self._chk(fk_read_field(self._h, ex.ctypes.data, ne.ctypes.data, 0))
        return ex, ne

    def tables(self):
        nv = self.shape[1] * self.shape[2]
        d, g, s = np.empty(nv), np.empty(nv), np.empty(nv)
        w = np.empty(self.shape[0])
        self._chk(fk_read_tables(self._h, d.ctypes.data, g.ctypes.data, s.ctypes.data, w.ctypes.data))
        v = self.shape[1:]
        return dict(delta=d.reshape(v), ghat=g.reshape(v), fsrc=s.reshape(v), wband=w)

    def trace(self, cap=1 << 20):
        buf = (fk_state * cap)()
        n = C.c_size_t(0)
        rc = fk_read_trace(self._h, buf, cap, C.byref(n))
        if rc not in (OK, E_STATE):
            self._chk(rc)
        return [buf[m].as_dict() for m in range(n.value)], rc == E_STATE

    def write_state(self, f=None, sigma=0.0, sigma_lo=0.0, step=0, device_ptr=None):
        if device_ptr is not None:
            self._chk(fk_write_state(self._h, device_ptr, 1, sigma, sigma_lo, int(step)))
        elif f is None:
            self._chk(fk_write_state(self._h, None, 0, sigma, sigma_lo, int(step)))
        else:
            a = np.ascontiguousarray(f, dtype=self.np_dtype).reshape(self.shape)
            self._chk(fk_write_state(self._h, a.ctypes.data, 0, sigma, sigma_lo, int(step)))

    def saturated(self, window_s=50e-12, rtol=1e-3):
        out = C.c_int(0)
        self._chk(fk_saturated(self._h, window_s, rtol, C.byref(out)))
        return bool(out.value)

    def profile(self, npts=256):
        out = np.empty(npts)
        self._chk(fk_read_profile(self._h, int(npts), out.ctypes.data, 0))
        return out

    def warm_start(self, profile, t_ev, step=0):
        a = np.ascontiguousarray(profile, dtype=np.float64)
        self._chk(fk_warm_start(self._h, a.ctypes.data, a.size, 0, float(t_ev), int(step)))

    def set_profiling(self, on=True, every=1):
        self._chk(fk_set_profiling(self._h, int(every) if on else 0))

    def autotune(self, trial_steps=16):
        info = fk_info()
        self._chk(fk_autotune(self._h, int(trial_steps), C.byref(info)))
        self.info = info.as_dict()
        return self.info

    def kernel_times(self):
        a, b = C.c_double(), C.c_double()
        na, nb = C.c_int64(), C.c_int64()
        self._chk(fk_kernel_times(self._h, C.byref(a), C.byref(na), C.byref(b), C.byref(nb)))
        return dict(sweep_ms=a.value, sweep_n=na.value, field_ms=b.value, field_n=nb.value)


class View(Solver):
    """Non-owning handle of one instance of a Batch (read and write state)."""

    def __init__(self, handle, cfg, dtype):
        self._h = handle
        self.params = make_params(cfg, dtype)
        self.np_dtype = np.float32
        info = fk_info()
        check(fk_query(self._h, C.byref(info)), self._h)
        self.info = info.as_dict()
        self.shape = (cfg["nx"], cfg["nvx"], cfg["nvy"])
        self.dt = self.info["dt"]

    def close(self):
        self._h = None


class Batch:
    """Independent FP32 instances stepped together by persistent launches
    (fk_batch_*): one sweep launch per step by default, split launches with
    ``single_launch=False``, or whatever ``autotune`` finds fastest."""

    def __init__(self, cfgs, stream=None, autotune=False, trace_stride=1, single_launch=True, single_threads=256,
                 **kw):
        self.cfgs = list(cfgs)
        strides = trace_stride if isinstance(trace_stride, (list, tuple)) else [trace_stride] * len(self.cfgs)
        arr = (fk_params * len(self.cfgs))(*[make_params(c, "f32", trace_stride=st, **kw)
                                             for c, st in zip(self.cfgs, strides)])
        h = _vp()
        mode = 1 if autotune else ((3 if single_threads == 192 else 2) if single_launch else 0)
        rc = fk_batch_create(arr, len(self.cfgs), stream, mode, C.byref(h))
        if rc != OK:
            raise FlashkinError(rc, (fk_batch_last_error(None) or b"").decode())
        self._h = h
        self.views = []
        for i, c in enumerate(self.cfgs):
            v = _ctx()
            self._chk(fk_batch_get(self._h, i, C.byref(v)))
            self.views.append(View(v, c, "f32"))

    def _chk(self, rc):
        if rc != OK:
            raise FlashkinError(rc, (fk_batch_last_error(self._h) or b"").decode())
        return rc

    def step(self, n=1):
        self._chk(fk_batch_step(self._h, int(n)))

    def sync(self):
        """Wait; raises FlashkinError with ``.instance`` set to the first
        flagged active instance."""
        bad = C.c_int(-1)
        rc = fk_batch_sync(self._h, C.byref(bad))
        if rc != OK:
            err = FlashkinError(rc, (fk_batch_last_error(self._h) or b"").decode())
            err.instance = bad.value
            raise err

    def retire(self, idx):
        idx = list(idx)
        arr = (C.c_int * max(1, len(idx)))(*idx)
        self._chk(fk_batch_retire(self._h, arr, len(idx)))

    def info(self):
        out = fk_batch_info_t()
        self._chk(fk_batch_info(self._h, C.byref(out)))
        return out.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            for v in self.views:
                v.close()
            fk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class MLP:
    """The surrogate network on the GPU (fk_mlp_*).  Inputs, outputs and
    targets are device pointers (e.g. torch tensor data_ptr())."""

    def __init__(self, dims, max_batch=256, stream=None):
        self.dims = list(dims)
        arr = (C.c_int32 * len(self.dims))(*self.dims)
        h = _vp()
        rc = fk_mlp_create(len(self.dims) - 1, arr, int(max_batch), stream, C.byref(h))
        if rc != OK:
            raise FlashkinError(rc, (fk_mlp_last_error(None) or b"").decode())
        self._h = h
        n = C.c_int64()
        self._chk(fk_mlp_num_params(self._h, C.byref(n)))
        self.n_params = n.value

    def _chk(self, rc):
        if rc != OK:
            raise FlashkinError(rc, (fk_mlp_last_error(self._h) or b"").decode())

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params
        self._chk(fk_mlp_set_params(self._h, a.ctypes.data, 0))

    def params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._chk(fk_mlp_get_params(self._h, out.ctypes.data, 0))
        return out

    def grads(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._chk(fk_mlp_get_grads(self._h, out.ctypes.data, 0))
        return out

    def forward(self, x_ptr, m, y_ptr=None):
        self._chk(fk_mlp_forward(self._h, x_ptr, int(m), y_ptr))

    def backward(self, t_ptr, m, read_loss=True):
        """Gradients for the last forward; returns the loss (a stream
        synchronisation) unless read_loss is False."""
        if not read_loss:
            self._chk(fk_mlp_backward(self._h, t_ptr, int(m), None))
            return None
        loss = C.c_float()
        self._chk(fk_mlp_backward(self._h, t_ptr, int(m), C.byref(loss)))
        return loss.value

    def take_loss(self):
        """(mean loss, number of steps) since the last take."""
        mean, count = C.c_double(), C.c_int64()
        self._chk(fk_mlp_take_loss(self._h, C.byref(mean), C.byref(count)))
        return mean.value, count.value

    def adamw(self, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4):
        self._chk(fk_mlp_adamw(self._h, lr, beta1, beta2, eps, weight_decay, int(step)))

    def train_step(self, x_ptr, t_ptr, m, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4):
        """Forward, loss, gradients and AdamW on one batch (fk_mlp_train_step)."""
        self._chk(fk_mlp_train_step(self._h, x_ptr, t_ptr, int(m), lr, beta1, beta2, eps, weight_decay, int(step)))

    def sync(self):
        self._chk(fk_mlp_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            fk_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
