"""The C-ABI library loads, exports every function include/flashkin.h
declares, and its host-only logic (parameter validation, launch shape,
saturation test) behaves as documented.  No GPU is touched."""
import ctypes as C
import os
import re

import pytest

from paper_2303_14119_amd import flashkin as fk
from paper_2303_14119_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "flashkin.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 19
    lib = C.CDLL(fk.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(declared_functions()) <= set(fk.SIGNATURES)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_validate_workloads(dtype):
    for cfg in (W.c0(), W.c1(), W.c4(), W.paper_default()):
        info = fk.validate(fk.make_params(cfg, dtype))
        assert info["cells"] == cfg["nx"] * cfg["nvx"] * cfg["nvy"]
        assert 0 < info["courant_x"] <= 1 and 0 <= info["courant_vy"] <= 1
        assert info["block"] % 64 == 0 and info["block"] >= cfg["nvy"]


def test_default_time_step_matches_the_cfl_rule():
    info = fk.validate(fk.make_params(W.c0(), "f64"))
    assert info["dt"] == pytest.approx(3.7489257835957387e-13, rel=1e-15)
    assert info["courant_x"] == pytest.approx(0.8859375, rel=1e-12)
    assert info["courant_vy"] == pytest.approx(0.5625, rel=1e-12)


def bad(**kw):
    cfg = W.c0()
    extra = {k: kw.pop(k) for k in list(kw) if k in ("tile_rows", "tile_planes", "trace_cap", "trace_stride")}
    cfg.update(kw)
    p = fk.make_params(cfg, "f32", **extra)
    return fk.fk_validate(C.byref(p), None)


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), fk.E_INVALID), (dict(nvy=1025), fk.E_INVALID), (dict(length=-1.0), fk.E_INVALID),
    (dict(t_se_ev=0.0), fk.E_INVALID), (dict(x_src_lo=2e-5, x_src_hi=1e-5), fk.E_INVALID),
    (dict(physics_mask=256), fk.E_INVALID), (dict(emission_norm=2), fk.E_INVALID),
    (dict(physics_mask=W.ALL | W.BGK, t_e_ev=0.0), fk.E_INVALID),
    (dict(physics_mask=W.BGK, ln_lambda=0.0), fk.E_INVALID),
    (dict(physics_mask=W.BGK, t_e_ev=float("inf")), fk.E_INVALID),
    (dict(r_refl=-0.1), fk.E_INVALID), (dict(r_refl=1.5), fk.E_INVALID), (dict(r_refl=float("nan")), fk.E_INVALID),
    (dict(r_inel=-0.1), fk.E_INVALID), (dict(r_refl=0.6, r_inel=0.5), fk.E_INVALID),
    (dict(r_inel=float("nan")), fk.E_INVALID), (dict(scheme=2), fk.E_INVALID), (dict(scheme=-1), fk.E_INVALID),
    (dict(scheme=1, physics_mask=W.ALL | W.BGK), fk.E_INVALID),
    (dict(tile_rows=3), fk.E_INVALID), (dict(trace_cap=0), fk.E_INVALID),
    (dict(dt=1e-11), fk.E_CFL), (dict(ey=-1e9, dt=3e-13), fk.E_CFL),
])
def test_validate_rejects(kw, code):
    assert bad(**kw) == code
    assert fk.fk_last_error(None)


@pytest.mark.parametrize("nx", [4, 64, 2048])
@pytest.mark.parametrize("mask", [W.ALL, W.ALL | W.BGK])
def test_width_limits_per_precision(nx, mask):
    """nvy up to 1024 in FP32, up to 960 in FP64 (the tile's v_y exchange
    must fit in 64 KB of LDS), at any x extent and with the collision term
    (the default x run shrinks to as few as 4 planes to leave room)."""
    for nvy, dtype, code in ((1024, "f32", fk.OK), (960, "f64", fk.OK), (1024, "f64", fk.E_INVALID)):
        cfg = W.config(nx=nx, nvx=6, nvy=nvy, length=1e-5 * nx / 4, ey=-4e6, delta_max=2.5, a_max_ev=400.0,
                       cfl=0.8, physics_mask=mask)
        p = fk.make_params(cfg, dtype)
        assert fk.fk_validate(C.byref(p), None) == code, (nvy, dtype)


def test_new_physics_parameters_are_accepted():
    """The inelastic share, the no-space-charge bit and the second-order
    scheme validate within their ranges."""
    for kw in (dict(r_refl=0.4, r_inel=0.6), dict(r_inel=1.0), dict(physics_mask=W.ALL | W.NOSC),
               dict(scheme=1), dict(scheme=1, r_refl=0.2, r_inel=0.1)):
        for dtype in ("f32", "f64"):
            p = fk.make_params(dict(W.c0(), **kw), dtype)
            assert fk.fk_validate(C.byref(p), None) == fk.OK, kw


def test_tile_rows_rule_and_limits():
    """The library's tile height (host rule): 8 rows up to 256 FP32 lanes,
    12 for 320-512 lanes when N_vx is a multiple of 24, else 16; 4 in FP64.
    12 and 16 rows are FP32 only and need N_vy <= 512."""
    def rows(nvx, nvy, dtype="f32", ti=0):
        cfg = W.config(nx=64, nvx=nvx, nvy=nvy, length=1e-4, ey=-4e6, delta_max=2.5, a_max_ev=400.0, cfl=0.8)
        p = fk.make_params(cfg, dtype, tile_rows=ti)
        rc = fk.fk_validate(C.byref(p), None)
        return fk.validate(p)["tile_rows"] if rc == fk.OK else rc
    assert rows(256, 256) == 8
    assert rows(384, 384) == 12 and rows(96, 400) == 12
    assert rows(448, 448) == 16 and rows(320, 320) == 16 and rows(100, 384) == 16
    assert rows(384, 384, "f64") == 4
    assert rows(48, 200, ti=12) == 12
    assert rows(48, 200, "f64", ti=12) == fk.E_INVALID
    assert rows(48, 600, ti=12) == fk.E_INVALID and rows(48, 600, ti=16) == fk.E_INVALID
    assert rows(48, 200, ti=6) == fk.E_INVALID


def test_struct_size_and_version_are_checked():
    p = fk.make_params(W.c0())
    p.struct_size -= 8
    assert fk.fk_validate(C.byref(p), None) == fk.E_INVALID
    p = fk.make_params(W.c0())
    p.abi_version = 99
    assert fk.fk_validate(C.byref(p), None) == fk.E_INVALID


def rec(t, sigma, gpe, gsee):
    r = fk.fk_state()
    r.t, r.sigma, r.g_pe, r.g_see = t, sigma, gpe, gsee
    return r


def test_saturation_check():
    """Section 2: converged when sigma and the fluxes change by less than the
    tolerance over the window."""
    flat = [rec(i * 1e-12, 1e-5, 1e24, 1e24) for i in range(200)]
    assert fk.saturation_check(flat, 50e-12, 1e-3)
    assert not fk.saturation_check(flat[:40], 50e-12, 1e-3)        # shorter than the window
    rising = [rec(i * 1e-12, 1e-5 * (1 + 1e-4 * i), 1e24, 1e24) for i in range(200)]
    assert not fk.saturation_check(rising, 50e-12, 1e-3)             # 0.5% over the window
    assert fk.saturation_check(rising, 50e-12, 1e-2)
    empty = [rec(i * 1e-12, 0.0, 0.0, 0.0) for i in range(200)]
    assert not fk.saturation_check(empty, 50e-12, 1e-3)              # nothing has arrived yet


def test_batch_rejects_before_touching_the_gpu():
    """Batched instances are FP32 with nvy <= 256 and the mode is 0 .. 3;
    these are checked on the host before any device call."""
    good = W.config(nx=16, nvx=16, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
    wide = dict(good, nvy=300)
    for cfgs, dtype in (([good], "f64"), ([good, wide], "f32")):
        arr = (fk.fk_params * len(cfgs))(*[fk.make_params(c, dtype) for c in cfgs])
        h = C.c_void_p()
        assert fk.fk_batch_create(arr, len(cfgs), None, 0, C.byref(h)) == fk.E_INVALID
        assert not h.value
        assert fk.fk_batch_last_error(None)
    arr = (fk.fk_params * 1)(fk.make_params(dict(good, scheme=1), "f32"))
    assert fk.fk_batch_create(arr, 1, None, 0, C.byref(C.c_void_p())) == fk.E_INVALID
    arr = (fk.fk_params * 1)(fk.make_params(good, "f32"))
    assert fk.fk_batch_create(arr, 0, None, 0, C.byref(C.c_void_p())) == fk.E_INVALID
    assert fk.fk_batch_create(arr, 1, None, 4, C.byref(C.c_void_p())) == fk.E_INVALID
    assert fk.fk_batch_create(arr, 1, None, -1, C.byref(C.c_void_p())) == fk.E_INVALID


def test_collision_term_is_opt_in_and_costs_lds_only_when_on():
    """The BGK bit is valid with a temperature and Coulomb logarithm; the
    parameters are ignored without it, and its per-wave coefficient table
    is the only change to the launch shape."""
    cfg = W.c1()
    plain = fk.validate(fk.make_params(dict(cfg, t_e_ev=0.0, ln_lambda=0.0), "f32"))
    on = fk.validate(fk.make_params(dict(cfg, physics_mask=W.ALL | W.BGK), "f32"))
    assert plain["tile_rows"] == on["tile_rows"] and plain["block"] == on["block"]
    assert on["bytes_device"] == plain["bytes_device"]
    # the widest FP32 tiles still fit with the larger table
    wide = fk.validate(fk.make_params(dict(W.c4(), physics_mask=W.ALL | W.BGK), "f32"))
    assert wide["tile_rows"] == 12
