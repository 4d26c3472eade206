"""Parity of the electron-electron collision term (FK_PHYS_BGK, Eq 3-5)
with the FP64 CPU oracle (GPU).

States are scaled so that nu_ee dt is 1e-3 .. 2e-2 per step, large enough
that the term's contribution to f is far above each precision's tolerance.
At such densities the self field would break the v_x Courant limit, so the
runs with every other part of the step on replace it by a uniform E_x; one
FP64 case keeps the self field at an ordinary density (the term is then
small per step but still far above the FP64 tolerance).

Tolerances as for the other parity tests: FP64 relative L2 <= 1e-12,
FP32 <= 1e-5 (f) and 1e-5 (sigma and fluxes).
"""
import os

import numpy as np
import pytest

from oracle.solver import Oracle, nu_ee, set_threads
from paper_2303_14119_amd import workloads as W

pytestmark = pytest.mark.gpu

set_threads(min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def fk():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14119_amd import flashkin
    return flashkin


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def compare_state(gpu, orc, tol):
    for q in ("g_pe", "g_see", "g_top", "n_total"):
        assert rel(gpu[q], orc[q]) <= tol or abs(gpu[q] - orc[q]) <= 1e-30, (q, gpu[q], orc[q])
    s = gpu["sigma"] + gpu["sigma_lo"]
    assert rel(s, orc["sigma"]) <= tol or abs(s - orc["sigma"]) <= 1e-30, ("sigma", s, orc["sigma"])


def collisional_state(cfg, seed, nudt):
    """The seeded random state with each plane scaled to a density where
    nu_ee dt lies between nudt and 2 nudt (planes differ)."""
    nx, nvx, nvy = cfg["nx"], cfg["nvx"], cfg["nvy"]
    f = W.random_state((nx, nvx, nvy), seed=seed, scale=1.0)
    o = Oracle(cfg)
    dv2 = (2 * cfg["vmax_x"] / nvx) * (2 * cfg["vmax_y"] / nvy)
    per_n = nu_ee(1.0, cfg["t_e_ev"], cfg["ln_lambda"]) * o.dt
    o.close()
    target = nudt * (1.0 + np.arange(nx) / max(1, nx - 1)) / per_n
    return f * (target / (f.sum(axis=(1, 2)) * dv2))[:, None, None]


def run_pair(fk, cfg, dtype, f0, steps, sigma0=0.0, tile_rows=0):
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    o = Oracle(cfg)
    o.set_state(f0, sigma0, 0)
    with fk.Solver(cfg, dtype, tile_rows=tile_rows) as s:
        s.write_state(f0, sigma0, 0.0, 0)
        o.step(steps)
        s.step(steps)
        s.sync()
        out = s.f(), s.state(), s.info
    return out, (o.f(), o.record(), o.nu_dt_max())


ALONE = [(3, 24, 20), (7, 37, 45), (5, 9, 130), (4, 16, 384)]


@pytest.mark.parametrize("shape", ALONE, ids=[f"{s[0]}x{s[1]}x{s[2]}" for s in ALONE])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_collisions_alone(fk, shape, dtype):
    nx, nvx, nvy = shape
    cfg = W.config(nx=nx, nvx=nvx, nvy=nvy, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                   dt=1e-13, physics_mask=W.BGK, t_e_ev=40.0, ln_lambda=10.0, j_src=0.0)
    f0 = collisional_state(cfg, 11 * nx + nvy, 1e-2)
    (g, gst, _), (r, rst, nudt) = run_pair(fk, cfg, dtype, f0, 12)
    assert nudt > 5e-3
    # the term changed f by far more than the tolerance
    assert rel_l2(r, f0) > 1e-2
    assert rel_l2(g, r) <= (1e-12 if dtype == "f64" else 1e-5)
    assert rel(gst["n_total"], rst["n_total"]) <= (1e-13 if dtype == "f64" else 1e-5)


FULL = [
    # (nx, nvx, nvy, tile_rows); tile_rows 0 = the library's choice
    (37, 29, 45, 0),
    (13, 33, 70, 0),
    (21, 17, 131, 0),
    (9, 40, 64, 4),
    (12, 48, 100, 8),
    (5, 9, 700, 0),
    (23, 48, 100, 12),
    (13, 45, 384, 16),
    (17, 41, 330, 12),
    # the widest blocks (FP64 up to 960 lanes) and degenerate velocity grids
    (4, 7, 960, 0),
    (3, 5, 1024, 4),
    (6, 1, 9, 0),
    (4, 2, 2, 0),
]


@pytest.mark.parametrize("case", FULL, ids=[f"{c[0]}x{c[1]}x{c[2]}-ti{c[3]}" for c in FULL])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_step_with_collisions(fk, case, dtype):
    nx, nvx, nvy, ti = case
    if dtype == "f64" and ti in (12, 16):
        pytest.skip("12- and 16-row tiles are FP32 only")
    if dtype == "f64" and nvy > 960:
        pytest.skip("FP64 v_y blocks end at 960 lanes")
    cfg = W.config(nx=nx, nvx=nvx, nvy=nvy, length=nx * 2e-6, ey=-4e6, delta_max=2.5, a_max_ev=400.0,
                   physics_mask=(W.ALL & ~W.SELF) | W.BGK, ex_external=1e5, x_src_lo=1e-6, x_src_hi=5e-6,
                   j_src=1e7, cfl=0.8, t_e_ev=40.0, ln_lambda=10.0)
    f0 = collisional_state(cfg, 7 * nx + nvy, 2e-3)
    (g, gst, info), (r, rst, nudt) = run_pair(fk, cfg, dtype, f0, 20, sigma0=3e-6, tile_rows=ti)
    if ti:
        assert info["tile_rows"] == ti
    assert nudt > 1e-3
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(g, r) <= tol
    compare_state(gst, rst, 1e-11 if dtype == "f64" else 1e-5)
    assert abs(gst["resid"]) <= (1e-12 if dtype == "f64" else 1e-5) * gst["n_total"]


def test_collisions_with_the_self_field_fp64(fk):
    """Every part of the step, collisions included, at an ordinary density."""
    cfg = W.config(nx=37, nvx=29, nvy=45, length=37 * 2e-6, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                   physics_mask=W.ALL | W.BGK, x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8,
                   t_e_ev=2.0, ln_lambda=10.0)
    f0 = W.random_state((37, 29, 45), seed=5, scale=1e3)
    (g, gst, _), (r, rst, nudt) = run_pair(fk, cfg, "f64", f0, 25, sigma0=3e-6)
    assert nudt > 1e-9
    # with the term switched off the oracle lands measurably elsewhere
    o = Oracle(dict(cfg, physics_mask=W.ALL))
    o.set_state(f0, 3e-6, 0)
    o.step(25)
    assert rel_l2(o.f(), r) > 1e-8
    assert rel_l2(g, r) <= 1e-12
    compare_state(gst, rst, 1e-11)


def test_relaxation_number_above_one_is_flagged(fk):
    """nu_ee dt > 1 makes the explicit relaxation overshoot: the library
    flags it like a Courant number above one (sticky until write_state)."""
    cfg = W.config(nx=4, nvx=16, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                   dt=1e-13, physics_mask=W.BGK, t_e_ev=40.0, ln_lambda=10.0, j_src=0.0)
    hot = collisional_state(cfg, 3, 3.0)
    calm = collisional_state(cfg, 3, 1e-3)
    with fk.Solver(cfg, "f64") as s:
        s.write_state(hot, 0.0, 0.0, 0)
        with pytest.raises(fk.FlashkinError) as e:
            s.sync()
        assert e.value.code == fk.E_CFL
        s.write_state(calm, 0.0, 0.0, 0)
        s.step(3)
        s.sync()


def test_collisions_in_a_batch(fk):
    """Batch members with and without the term against the oracle (the
    batch runs the sweep variant with it; members without it skip it)."""
    rng = np.random.default_rng(31)
    cfgs, states = [], []
    for m in range(4):
        nv = int(rng.integers(24, 200))
        mask = (W.ALL & ~W.SELF) | (W.BGK if m != 1 else 0)
        c = W.config(nx=int(rng.integers(20, 90)), nvx=nv, nvy=nv, length=float(rng.uniform(1e-4, 5e-4)),
                     ey=-float(rng.uniform(2e6, 8e6)), delta_max=2.5, a_max_ev=400.0, j_src=1e5,
                     physics_mask=mask, ex_external=1e5, t_e_ev=40.0, ln_lambda=10.0)
        cfgs.append(c)
        states.append(collisional_state(dict(c, physics_mask=c["physics_mask"] | W.BGK), 40 + m, 2e-3)
                      .astype(np.float32))
    steps = 20
    with fk.Batch(cfgs) as b:
        for v, f0 in zip(b.views, states):
            v.write_state(f0, 2e-6, 0.0, 0)
        b.step(steps)
        b.sync()
        for m, (c, v, f0) in enumerate(zip(cfgs, b.views, states)):
            o = Oracle(c)
            o.set_state(f0.astype(np.float64), 2e-6, 0)
            o.step(steps)
            if m != 1:
                assert o.nu_dt_max() > 1e-3
            st, orc = v.state(), o.record()
            assert rel_l2(v.f(), o.f()) < 1e-5, m
            compare_state(st, orc, 1e-5)
