"""GPU parity of the second-order scheme (FK_SCHEME_LIMITED2) with the FP64
oracle's scheme 1: minmod-limited flux-form sweeps, the split order reversed
on odd steps.  The library runs a step's sweep as one fused launch (the
workgroups of the edge and mixed-direction tiles first, then those of the
tiles with a fast body): forward bodies on even steps, reversed bodies on
odd ones, two-cell halos.

Cases cover 4- and 8-row tiles, short x chunks (so chunk boundaries and the
halo planes of the reversed body are exercised), ragged v_x and v_y, odd
grids with a v = 0 row, wall reflection of both kinds, the field without
space charge, the continuum emission prefactor, parts of the step switched
off, a start on an odd step, and the bench-size grid.

Tolerances: FP64 relative L2 <= 1e-12 (rounding order only: fused
multiply-adds and sums); FP32 <= 1e-5 after 25 steps of a random state;
sigma and the fluxes <= 1e-11 (FP64) / 1e-5 (FP32).
"""
import os

import numpy as np
import pytest

from oracle.solver import Oracle, set_threads
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


CASES = [
    # (nx, nvx, nvy, tile_rows, tile_planes, extra)
    (37, 29, 45, 0, 0, {}),
    (37, 29, 45, 4, 5, {}),
    (21, 17, 131, 8, 4, dict(r_refl=0.3, r_inel=0.2)),
    (13, 33, 70, 0, 6, dict(emission_norm=1, ex_external=3e5, ey=-2e6)),
    (40, 48, 100, 8, 16, dict(physics_mask=W.ALL | W.NOSC)),
    (9, 16, 64, 4, 4, dict(physics_mask=W.X | W.VX | W.SELF | W.SEE, ey=0.0)),
    (64, 40, 257, 4, 0, dict(physics_mask=W.VX | W.VY, ex_external=2e6)),
    (5, 7, 3, 0, 0, {}),
    (1, 4, 1, 0, 0, {}),
    (30, 24, 200, 8, 7, dict(physics_mask=W.X | W.SEE | W.SRC)),
    (4, 1, 9, 0, 0, {}),
    (3, 2, 2, 4, 4, dict(r_refl=0.2)),
]


@pytest.mark.parametrize("start", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}-ti{c[3]}-kc{c[4]}-{i}" for i, c in enumerate(CASES)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_state_matches_oracle(fk, case, dtype, start):
    nx, nvx, nvy, ti, kc, extra = case
    cfg = W.config(nx=nx, nvx=nvx, nvy=nvy, length=nx * 2e-6, ey=-4e6, delta_max=2.5, a_max_ev=400.0,
                   x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8, scheme=1)
    cfg.update(extra)
    f0 = W.random_state((nx, nvx, nvy), seed=11 * nx + nvy, scale=1e3)
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    o = Oracle(cfg)
    o.set_state(f0, 3e-6, start)
    steps = 25
    with fk.Solver(cfg, dtype, tile_rows=ti, tile_planes=kc) as s:
        if ti:
            assert s.info["tile_rows"] == ti
        s.write_state(f0, 3e-6, 0.0, start)
        o.step(steps)
        s.step(steps)
        s.sync()
        g, st = s.f(), s.state()
    r, orc = o.f(), o.record()
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(g, r) <= tol
    tol_s = 1e-11 if dtype == "f64" else 1e-5
    for q in ("g_pe", "g_see", "g_top", "emitted", "n_total"):
        assert rel(st[q], orc[q]) <= tol_s or abs(st[q] - orc[q]) <= 1e-30, q
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= tol_s
    assert abs(st["resid"]) <= (1e-12 if dtype == "f64" else 1e-5) * max(st["n_total"], 1e-300)
    assert st["step"] == start + steps


WIDEST = [("f32", 4, 768), ("f32", 8, 512), ("f64", 4, 384), ("f64", 8, 256)]


@pytest.mark.parametrize("dtype,ti,nvy", WIDEST, ids=[f"{d}-ti{t}-{n}" for d, t, n in WIDEST])
def test_widest_v_y_blocks(fk, dtype, ti, nvy):
    """The widest v_y block each tile height and precision accepts (the
    v_y exchange at its LDS limit), with a ragged last v_x tile and short x
    chunks, from an odd step (reversed bodies first)."""
    cfg = W.config(nx=6, nvx=11, nvy=nvy, length=12e-6, ey=-4e6, delta_max=2.5, a_max_ev=400.0,
                   x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8, scheme=1)
    f0 = W.random_state((6, 11, nvy), seed=nvy + ti, scale=1e3)
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    o = Oracle(cfg)
    o.set_state(f0, 3e-6, 1)
    with fk.Solver(cfg, dtype, tile_rows=ti, tile_planes=4) as s:
        assert s.info["tile_rows"] == ti
        s.write_state(f0, 3e-6, 0.0, 1)
        o.step(20)
        s.step(20)
        s.sync()
        g, st = s.f(), s.state()
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(g, o.f()) <= tol
    assert rel(st["sigma"] + st["sigma_lo"], o.record()["sigma"]) <= (1e-11 if dtype == "f64" else 1e-5)
    with pytest.raises(fk.FlashkinError):
        fk.Solver(dict(cfg, nvy=nvy + 1), dtype, tile_rows=ti)


def test_second_order_differs_from_first_order(fk):
    """The scheme switch takes effect: the same state advanced by the two
    schemes ends apart by far more than rounding."""
    cfg = W.config(nx=37, nvx=29, nvy=45, length=74e-6, ey=-4e6, delta_max=2.5, a_max_ev=400.0, cfl=0.8)
    f0 = W.random_state((37, 29, 45), seed=3, scale=1e3)
    out = []
    for scheme in (0, 1):
        with fk.Solver(dict(cfg, scheme=scheme), "f64") as s:
            s.write_state(f0, 3e-6, 0.0, 0)
            s.step(20)
            out.append(s.f())
    assert rel_l2(out[0], out[1]) > 1e-3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c0_run_with_the_second_order_scheme(fk, dtype):
    """The 128 x 64 x 64 run from f = 0 through the avalanche (1000 steps)
    against the oracle along the trace."""
    cfg = dict(W.c0(), scheme=1)
    o = Oracle(cfg)
    with fk.Solver(cfg, dtype, trace_cap=2048) as s:
        otr = o.step(W.C0_STEPS, trace=True)
        s.step(W.C0_STEPS)
        s.sync()
        gtr, lost = s.trace()
        g, st = s.f(), s.state()
    assert not lost
    tol = 1e-11 if dtype == "f64" else 1e-6
    worst = 0.0
    for gr, r in zip(gtr[1:], otr):
        assert gr["step"] == r["step"]
        if abs(r["sigma"]) > 1e-3 * abs(otr[-1]["sigma"]):
            worst = max(worst, rel(gr["sigma"] + gr["sigma_lo"], r["sigma"]))
    print(dtype, "128x64x64 second order: f", rel_l2(g, o.f()), "worst sigma along the trace", worst)
    assert worst <= tol
    assert rel_l2(g, o.f()) <= (1e-12 if dtype == "f64" else 1e-4)
    orc = o.record()
    for q in ("g_pe", "g_see", "n_total"):
        assert rel(st[q], orc[q]) <= tol, q


def test_graph_replay_equals_direct_launches(fk):
    """Steps replayed from the captured graphs (16 steps from an even step,
    after one direct step when the state is at an odd step) are bitwise the
    same as direct launches with events."""
    cfg = dict(W.c0(), scheme=1)
    f0 = W.random_state((128, 64, 64), seed=5, scale=1e3).astype(np.float32)
    res = []
    for prof in (0, 1):
        with fk.Solver(cfg, "f32") as s:
            s.write_state(f0, 2e-6, 0.0, 3)
            if prof:
                s.set_profiling(True, every=3)
            s.step(37)
            s.sync()
            res.append((s.f(), s.state()))
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1]["sigma"] == res[1][1]["sigma"] and res[0][1]["step"] == 40


def test_bench_size_grid_both_orders(fk):
    """2048 x 256 x 256 (the launch the second-order bench times): a dense
    seeded state and a charged surface, 4 FP32 steps (two of each order)
    against the FP64 oracle."""
    from test_gpu_fullsize import separable_state
    cfg = dict(W.c1(), scheme=1)
    f0 = separable_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=17, scale=2e3)
    o = Oracle(cfg)
    o.set_state(f0.astype(np.float64), 4e-6, 0)
    o.step(4)
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f0, 4e-6, 0.0, 0)
        s.step(4)
        s.sync()
        g, st = s.f(), s.state()
    ref, orc = o.f(), o.record()
    o.close()
    err = rel_l2(g, ref)
    print("2048x256x256 second order, 4 steps: f", err)
    assert err <= 1e-6
    for q in ("g_pe", "g_see", "g_top", "n_total"):
        assert rel(st[q], orc[q]) <= 1e-6, q
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= 1e-6
