"""Parity of the wall reflection (coefficient R_f, fk_params.r_refl) with the
FP64 CPU oracle (GPU).

The reflected part of the emission row is read from the wall cell's mirror
v_x row when the first x chunk of a tile starts, in both sweep bodies; the
field kernel scales the secondary flux by 1 - R_f and leaves the reflected
electrons out of Eq 18.  Shapes cover 4-, 8-, 12- and 16-row tiles, ragged
and inside-split tiles (generic body), odd and even v_x grids and wide v_y
blocks; batches carry the coefficient per instance.

Tolerances as for the other parity tests: FP64 relative L2 <= 1e-12, FP32
<= 1e-5.
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
    # (nx, nvx, nvy, tile_rows, r_refl)
    (37, 29, 45, 0, 0.3),
    (13, 33, 70, 0, 1.0),
    (21, 17, 131, 0, 0.55),
    (9, 40, 64, 4, 0.3),
    (12, 48, 100, 8, 0.8),
    (5, 9, 700, 0, 0.3),
    (23, 48, 100, 12, 0.3),
    (13, 45, 384, 16, 0.6),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}-ti{c[3]}-r{c[4]}" for c in CASES])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reflection_matches_oracle(fk, case, dtype):
    nx, nvx, nvy, ti, rf = case
    if dtype == "f64" and ti in (12, 16):
        pytest.skip("12- and 16-row tiles are FP32 only")
    cfg = W.config(nx=nx, nvx=nvx, nvy=nvy, length=nx * 2e-6, ey=-4e6, delta_max=2.5, a_max_ev=400.0,
                   x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8, r_refl=rf)
    f0 = W.random_state((nx, nvx, nvy), seed=13 * nx + nvy, scale=1e3)
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    o = Oracle(cfg)
    o.set_state(f0, 3e-6, 0)
    # the reflection must matter: the run without it ends elsewhere
    o0 = Oracle(dict(cfg, r_refl=0.0))
    o0.set_state(f0, 3e-6, 0)
    with fk.Solver(cfg, dtype, tile_rows=ti) as s:
        if ti:
            assert s.info["tile_rows"] == ti
        s.write_state(f0, 3e-6, 0.0, 0)
        o.step(25)
        o0.step(25)
        s.step(25)
        s.sync()
        g, st = s.f(), s.state()
    r, orc = o.f(), o.record()
    assert rel_l2(o0.f(), r) > 1e-4
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(g, r) <= tol
    for q in ("g_pe", "g_see", "g_top", "emitted", "n_total"):
        assert rel(st[q], orc[q]) <= (1e-11 if dtype == "f64" else 1e-5) or abs(st[q] - orc[q]) <= 1e-30, q
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= (1e-11 if dtype == "f64" else 1e-5)


def test_reflection_in_a_batch(fk):
    """Batch members with different coefficients against the oracle."""
    rng = np.random.default_rng(21)
    cfgs = []
    for m in range(4):
        nv = int(rng.integers(24, 150))
        cfgs.append(W.config(nx=int(rng.integers(20, 90)), nvx=nv, nvy=nv, length=float(rng.uniform(1e-4, 5e-4)),
                             ey=-float(rng.uniform(2e6, 8e6)), delta_max=2.5, a_max_ev=400.0, j_src=1e5,
                             r_refl=[0.0, 0.25, 0.6, 1.0][m]))
    steps = 40
    states = [W.random_state((c["nx"], c["nvx"], c["nvy"]), seed=m, scale=1e1).astype(np.float32)
              for m, c in enumerate(cfgs)]
    with fk.Batch(cfgs) as b:
        for v, f0 in zip(b.views, states):
            v.write_state(f0, 2e-6, 0.0, 0)
        b.step(steps)
        b.sync()
        for m, (c, v, f0) in enumerate(zip(cfgs, b.views, states)):
            o = Oracle(c)
            o.set_state(f0.astype(np.float64), 2e-6, 0)
            o.step(steps)
            st, orc = v.state(), o.record()
            assert rel_l2(v.f(), o.f()) < 1e-5, m
            for q in ("g_pe", "g_see", "n_total"):
                assert abs(st[q] - orc[q]) <= 1e-5 * abs(orc[q]) + 1e-30, (m, q)
            assert abs(st["sigma"] + st["sigma_lo"] - orc["sigma"]) <= 1e-5 * abs(orc["sigma"]), m


def test_saturated_balance_with_reflection(fk):
    """At saturation sigma stops changing, so by Eq 18 with reflection the
    secondaries plus the reflected electrons balance the primaries:
    Gamma_see / Gamma_pe = 1 - R_f (the paper's default run, R_f = 0.3)."""
    cfg = dict(W.paper_default(), r_refl=0.3)
    with fk.Solver(cfg, "f32", trace_cap=8192, trace_stride=100) as s:
        done = False
        for _ in range(80):
            s.step(5000)
            if s.saturated(50e-12, 1e-3):
                done = True
                break
        st = s.state()
    print("paper default with R_f = 0.3: sigma", st["sigma"] + st["sigma_lo"], "Gsee/Gpe", st["g_see"] / st["g_pe"])
    assert done
    assert abs(st["g_see"] / st["g_pe"] - 0.7) < 2e-3


def test_c0_run_with_reflection_and_collisions_fp64(fk):
    """The 128 x 64 x 64 parity run (1000 steps from f = 0) with both
    optional parts of the step on: R_f = 0.3 and the collision term.  FP64
    against the oracle along the whole trace."""
    cfg = dict(W.c0(), physics_mask=W.ALL | W.BGK, t_e_ev=2.0, ln_lambda=10.0, r_refl=0.3)
    o = Oracle(cfg)
    otr = o.step(W.C0_STEPS, trace=True)
    plain = Oracle(W.c0())
    plain.step(W.C0_STEPS)
    assert rel_l2(plain.f(), o.f()) > 1e-3          # the two parts change the run
    with fk.Solver(cfg, "f64", trace_cap=2048) as s:
        s.step(W.C0_STEPS)
        s.sync()
        gtr, lost = s.trace()
        g, st = s.f(), s.state()
    assert not lost and len(gtr) == W.C0_STEPS + 1
    for a, b in zip(gtr[1::50], otr[::50]):
        assert a["step"] == b["step"]
        for q in ("g_pe", "g_see", "n_total"):
            assert rel(a[q], b[q]) <= 1e-11 or abs(a[q] - b[q]) <= 1e-30, (a["step"], q)
        assert rel(a["sigma"] + a["sigma_lo"], b["sigma"]) <= 1e-11 or abs(b["sigma"]) < 1e-30
    assert rel_l2(g, o.f()) <= 1e-12
    orc = o.record()
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= 1e-12
