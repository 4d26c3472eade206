"""Seeded random cases against the FP64 oracle: grid shapes (ragged tiles,
odd grids, single rows and columns, widths across the v_y block sizes), both
precisions, both schemes, tile heights and x chunk lengths, subsets of the
step's parts, the collision term, both reflection shares, both emission
normalisations, external fields and starts on odd steps.  Each case runs 12
steps from a seeded random state and a charged surface.

Tolerances as in the fixed cases: f relative L2 <= 1e-12 (FP64) / 1e-5
(FP32); sigma and the fluxes <= 1e-11 / 1e-5 relative (or 1e-30 absolute
where they vanish)."""
import os

import numpy as np
import pytest

from oracle.solver import Oracle, set_threads
from paper_2303_14119_amd import workloads as W

pytestmark = pytest.mark.gpu

set_threads(min(16, os.cpu_count() or 1))

N_CASES = 64
PARTS = (W.X, W.VX, W.VY, W.SRC, W.SEE, W.SELF)


def draw_case(rng):
    """One random configuration, redrawn until the library accepts it."""
    from paper_2303_14119_amd import flashkin as fk
    while True:
        scheme = int(rng.integers(0, 2))
        dtype = "f64" if rng.random() < 0.5 else "f32"
        # mostly ordinary ragged grids, now and then a degenerate one
        nx = int(rng.integers(1, 4)) if rng.random() < 0.15 else int(rng.integers(4, 48))
        nvx = int(rng.integers(1, 3)) if rng.random() < 0.15 else int(rng.integers(3, 40))
        u = rng.random()
        nvy = (1 if u < 0.1 else int(rng.integers(2, 70)) if u < 0.45 else int(rng.integers(120, 330)) if u < 0.85
               else int(rng.integers(500, 700)))
        mask = 0
        for bit in PARTS:
            if rng.random() < 0.8:
                mask |= bit
        if mask & W.SELF and rng.random() < 0.3:
            mask |= W.NOSC
        if scheme == 0 and rng.random() < 0.3:
            mask |= W.BGK
        if scheme == 1:
            ti = int(rng.choice([0, 4, 8]))
        else:
            ti = int(rng.choice([0, 4, 8, 12, 16]))
        kc = int(rng.choice([0, 4, int(rng.integers(5, 20))]))
        cfg = W.config(nx=nx, nvx=nvx, nvy=nvy, length=nx * 2e-6, ey=-float(rng.uniform(1e6, 6e6)),
                       delta_max=float(rng.uniform(1.5, 3.0)), a_max_ev=float(rng.uniform(300, 500)),
                       t_se_ev=float(rng.uniform(1, 4)), x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8,
                       physics_mask=mask, ex_external=float(rng.choice([0.0, rng.uniform(-2e5, 2e5)])),
                       emission_norm=int(rng.integers(0, 2)), r_refl=float(rng.choice([0.0, 0.2])),
                       r_inel=float(rng.choice([0.0, 0.1])), t_e_ev=40.0, ln_lambda=10.0, scheme=scheme)
        try:
            fk.validate(fk.make_params(cfg, dtype, tile_rows=ti, tile_planes=kc))
        except fk.FlashkinError:
            continue
        return cfg, dtype, ti, kc, int(rng.integers(0, 3))


def cases():
    rng = np.random.default_rng(20261203)
    return [draw_case(rng) for _ in range(N_CASES)]


@pytest.fixture(scope="module")
def fk():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14119_amd import flashkin
    return flashkin


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def close(a, b, tol):
    return abs(a - b) <= tol * abs(b) or abs(a - b) <= 1e-30


@pytest.mark.parametrize("idx", range(N_CASES))
def test_random_case_matches_oracle(fk, idx):
    cfg, dtype, ti, kc, start = cases()[idx]
    shape = (cfg["nx"], cfg["nvx"], cfg["nvy"])
    print(idx, shape, dtype, "scheme", cfg["scheme"], "ti", ti, "kc", kc, "mask", cfg["physics_mask"],
          "start", start, flush=True)
    f0 = W.random_state(shape, seed=1000 + idx, scale=1e3)
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    o = Oracle(cfg)
    o.set_state(f0, 3e-6, start)
    with fk.Solver(cfg, dtype, tile_rows=ti, tile_planes=kc) as s:
        s.write_state(f0, 3e-6, 0.0, start)
        o.step(12)
        s.step(12)
        s.sync()
        g, st = s.f(), s.state()
    r, orc = o.f(), o.record()
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(g, r) <= tol
    tol_s = 1e-11 if dtype == "f64" else 1e-5
    for q in ("g_pe", "g_see", "g_top", "emitted", "n_total"):
        assert close(st[q], orc[q], tol_s), (q, st[q], orc[q])
    assert close(st["sigma"] + st["sigma_lo"], orc["sigma"], tol_s)
    assert st["step"] == start + 12
