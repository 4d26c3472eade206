"""Full-size and behavioural GPU tests: the benchmark's grids against the
FP64 oracle, the library's error paths, and the physics of Section 3.

Sizes: 2048 x 256 x 256 (the bench workload) and 4096 x 384 x 384 run in the
same launch configuration the benchmark times.  Inputs are seeded synthetic
states; the oracle runs the same number of steps on the host cores.
"""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import theory
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
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel(a, b):
    return abs(a - b) / abs(b)


def separable_state(shape, seed, scale):
    """Cheap seeded state for very large grids: a product of 1D profiles
    times uniform noise in [0.5, 1.5), as FP32."""
    rng = np.random.default_rng(seed)
    nx, nvx, nvy = shape
    px = np.exp(-((np.linspace(0, 1, nx) - 0.1) / 0.2) ** 2) + 0.01
    pv = np.exp(-((np.linspace(-1, 1, nvx) - rng.uniform(-0.3, 0.3)) / 0.3) ** 2)
    pw = np.exp(-((np.linspace(-1, 1, nvy) - rng.uniform(-0.3, 0.3)) / 0.3) ** 2)
    f = (scale * px[:, None, None] * pv[None, :, None] * pw[None, None, :]).astype(np.float32)
    f *= (0.5 + rng.random(shape, dtype=np.float32))
    return f


def test_bench_workload_cold_start_500_steps(fk):
    """The 2048 x 256 x 256 workload from f = 0 through the first 500 steps
    (source, first wall arrivals, SEE): FP32 against FP64."""
    cfg = W.c1()
    o = Oracle(cfg)
    with fk.Solver(cfg, "f32") as s:
        s.step(500)
        s.sync()
        g, st = s.f(), s.state()
    o.step(500)
    ref, orc = o.f(), o.record()
    err = rel_l2(g, ref)
    print("2048x256x256 cold 500 steps: f", err, "g_pe", rel(st["g_pe"], orc["g_pe"]),
          "sigma", rel(st["sigma"] + st["sigma_lo"], orc["sigma"]))
    assert err <= 1e-4
    assert rel(st["n_total"], orc["n_total"]) <= 1e-6
    assert rel(st["g_pe"], orc["g_pe"]) <= 1e-6
    assert rel(st["g_see"], orc["g_see"]) <= 1e-6
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= 1e-6


def test_bench_workload_random_state(fk):
    """A dense seeded state everywhere in phase space with a charged surface:
    every tile, halo and boundary path of the bench launch is exercised."""
    cfg = W.c1()
    f0 = separable_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=11, scale=2e3)
    o = Oracle(cfg)
    o.set_state(f0.astype(np.float64), 4e-6, 0)
    o.step(3)
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f0, 4e-6, 0.0, 0)
        s.step(3)
        s.sync()
        g, st = s.f(), s.state()
    ref, orc = o.f(), o.record()
    assert rel_l2(g, ref) <= 1e-6
    for q in ("g_pe", "g_see", "g_top", "n_total"):
        assert rel(st[q], orc[q]) <= 1e-6, q
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= 1e-6


def test_bench_workload_with_collisions(fk):
    """The 2048 x 256 x 256 launch with the collision term (Eq 3-5) on, at
    densities where nu_ee dt reaches 1e-3 in the densest planes (the self
    field is replaced by a uniform E_x there, as it would break the v_x
    Courant limit): FP32 against FP64 after three steps."""
    from oracle.solver import nu_ee
    cfg = dict(W.c1(), physics_mask=(W.ALL & ~W.SELF) | W.BGK, ex_external=1e5, t_e_ev=2.0, ln_lambda=10.0)
    f0 = separable_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=13, scale=1.0)
    o = Oracle(cfg)
    dv2 = (2 * cfg["vmax_x"] / cfg["nvx"]) * (2 * cfg["vmax_y"] / cfg["nvy"])
    dens = f0.sum(axis=(1, 2), dtype=np.float64) * dv2
    f0 *= np.float32(1e-3 / (nu_ee(dens.max(), 2.0, 10.0) * o.dt))
    o.set_state(f0.astype(np.float64), 4e-6, 0)
    o.step(3)
    assert o.nu_dt_max() > 9e-4
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f0, 4e-6, 0.0, 0)
        s.step(3)
        s.sync()
        g, st = s.f(), s.state()
    ref, orc = o.f(), o.record()
    o.close()
    err = rel_l2(g, ref)
    print("2048x256x256 with collisions, 3 steps: f", err)
    assert err <= 1e-6
    for q in ("g_pe", "g_see", "g_top", "n_total"):
        assert rel(st[q], orc[q]) <= 1e-6, q
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) <= 1e-6


def test_large_grid_two_steps(fk):
    """4096 x 384 x 384 (604M cells, 2.4 GB per f buffer)."""
    cfg = W.c4()
    f0 = separable_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=12, scale=2e3)
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f0, 3e-6, 0.0, 0)
        s.step(2)
        s.sync()
        g, st = s.f(), s.state()
    o = Oracle(cfg)
    o.set_state(f0.astype(np.float64), 3e-6, 0)
    del f0
    o.step(2)
    ref, orc = o.f(), o.record()
    o.close()
    assert rel_l2(g, ref) <= 1e-6
    for q in ("g_pe", "g_see", "n_total"):
        assert rel(st[q], orc[q]) <= 1e-6, q


def test_grid_past_two_to_the_31_cells(fk):
    """14720 x 384 x 384 = 2.17e9 cells, past 2^31 (8.7 GB per FP32 f
    buffer), at the 4096 x 384 x 384 run's cell size: every flat offset on
    the path must be 64-bit.  Two FP32 steps from a separable state against
    the FP64 oracle: sampled planes (the first and last two, both sides of
    chunk boundaries, planes past 2^31 / (384 x 384) = 14564) to 1e-6
    relative L2, the wall fluxes and the electron total to 1e-6."""
    nx = 14720
    cfg = W.config(nx=nx, nvx=384, nvy=384, length=1e-3 * nx / 4096, ey=-6e6, delta_max=2.8, a_max_ev=450.0)
    assert nx * 384 * 384 > 2 ** 31
    f0 = separable_state((nx, 384, 384), seed=13, scale=2e3)
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f0, 3e-6, 0.0, 0)
        s.step(2)
        s.sync()
        g, st = s.f(), s.state()
    planes = [0, 1, 127, 128, 129, 7360, 14563, 14564, 14565, nx - 2, nx - 1]
    gs = g[planes].astype(np.float64)
    del g
    o = Oracle(cfg)
    o.set_state(f0, 3e-6, 0)
    del f0
    o.step(2)
    orc = o.record()
    ref = o.f()
    o.close()
    rs = ref[planes]
    del ref
    for m, k in enumerate(planes):
        assert rel_l2(gs[m], rs[m]) <= 1e-6, k
    for q in ("g_pe", "g_see", "n_total"):
        assert rel(st[q], orc[q]) <= 1e-6, q


def test_large_grid_charged_profile_fifty_steps(fk):
    """4096 x 384 x 384 (the largest single-GPU workload) from a charged
    state built by fk_warm_start: an enclosed-charge profile falling from
    4.6e-5 C/m^2 at the wall over a few micrometres (the hopping cloud of a
    saturated run), then 50 FP32 steps against the FP64 oracle started from
    the same profile.  Bars (FP32 f, FP64 reductions): f relative L2
    <= 1e-4, sigma and the wall fluxes <= 1e-6."""
    from oracle import warm
    cfg = W.c4()
    L = cfg["length"]
    xs = np.linspace(0.0, L, 256)
    profile = 4.6e-5 * np.exp(-xs / 3e-6) - 2e-7 * (xs / L)
    steps = 50
    with fk.Solver(cfg, "f32") as s:
        s.warm_start(profile, cfg["t_se_ev"], step=0)
        s.step(steps)
        s.sync()
        g, st = s.f(), s.state()
    f0, sigma0 = warm.warm_state(profile, L, cfg["nx"], cfg["nvx"], cfg["nvy"], cfg["vmax_x"], cfg["vmax_y"],
                                 cfg["t_se_ev"])
    o = Oracle(cfg)
    o.set_state(f0, sigma0, 0)
    del f0
    r0 = o.record()
    assert r0["g_pe"] > 0 and r0["n_total"] > 0
    o.step(steps)
    ref, orc = o.f(), o.record()
    o.close()
    err = rel_l2(g, ref)
    del ref
    errs = {q: rel(st[q], orc[q]) for q in ("g_pe", "g_see", "g_top", "n_total")}
    errs["sigma"] = rel(st["sigma"] + st["sigma_lo"], orc["sigma"])
    print("4096x384x384 charged, 50 FP32 steps: f", err, errs)
    assert err <= 1e-4
    for q in ("g_pe", "g_see", "sigma"):
        assert errs[q] <= 1e-6, q
    assert errs["n_total"] <= 1e-6


def test_cfl_violation_is_reported(fk):
    """A surface charge whose field moves electrons by more than one velocity
    cell per step must raise FK_E_CFL at the next sync (and stay sticky)."""
    cfg = W.c0()
    with fk.Solver(cfg, "f32") as s:
        s.write_state(None, 5e-3, 0.0, 0)     # E_x = sigma/2eps0 ~ 3e8 V/m
        s.step(2)
        with pytest.raises(fk.FlashkinError) as ei:
            s.sync()
        assert ei.value.code == fk.E_CFL
        with pytest.raises(fk.FlashkinError):
            s.step(1)
        s.write_state(None, 0.0, 0.0, 0)      # clears the sticky error
        s.step(5)
        s.sync()


def test_nonfinite_state_is_reported(fk):
    cfg = W.c0()
    f = np.zeros((cfg["nx"], cfg["nvx"], cfg["nvy"]), dtype=np.float32)
    f[40, 10, 10] = np.nan
    with fk.Solver(cfg, "f32") as s:
        s.write_state(f, 0.0, 0.0, 0)
        s.step(1)
        with pytest.raises(fk.FlashkinError) as ei:
            s.sync()
        assert ei.value.code == fk.E_NONFINITE


def test_invalid_parameters_fail_before_the_gpu(fk):
    cfg = W.c0()
    cfg["nvy"] = 2000
    with pytest.raises(fk.FlashkinError) as ei:
        fk.Solver(cfg, "f32")
    assert ei.value.code == fk.E_INVALID


def test_borrowed_torch_buffers_and_stream(fk):
    import torch
    cfg = W.c0()
    n = cfg["nx"] * cfg["nvx"] * cfg["nvy"]
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.zeros(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = fk.Solver(cfg, "f32", stream=stream.cuda_stream, borrowed=(a.data_ptr(), b.data_ptr()))
        s.step(101)
        s.sync()
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        s.f_to_device(out.data_ptr(), out.numel() * 4)
        host = s.f()
        s.close()
    stream.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(host.shape), host)
    assert np.array_equal(b.cpu().numpy().reshape(host.shape), host)   # odd step count: state in b
    with fk.Solver(cfg, "f32") as ref:
        ref.step(101)
        assert np.array_equal(ref.f(), host)


def test_trace_ring_and_overflow(fk):
    cfg = W.c0()
    with fk.Solver(cfg, "f32", trace_cap=16, trace_stride=5) as s:
        s.step(40)
        recs, lost = s.trace()
        assert not lost and [r["step"] for r in recs] == list(range(0, 41, 5))
        s.step(200)
        recs, lost = s.trace()
        assert lost and len(recs) == 16 and recs[-1]["step"] == 240
        s.step(10)
        recs, lost = s.trace()
        assert not lost and [r["step"] for r in recs] == [245, 250]


def test_saturation_detected_and_matches_oracle(fk):
    """Section 2's test (0.1% over a window) fires once Gamma_see = Gamma_pe;
    the saturated sigma agrees with the oracle."""
    cfg = W.c0()
    window = 50e-12
    with fk.Solver(cfg, "f32", trace_cap=4096) as s:
        sat_at = None
        for chunk in range(40):
            s.step(100)
            if s.saturated(window, 1e-3):
                sat_at = (chunk + 1) * 100
                break
        assert sat_at is not None
        st = s.state()
    assert abs(st["g_see"] / st["g_pe"] - 1) < 1e-3 and st["sigma"] > 0
    o = Oracle(cfg)
    o.step(sat_at)
    orc = o.record()
    assert rel(st["sigma"] + st["sigma_lo"], orc["sigma"]) < 1e-5
