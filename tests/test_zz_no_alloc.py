"""The allocation-free entry point (fk_step_noalloc) against the context
path (fk_create_borrowed + fk_write_state + fk_step + fk_read_state) on the
same inputs: the same kernels in the same order, so f, sigma and the fluxes
must agree bit for bit.  Two calls in a row, the second with a smaller grid
(the scratch array keeps the first call's contents and must be cleared),
plus the size limit and argument checks.  GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2303_14119_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14119_amd import flashkin
    return torch, flashkin


def context_run(torch, fk, cfg, dtype, f0, sigma0, steps):
    td = torch.float32 if dtype == "f32" else torch.float64
    n = f0.size
    a = torch.zeros(n, dtype=td, device="cuda")
    b = torch.zeros(n, dtype=td, device="cuda")
    s = fk.Solver(cfg, dtype, stream=torch.cuda.current_stream().cuda_stream, borrowed=(a.data_ptr(), b.data_ptr()),
                  trace_cap=64, trace_stride=10)
    s.write_state(f0, sigma0, 0.0, 0)
    s.step(steps)
    s.sync()
    f, st = s.f(), s.state()
    s.close()
    return f, st


def noalloc_run(torch, fk, cfg, dtype, f0, sigma0, steps):
    td = torch.float32 if dtype == "f32" else torch.float64
    a = torch.from_numpy(np.ascontiguousarray(f0).ravel()).to("cuda")
    assert a.dtype == td
    b = torch.full_like(a, 7.0)            # garbage in the second buffer
    out = torch.zeros(C.sizeof(fk.fk_state), dtype=torch.uint8, device="cuda")
    flags = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    p = fk.make_params(cfg, dtype, trace_cap=64, trace_stride=10)
    rc = fk.fk_step_noalloc(C.byref(p), torch.cuda.current_stream().cuda_stream, a.data_ptr(), b.data_ptr(),
                            sigma0, 0.0, 0, steps, out.data_ptr(), flags.data_ptr())
    assert rc == fk.OK, (fk.fk_last_error(None) or b"").decode()
    torch.cuda.synchronize()
    f = (a if steps % 2 == 0 else b).cpu().numpy().reshape(f0.shape)
    raw = out.cpu().numpy().tobytes()
    st = fk.fk_state.from_buffer_copy(raw).as_dict()
    return f, st, int(flags.cpu().item())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_the_context_path_twice(env, dtype):
    torch, fk = env
    cases = [
        (W.config(nx=128, nvx=64, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0, r_refl=0.2,
                  r_inel=0.1), 3e-6, 37),
        (W.config(nx=48, nvx=40, nvy=72, length=0.4e-3, ey=-4e6, delta_max=2.5, a_max_ev=400.0), 1e-6, 20),
    ]
    for m, (cfg, sigma0, steps) in enumerate(cases):
        f0 = W.random_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=40 + m, scale=1e3)
        f0 = f0.astype(np.float32 if dtype == "f32" else np.float64)
        fr, sr = context_run(torch, fk, cfg, dtype, f0, sigma0, steps)
        fn, sn, flags = noalloc_run(torch, fk, cfg, dtype, f0, sigma0, steps)
        assert flags == 0
        assert np.array_equal(fn, fr), m
        for q in ("step", "t", "sigma", "sigma_lo", "g_pe", "g_see", "g_top", "emitted", "loss_v", "n_total",
                  "resid"):
            assert sn[q] == sr[q], (m, q, sn[q], sr[q])
        assert sn["step"] == steps and sn["g_pe"] > 0


def test_noalloc_reports_cfl_and_rejects_oversized(env):
    torch, fk = env
    cfg = W.c0()
    f0 = np.zeros((cfg["nx"], cfg["nvx"], cfg["nvy"]), dtype=np.float32)
    _, _, flags = noalloc_run(torch, fk, cfg, "f32", f0, 5e-3, 2)   # E_x ~ 3e8 V/m
    assert flags & 1
    big = W.config(nx=65536, nvx=384, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
    p = fk.make_params(big, "f32")
    x = torch.zeros(8, device="cuda")
    rc = fk.fk_step_noalloc(C.byref(p), None, x.data_ptr(), x.data_ptr() + 4, 0.0, 0.0, 0, 1, None, None)
    assert rc == fk.E_INVALID and b"32 MiB" in fk.fk_last_error(None)
    p = fk.make_params(cfg, "f32")
    assert fk.fk_step_noalloc(C.byref(p), None, x.data_ptr(), x.data_ptr(), 0.0, 0.0, 0, 1, None, None) == fk.E_INVALID


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_second_order_and_collisions(env, dtype):
    """The same bitwise agreement with the second-order scheme (both split
    orders: an odd number of steps from step 0) and with the collision
    term."""
    torch, fk = env
    base = dict(nx=64, nvx=48, nvy=64, length=0.5e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
    cases = [
        (W.config(scheme=fk.SCHEME_LIMITED2, r_refl=0.1, **base), 2e-6, 21),
        (W.config(physics_mask=W.ALL | W.BGK, t_e_ev=2.0, ln_lambda=10.0, **base), 2e-6, 19),
    ]
    for m, (cfg, sigma0, steps) in enumerate(cases):
        f0 = W.random_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=60 + m, scale=1e3)
        f0 = f0.astype(np.float32 if dtype == "f32" else np.float64)
        fr, sr = context_run(torch, fk, cfg, dtype, f0, sigma0, steps)
        fn, sn, flags = noalloc_run(torch, fk, cfg, dtype, f0, sigma0, steps)
        assert flags == 0
        assert np.array_equal(fn, fr), m
        for q in ("step", "sigma", "sigma_lo", "g_pe", "g_see", "g_top", "emitted", "loss_v", "n_total", "resid"):
            assert sn[q] == sr[q], (m, q, sn[q], sr[q])


def test_noalloc_random_shapes_in_sequence(env):
    """Eight seeded random grids in a row (both precisions and schemes,
    ragged and degenerate shapes, subsets of the step's parts), growing and
    shrinking from call to call, so every call starts on the scratch array
    another grid left behind: bitwise the context path each time."""
    torch, fk = env
    rng = np.random.default_rng(99)
    done = 0
    while done < 8:
        scheme = int(rng.integers(0, 2))
        dtype = "f64" if rng.random() < 0.5 else "f32"
        mask = W.ALL if rng.random() < 0.6 else int(rng.choice([W.X | W.VX | W.VY | W.SEE | W.SELF, W.ALL | W.NOSC]))
        if scheme == 0 and rng.random() < 0.3:
            mask |= W.BGK
        nx = int(rng.integers(1, 80))
        cfg = W.config(nx=nx, nvx=int(rng.integers(1, 70)), nvy=int(rng.integers(1, 300)), length=nx * 3e-6,
                       ey=-float(rng.uniform(1e6, 6e6)), delta_max=2.5, a_max_ev=400.0, x_src_lo=1e-6,
                       x_src_hi=5e-6, j_src=1e7, cfl=0.8, physics_mask=mask, r_refl=float(rng.choice([0.0, 0.2])),
                       r_inel=float(rng.choice([0.0, 0.1])), t_e_ev=40.0, ln_lambda=10.0, scheme=scheme)
        try:
            fk.validate(fk.make_params(cfg, dtype))
        except fk.FlashkinError:
            continue
        steps = int(rng.integers(1, 12))
        f0 = W.random_state((cfg["nx"], cfg["nvx"], cfg["nvy"]), seed=200 + done, scale=1e3)
        f0 = f0.astype(np.float32 if dtype == "f32" else np.float64)
        fr, sr = context_run(torch, fk, cfg, dtype, f0, 2e-6, steps)
        fn, sn, flags = noalloc_run(torch, fk, cfg, dtype, f0, 2e-6, steps)
        print(done, (cfg["nx"], cfg["nvx"], cfg["nvy"]), dtype, "scheme", scheme, "mask", mask, "steps", steps)
        assert flags == 0
        assert np.array_equal(fn, fr), done
        for q in ("step", "sigma", "sigma_lo", "g_pe", "g_see", "g_top", "emitted", "loss_v", "n_total", "resid"):
            assert sn[q] == sr[q], (done, q, sn[q], sr[q])
        done += 1
