"""Batched instances (persistent sweep launches: split by work class, or one per step) and the tiling
autotuner, on the GPU: every instance against the FP64 oracle, and bitwise
against a standalone context with the same tiling."""
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
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_instances(seed, n):
    """Uneven instances drawn like the batched sweep, at sizes the oracle runs
    quickly: odd and even velocity grids, ragged tiles, 1..4 tiles per group."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(20, 140))
        nv = int(rng.integers(20, 200))
        out.append(W.config(nx=nx, nvx=nv, nvy=nv, length=float(rng.uniform(0.1e-3, 1e-3)),
                            ey=-float(rng.uniform(1e6, 10e6)), delta_max=float(rng.uniform(1.5, 3.5)),
                            a_max_ev=float(rng.uniform(250, 600)), t_se_ev=float(rng.uniform(1, 5)),
                            j_src=1e5))
    return out


@pytest.mark.parametrize("autotune", [False, True])
def test_batch_members_match_oracle(fk, autotune):
    cfgs = small_instances(5, 7)
    steps = 60
    with fk.Batch(cfgs, autotune=autotune) as b:
        info = b.info()
        assert info["n"] == 7 and info["items"] > 0
        for m, (c, v) in enumerate(zip(cfgs, b.views)):
            f0 = W.random_state((c["nx"], c["nvx"], c["nvy"]), seed=m, scale=1e1).astype(np.float32)
            v.write_state(f0, 1e-6 * m, 0.0, 0)
        b.step(steps)
        b.sync()
        for m, (c, v) in enumerate(zip(cfgs, b.views)):
            o = Oracle(c)
            f0 = W.random_state((c["nx"], c["nvx"], c["nvy"]), seed=m, scale=1e1).astype(np.float32)
            o.set_state(f0.astype(np.float64), 1e-6 * m, 0)
            o.step(steps)
            st, orc = v.state(), o.record()
            assert st["step"] == steps
            assert rel_l2(v.f(), o.f()) < 1e-5, m
            for q in ("g_pe", "g_see", "n_total"):
                assert abs(st[q] - orc[q]) <= 1e-5 * abs(orc[q]) + 1e-30, (m, q)
            s = st["sigma"] + st["sigma_lo"]
            assert abs(s - orc["sigma"]) <= 1e-5 * abs(orc["sigma"]) + 1e-30, m


@pytest.mark.parametrize("single,threads", [(False, 256), (True, 256), (True, 192)])
def test_batch_is_bitwise_a_standalone_context(fk, single, threads):
    """Split launches and one sweep launch per step (in workgroups of 256 or
    192 threads) give the same bits as single contexts with the same
    tiling."""
    cfgs = [c for c in small_instances(9, 8) if c["nvy"] <= 192][:5]
    assert len(cfgs) == 5 and len({-(-c["nvy"] // 64) for c in cfgs}) >= 2
    with fk.Batch(cfgs, tile_planes=16, single_launch=single, single_threads=threads) as b:
        info = b.info()
        assert (info["sweep_launches"] == 1) == single
        assert info["single_threads"] == (threads if single else 0)
        b.step(45)
        b.sync()
        outs = [(v.f(), v.state()) for v in b.views]
        ti = info["tile_rows"]
    for c, (fb, sb) in zip(cfgs, outs):
        with fk.Solver(c, "f32", tile_rows=ti, tile_planes=min(16, c["nx"])) as s:
            s.step(45)
            assert np.array_equal(s.f(), fb)
            ss = s.state()
            for q in ("sigma", "sigma_lo", "g_pe", "g_see", "n_total"):
                assert ss[q] == sb[q], q


def edge_instances():
    """Instances at the v_y block edges (64, 128, 192 and 256 lanes and one
    past each) and at the batch's maximum width, with N_vx apart from N_vy,
    a single v_y cell, and one x plane."""
    shapes = [(17, 9, 256), (12, 30, 193), (9, 13, 192), (20, 7, 129), (11, 24, 128), (15, 5, 65),
              (8, 19, 64), (6, 3, 1), (1, 10, 100)]
    return [W.config(nx=nx, nvx=nvx, nvy=nvy, length=nx * 3e-6, ey=-4e6 - 1e5 * k, delta_max=2.5,
                     a_max_ev=400.0, x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7, cfl=0.8)
            for k, (nx, nvx, nvy) in enumerate(shapes)]


@pytest.mark.parametrize("single,threads", [(False, 256), (True, 256), (True, 192)])
def test_batch_block_edges_match_oracle(fk, single, threads):
    """Instances at every v_y block edge and at the largest accepted width,
    in each launch mode (192-thread workgroups fall back to 256 since an
    instance is wider than 192), against the FP64 oracle from random
    states; a width past the maximum is refused."""
    cfgs = edge_instances()
    steps = 30
    states = [W.random_state((c["nx"], c["nvx"], c["nvy"]), seed=40 + m, scale=1e1).astype(np.float32)
              for m, c in enumerate(cfgs)]
    with fk.Batch(cfgs, single_launch=single, single_threads=threads) as b:
        info = b.info()
        assert info["single_threads"] == (256 if single else 0)
        for m, v in enumerate(b.views):
            v.write_state(states[m], 2e-6, 0.0, 0)
        b.step(steps)
        b.sync()
        outs = [(v.f(), v.state()) for v in b.views]
    for m, (c, (fb, st)) in enumerate(zip(cfgs, outs)):
        o = Oracle(c)
        o.set_state(states[m].astype(np.float64), 2e-6, 0)
        o.step(steps)
        orc = o.record()
        assert st["step"] == steps
        assert rel_l2(fb, o.f()) < 1e-5, (m, c["nx"], c["nvx"], c["nvy"])
        for q in ("g_pe", "g_see", "n_total"):
            assert abs(st[q] - orc[q]) <= 1e-5 * abs(orc[q]) + 1e-30, (m, q)
        assert abs(st["sigma"] + st["sigma_lo"] - orc["sigma"]) <= 1e-5 * abs(orc["sigma"]) + 1e-30, m
    with pytest.raises(fk.FlashkinError):
        fk.Batch([dict(cfgs[0], nvy=257)])


def test_batch_views_refuse_single_steps(fk):
    with fk.Batch(small_instances(3, 2)) as b:
        with pytest.raises(fk.FlashkinError) as ei:
            b.views[0].step(1)
        assert ei.value.code == fk.E_STATE


def test_autotune_keeps_state_and_results(fk):
    cfg = W.c0()
    with fk.Solver(cfg, "f32") as a:
        a.step(120)
        before = a.f()
        st = a.state()
        chosen = a.autotune(8)
        assert chosen["tile_rows"] in (4, 8, 12, 16)
        assert np.array_equal(a.f(), before)
        st2 = a.state()
        for q in ("step", "sigma", "sigma_lo"):
            assert st2[q] == st[q], q
        # the moments are formed again from the chosen tiling's partials:
        # the same to rounding
        for q in ("g_pe", "n_total"):
            assert abs(st2[q] - st[q]) <= 1e-14 * abs(st[q]), q
        a.step(80)
        tuned = a.f()
    o = Oracle(cfg)
    o.step(200)
    assert rel_l2(tuned, o.f()) < 1e-5


def test_c2_sweep_workload_runs(fk):
    """The 64-instance sweep (7e8 cells): a short run, finite and conserving."""
    cfgs = W.c2_instances(seed=0, n=64)
    with fk.Batch(cfgs, autotune=True) as b:
        b.step(50)
        b.sync()
        for v in b.views[::9]:
            st = v.state()
            assert np.isfinite(st["n_total"]) and st["n_total"] > 0
            assert abs(st["resid"]) <= 1e-5 * st["n_total"]


def random_batch(seed):
    """Uneven instances drawn from a seed: shapes up to the batch's widest
    block, subsets of the step's parts, the collision term on some members,
    both reflection shares and emission normalisations."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(int(rng.integers(4, 9))):
        mask = W.ALL if rng.random() < 0.6 else int(rng.choice([W.X | W.VX | W.VY | W.SEE | W.SELF, W.ALL | W.NOSC]))
        if rng.random() < 0.3:
            mask |= W.BGK
        nx = int(rng.integers(1, 60))
        out.append(W.config(nx=nx, nvx=int(rng.integers(1, 60)), nvy=int(rng.integers(1, 257)), length=nx * 3e-6,
                            ey=-float(rng.uniform(1e6, 6e6)), delta_max=float(rng.uniform(1.5, 3.0)),
                            a_max_ev=float(rng.uniform(300, 500)), x_src_lo=1e-6, x_src_hi=5e-6, j_src=1e7,
                            cfl=0.8, physics_mask=mask, r_refl=float(rng.choice([0.0, 0.2])),
                            r_inel=float(rng.choice([0.0, 0.1])), emission_norm=int(rng.integers(0, 2)),
                            t_e_ev=40.0, ln_lambda=10.0))
    return out


@pytest.mark.parametrize("seed,single,threads", [(71, False, 256), (72, True, 256), (73, True, 192)])
def test_random_batches_match_oracle(fk, seed, single, threads):
    """Seeded random batches, one per launch mode: every member against the
    FP64 oracle after 15 steps from a random state and a charged surface."""
    cfgs = random_batch(seed)
    steps = 15
    states = [W.random_state((c["nx"], c["nvx"], c["nvy"]), seed=seed * 100 + m, scale=1e1).astype(np.float32)
              for m, c in enumerate(cfgs)]
    with fk.Batch(cfgs, single_launch=single, single_threads=threads) as b:
        for m, v in enumerate(b.views):
            v.write_state(states[m], 2e-6, 0.0, 0)
        b.step(steps)
        b.sync()
        outs = [(v.f(), v.state()) for v in b.views]
    for m, (c, (fb, st)) in enumerate(zip(cfgs, outs)):
        o = Oracle(c)
        o.set_state(states[m].astype(np.float64), 2e-6, 0)
        o.step(steps)
        orc = o.record()
        print(seed, m, (c["nx"], c["nvx"], c["nvy"]), c["physics_mask"], rel_l2(fb, o.f()))
        assert rel_l2(fb, o.f()) < 1e-5, m
        for q in ("g_pe", "g_see", "n_total"):
            assert abs(st[q] - orc[q]) <= 1e-5 * abs(orc[q]) + 1e-30, (m, q)
        assert abs(st["sigma"] + st["sigma_lo"] - orc["sigma"]) <= 1e-5 * abs(orc["sigma"]) + 1e-30, m
