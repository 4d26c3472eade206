#!/usr/bin/env python3
"""Throughput of the 1D2V flashover step on one MI355X.

Workload (default): 4096 (x) x 384 (v_x) x 384 (v_y) cells = 603,979,776
(1 mm, |E_y| = 6 MV/m, delta_max = 2.8, A_max = 450 eV), FP32 f with FP64
sigma and fluxes: the largest single-GPU run (2.4 GB per f buffer).
``--workload c1`` runs 2048 x 256 x 256 (8 MV/m, delta_max 2.2, A_max
350 eV).  The state is first driven into the avalanche so the timed steps
move real data; inputs are resident in HBM before the timed region starts.

One step = the fused sweep kernel over all of f plus the reduction/field
kernel (every part of the method).  ``value`` is cell-updates per second of
the timed steps.  The roofline object prices the sweep kernel at its
algorithmic traffic (read f once, write f once: 8 bytes per cell in FP32)
against the MI355X HBM peak, with the kernel's launch durations measured by
HIP events on the library's stream.  The CPU baseline is the FP64 oracle on a
bounded sample of the same workload (built for the host it runs on).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = {"c1": os.path.join(ROOT, "profiles", "sweep_c1_rocprof.md"),
                   "c4": os.path.join(ROOT, "profiles", "sweep_c4_rocprof.md")}


def kernel_source_digest():
    """Hash of the first-order sweep kernel's device code and of the code
    that shapes its launch (tile rows, planes, workgroup size, arguments:
    the marked region of fk_solver.hip), comments and whitespace left out."""
    h = hashlib.sha256()
    for name in ("fk_internal.h", "fk_kernels.h", "fk_sweep_fast.h", "fk_host.cpp", "fk_solver.hip"):
        with open(os.path.join(ROOT, "paper_2303_14119_amd", "csrc", name), encoding="utf-8") as fh:
            text = fh.read()
        if name == "fk_solver.hip":
            a = text.index("// ---- sweep launch shape (begin)")
            b = text.index("// ---- sweep launch shape (end)")
            text = text[a:b]
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary of the workload, if it was taken on the current kernel source."""
    path = PROFILE_SUMMARY.get(workload)
    if not path or not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != kernel_source_digest():
        return None
    return float(m_b.group(1))


def cpu_baseline(cfg, budget_s=12.0, budget_1t_s=6.0):
    """FP64 oracle on the host, built there with -O3 -march=native: whole
    steps of the same workload until about budget_s seconds of CPU work have
    run on all the host's threads (at most 16, the box's share), then about
    budget_1t_s seconds on one thread."""
    from oracle import solver
    solver.use_native_build()
    threads = min(16, os.cpu_count() or 1)
    cells = cfg["nx"] * cfg["nvx"] * cfg["nvy"]
    o = solver.Oracle(cfg)

    def timed(nthreads, budget):
        solver.set_threads(nthreads)
        o.step(1)                   # first touch of the arrays / warm caches
        n, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return n, el, solver.get_threads()

    n, el, used = timed(threads, budget_s)
    n1, el1, _ = timed(1, budget_1t_s)
    o.close()
    shape = f"{cfg['nx']}x{cfg['nvx']}x{cfg['nvy']}"
    return {"value": cells * n / el / 1e9, "unit": "Gcell-updates/s", "cores": used,
            "kind": "oracle",
            "sample": f"{n} whole FP64 steps of the same {shape} workload on {used} threads ({el:.1f} s); "
                      f"oracle built with gcc -O3 -march=native on this host",
            "value_1_thread": cells * n1 / el1 / 1e9,
            "sample_1_thread": f"{n1} whole steps on 1 thread ({el1:.1f} s)"}


WEIGHTS = os.path.join(ROOT, "paper_2303_14119_amd", "weights", "surrogate.npz")


def time_to_saturation(cfg, stream, t_max=5e-9):
    """The metric's second half: steps and wall time to the Section 2
    saturation test (sigma, Gamma_pe and Gamma_see within 0.1% over 50 ps)
    from the plain cold start and from the surrogate's warm start, on the
    same GPU, and the relative L2 distance of the two final sigma_enc(x)
    profiles (256 points)."""
    import numpy as np
    from paper_2303_14119_amd import flashkin as fk
    from paper_2303_14119_amd import surrogate as S
    if not os.path.exists(WEIGHTS):
        return None
    sur = S.Surrogate.from_file(WEIGHTS, stream=stream)
    out, profiles = {}, {}
    dt = fk.validate(fk.make_params(cfg))["dt"]
    for mode in ("cold", "warm"):
        with fk.Solver(cfg, "f32", stream=stream, trace_cap=8192, trace_stride=S.trace_stride(dt)) as s:
            setup, why = 0.0, None
            if mode == "warm":
                t0 = time.perf_counter()
                _, why = S.warm_start(s, cfg, sur)
                setup = time.perf_counter() - t0
            sat, steps, wall = S.time_to_saturation(
                s, t_max=t_max, check_steps=500,
                log=lambda m, mode=mode: print(f"time to saturation, {mode} start:{m}", file=sys.stderr, flush=True))
            st = s.state()
            profiles[mode] = s.profile(S.NPTS)
        out[mode] = {"saturated": bool(sat), "steps": steps, "sim_time_s": steps * dt, "wall_s": round(wall, 3),
                     "setup_s": round(setup, 4), "sigma": st["sigma"] + st["sigma_lo"]}
        if mode == "warm":
            out[mode]["fallback"] = why
    d = profiles["warm"] - profiles["cold"]
    out["final_sigma_enc_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(profiles["cold"]))
    out["wall_speedup"] = round(out["cold"]["wall_s"] / (out["warm"]["wall_s"] + out["warm"]["setup_s"]), 3)
    h = hashlib.sha256(open(WEIGHTS, "rb").read()).hexdigest()[:16]
    out["weights"] = f"paper_2303_14119_amd/weights/surrogate.npz sha256 {h}"
    return out


def bench_batch(args):
    """64 uneven instances (seed 0), tiling and launch mode picked by the
    library's autotuner at creation (not timed): Gcell-updates/s over
    args.steps steps after args.warmup steps."""
    import torch
    from paper_2303_14119_amd import flashkin as fk
    from paper_2303_14119_amd import workloads as W
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    b = fk.Batch(W.c2_instances(seed=0, n=64), stream=stream, trace_cap=16, trace_stride=1000,
                 autotune=not args.batch_default)
    info = b.info()
    b.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # instances whose avalanche outgrows their grid are flagged; the timing
    # is unaffected, the count is reported
    flagged = sum(1 for v in b.views if fk.fk_sync(v._h) != 0)
    b.close()
    v = info["cells"] * args.steps / el / 1e9
    print(json.dumps({"mode": "batch", "metric": "Gcell-updates/s", "value": round(v, 3), "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 4),
                      "hbm_frac_algorithmic": round(8.0 * v * 1e9 / (HBM_PEAK_GBS * 1e9), 4),
                      "cells": info["cells"], "instances": info["n"], "flagged_instances": flagged,
                      "tile_rows": info["tile_rows"], "tile_planes": info["tile_planes"],
                      "autotuned": not args.batch_default, "sweep_launches_per_step": info["sweep_launches"],
                      "persistent_grid": info["grid"], "schedule": info["schedule"],
                      "workgroup_threads": info["single_threads"] or None}), flush=True)


def bench_mlp(args):
    """Surrogate training steps (forward, loss, backward, AdamW) at batch 256
    on the 7-512-512-512-512-258 network: fk_mlp_train_step as the value, the
    three separate calls beside it."""
    import numpy as np
    import torch
    from paper_2303_14119_amd import flashkin as fk
    from paper_2303_14119_amd import surrogate as S
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    dims, m = S.DIMS, 256
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.uniform(-1, 1, (m, dims[0])).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((m, dims[-1])).astype(np.float32)).cuda()
    flops = sum(2 * m * dims[l] * dims[l + 1] * 3 for l in range(len(dims) - 1))
    res = {}
    for mode in ("separate", "fused"):
        net = fk.MLP(dims, max_batch=m, stream=stream)
        net.set_params(S.init_params(dims, 0))
        step = 0

        def one():
            nonlocal step
            step += 1
            if mode == "fused":
                net.train_step(x.data_ptr(), t.data_ptr(), m, step)
            else:
                net.forward(x.data_ptr(), m)
                net.backward(t.data_ptr(), m, read_loss=False)
                net.adamw(step)
        for _ in range(args.warmup):
            one()
        net.take_loss()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the loss of every step is summed on the device and read once at the end
        for _ in range(args.steps):
            one()
        mean_loss, _ = net.take_loss()
        el = time.perf_counter() - t0
        net.close()
        res[mode] = (el * 1e3 / args.steps, mean_loss)
    ms, mean_loss = res["fused"]
    print(json.dumps({"mode": "mlp", "ms_per_step": round(ms, 4), "steps": args.steps,
                      "gflop_per_step": round(flops / 1e9, 4), "tflops": round(flops / ms / 1e9, 3),
                      "mean_loss": mean_loss, "separate_calls_ms_per_step": round(res["separate"][0], 4),
                      "separate_calls_mean_loss": res["separate"][1],
                      "mfma_bf16_peak_tflops": 2500.0}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the time-to-saturation comparison (cold start vs surrogate warm start, 4096x384x384)")
    ap.add_argument("--batch-default", action="store_true",
                    help="batch mode: the default tiling and launch mode instead of the autotuned choice")
    ap.add_argument("--sample-every", type=int, default=0,
                    help="HIP events around every n-th step's kernels in the timed region "
                         "(0: every step when --steps is below 100, else every 16th)")
    ap.add_argument("--pre-steps", type=int, default=3000,
                    help="steps run before the warmup to drive the state into the avalanche")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (counter calibration)")
    ap.add_argument("--workload", choices=("c1", "c4", "c4slab"), default="c4",
                    help="c4: 4096x384x384 (the headline, the largest single-GPU run); c1: 2048x256x256; "
                         "c4slab: one GPU's share of 4096x384x384 split over 8 GPUs in x "
                         "(512x384x384 over 1/8 mm, the same cells)")
    ap.add_argument("--bgk", action="store_true",
                    help="with the electron-electron collision term (Eq 3-5, T_e 2 eV, ln Lambda 10), "
                         "starting from a thin Maxwellian background in every x plane so that every "
                         "plane takes the term")
    ap.add_argument("--second-order", action="store_true",
                    help="the second-order limited scheme (FK_SCHEME_LIMITED2, an accuracy extension beyond the "
                         "paper) instead of the paper's first-order upwind step")
    ap.add_argument("--tile-rows", type=int, default=0, help="v_x rows per tile (0: the library's choice)")
    ap.add_argument("--tile-planes", type=int, default=0, help="x planes per tile (0: the library's choice)")
    ap.add_argument("--mode", choices=("single", "batch", "mlp"), default="single",
                    help="single: one run of --workload, the headline line (default); batch: the 64-instance "
                         "batched sweep; mlp: surrogate training steps (both for profiling, one JSON line each)")
    args = ap.parse_args()
    if args.sample_every <= 0:
        args.sample_every = 1 if args.steps < 100 else 16
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); a run over several GPUs "
              "would split x into slabs exchanging one half-plane per neighbour and step", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "mlp":
        return bench_mlp(args)

    import torch
    from paper_2303_14119_amd import flashkin as fk
    from paper_2303_14119_amd import workloads as W

    if args.workload == "c1":
        cfg = W.c1()
    elif args.workload == "c4":
        cfg = W.c4()
    else:
        c4 = W.c4()
        cfg = dict(c4, nx=c4["nx"] // 8, length=c4["length"] / 8)
    if args.bgk:
        cfg = dict(cfg, physics_mask=W.ALL | W.BGK, t_e_ev=2.0, ln_lambda=10.0)
    if args.second_order:
        cfg = dict(cfg, scheme=1)
    dev = torch.device("cuda:0")
    torch.cuda.init()
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    stream = torch.cuda.current_stream().cuda_stream
    s = fk.Solver(cfg, "f32", stream=stream, trace_cap=64, trace_stride=1000, tile_rows=args.tile_rows,
                  tile_planes=args.tile_planes)
    cells = s.info["cells"]
    if args.bgk:
        # background of 1e12 electrons per m^3 in every plane (a Maxwellian at
        # T_e, unnormalised shape times a scale); far below the avalanche's
        # densities, it only keeps every plane's collision coefficient non-zero
        vx = (torch.arange(cfg["nvx"], device=dev, dtype=torch.float64) + 0.5 - 0.5 * cfg["nvx"]) * (2 * cfg["vmax_x"] / cfg["nvx"])
        vy = (torch.arange(cfg["nvy"], device=dev, dtype=torch.float64) + 0.5 - 0.5 * cfg["nvy"]) * (2 * cfg["vmax_y"] / cfg["nvy"])
        kt_over_m = cfg["t_e_ev"] * 1.602176634e-19 / 9.1093837015e-31
        shape = torch.exp(-(vx[:, None] ** 2 + vy[None, :] ** 2) / (2 * kt_over_m))
        shape *= 1e12 / (shape.sum() * (2 * cfg["vmax_x"] / cfg["nvx"]) * (2 * cfg["vmax_y"] / cfg["nvy"]))
        bg = shape.to(torch.float32).expand(cfg["nx"], -1, -1).contiguous()
        torch.cuda.synchronize()
        s.write_state(device_ptr=bg.data_ptr())
        del bg
    # drive the state into the avalanche so the timed steps carry real data
    s.step(args.pre_steps + args.warmup)
    s.sync()
    torch.cuda.synchronize()

    # timed region: direct launches; every sample_every-th step has HIP
    # events on the library's stream around its sweep launch and its
    # reduction and field kernels (the live kernel timing)
    s.set_profiling(True, every=args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = s.kernel_times()
    s.set_profiling(False)
    s.sync()
    # the same number of steps replayed from the captured HIP graphs, for
    # reference (no per-kernel events there)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    s.sync()
    st = s.state()
    s.close()

    el = t1 - t0
    ms_per_step = el * 1e3 / args.steps
    value = cells * args.steps / el / 1e9
    sweep_ms = kt["sweep_ms"] / max(kt["sweep_n"], 1)
    field_ms = kt["field_ms"] / max(kt["field_n"], 1)
    bytes_per_launch = 8.0 * cells
    achieved = bytes_per_launch / (sweep_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload) if not (args.bgk or args.second_order) else None
    out = {
        "metric": "Gcell-updates/s",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (("one GPU's x slab of the 4096x384x384 run split over 8 GPUs (wall and vacuum "
                                 "boundaries stand in for the neighbours' half-planes), "
                                 if args.workload == "c4slab" else "plain single run, ")
                                + f"{cfg['nx']}x{cfg['nvx']}x{cfg['nvy']} cells over {cfg['length'] * 1e3:g} mm, "
                                f"|E_y| {abs(cfg['ey']) / 1e6:g} MV/m, delta_max {cfg['delta_max']:g}, "
                                f"A_max {cfg['a_max_ev']:g} eV, FP32 f, FP64 sigma and fluxes"
                                + (", with e-e collisions (BGK, T_e 2 eV) from a 1e12 m^-3 background"
                                   if args.bgk else "")
                                + (", second-order limited scheme (alternating split order)"
                                   if args.second_order else "")),
                   "nx": cfg["nx"], "nvx": cfg["nvx"], "nvy": cfg["nvy"], "cells": cells,
                   "tile_rows": s.info["tile_rows"], "tile_planes": s.info["tile_planes"],
                   "dt_s": s.dt, "step_start": st["step"] - 2 * args.steps,
                   "sigma_at_end": st["sigma"] + st["sigma_lo"],
                   "graph_replay_value": round(cells * args.steps / (g1 - g0) / 1e9, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": ("k_sweep2 (fused limited x/v_x/v_y + source + moments, both split orders)"
                                if args.second_order else "k_sweep (fused x/v_x/v_y upwind + source + moments)"),
                     "kernel_ms": round(sweep_ms, 5), "reduce_field_interval_ms": round(field_ms, 5),
                     "timed_launches": kt["sweep_n"], "sample_every": args.sample_every,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": None,
    }
    if not args.no_tts and args.workload == "c4" and not (args.bgk or args.second_order):
        out["time_to_saturation"] = time_to_saturation(cfg, stream)
    if not args.no_cpu and args.workload in ("c1", "c4") and not (args.bgk or args.second_order):
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
