"""Surrogate of the saturated state and the warm start it feeds.

A project addition beyond the paper: the paper advances every run from an
empty domain to saturation (Section 3).  Here a multilayer perceptron maps a
run's parameters (|E_y|, delta_max, A_max, T_se, L) and its grid
resolution (N_x, N_v) to its saturated
x-resolved enclosed charge sigma_enc(x) on 256 points plus the primary and
secondary fluxes; its prediction initialises a new run, which then continues
to saturation.  The plain cold start stays the fallback and the reference
against which the prediction's error is measured.

Every step runs in the library's kernels: the batched solver generates the
data, fk_read_profile resamples it, the network trains with fk_mlp_* and
fk_warm_start builds the initial state.  This module only moves arrays
between them (torch holds the device buffers).
"""
import json
import math
import time

import numpy as np

from . import flashkin as fk
from . import workloads as W

NPTS = 256
DIMS = [7, 512, 512, 512, 512, NPTS + 2]
EPS0 = 8.8541878128e-12
# physical inputs: |E_y|, delta_max, A_max, T_se, L over the sweep's ranges;
# grid inputs: 1/N_x and 1/N_v (cell sizes in units of the domain), over the
# sweep's N_x 256..1024 and N_v 64..192, so a finer grid than the sweep's
# lies just beyond -1 rather than far outside the box
FEATURE_RANGES = np.array([(1e6, 10e6), (1.5, 3.5), (250.0, 600.0), (1.0, 5.0), (0.5e-3, 5e-3),
                           (1 / 1024, 1 / 256), (1 / 192, 1 / 64)])
# How far past [-1, 1] an encoded input may lie before the prediction is not
# trusted and the run cold-starts instead: 0.1 for the physical inputs (the
# sweep's own box), 0.75 for the two cell sizes (a finer grid than the
# sweep's lies just below -1: 4096 x 384 x 384 encodes to -1.5 on both).
FEATURE_MARGIN = np.array([0.1, 0.1, 0.1, 0.1, 0.1, 0.75, 0.75])


def features_raw(ey, delta_max, a_max_ev, t_se_ev, length, nx, nv):
    """Inputs scaled to [-1, 1] from the sweep's ranges (array arguments)."""
    raw = np.stack([np.abs(ey), delta_max, a_max_ev, t_se_ev, length,
                    1.0 / np.asarray(nx, dtype=np.float64), 1.0 / np.asarray(nv, dtype=np.float64)], axis=-1)
    lo, hi = FEATURE_RANGES[:, 0], FEATURE_RANGES[:, 1]
    return (2.0 * (raw - lo) / (hi - lo) - 1.0).astype(np.float32)


def features(cfgs):
    """Network inputs of run dictionaries.  The velocity resolution is taken
    from N_vx (the sweep draws N_vx = N_vy)."""
    cols = np.array([[c["ey"], c["delta_max"], c["a_max_ev"], c["t_se_ev"], c["length"], c["nx"], c["nvx"]]
                     for c in cfgs], dtype=np.float64).reshape(-1, 7)
    return features_raw(*cols.T)


def encode(profile, g_pe, g_see, ey):
    """Targets: the profile in units of 2 eps0 |E_y| (the scale of Eq 20) and
    the log10 fluxes, centred."""
    scale = 2.0 * EPS0 * abs(ey)
    lg = [(math.log10(max(g, 1e10)) - 24.0) / 2.0 for g in (g_pe, g_see)]
    return np.concatenate([np.asarray(profile) / scale, lg]).astype(np.float32)


def decode(y, ey):
    scale = 2.0 * EPS0 * abs(ey)
    y = np.asarray(y, dtype=np.float64)
    return y[:NPTS] * scale, 10.0 ** (2.0 * y[NPTS] + 24.0), 10.0 ** (2.0 * y[NPTS + 1] + 24.0)


def trace_stride(dt, every_s=1e-12):
    return max(1, int(round(every_s / dt)))


def run_to_saturation(batch, cfgs, window_s=50e-12, rtol=1e-3, t_max=3e-9, check_steps=400, log=None):
    """Step a Batch, retiring instances once the Section 2 test holds or
    their time exceeds t_max, and any instance the library flags (CFL or
    non-finite; the rest go on).  Returns per instance (saturated, steps, t,
    status) with status "ok" or the flag's message."""
    n = len(cfgs)
    done = [None] * n
    dts = [v.dt for v in batch.views]
    steps = 0
    while any(d is None for d in done):
        batch.step(check_steps)
        steps += check_steps
        while True:
            try:
                batch.sync()
                break
            except fk.FlashkinError as e:
                m = getattr(e, "instance", -1)
                if m < 0 or done[m] is not None:
                    raise
                done[m] = (False, steps, steps * dts[m], str(e))
                batch.retire([m])
                if log:
                    log(f"  step {steps}: instance {m} flagged and retired: {e}")
        retire = []
        for m, v in enumerate(batch.views):
            if done[m] is not None:
                continue
            t = steps * dts[m]
            if v.saturated(window_s, rtol):
                done[m] = (True, steps, t, "ok")
                retire.append(m)
            elif t >= t_max:
                done[m] = (False, steps, t, "ok")
                retire.append(m)
        if retire:
            batch.retire(retire)
            if log:
                log(f"  step {steps}: retired {len(retire)} (active {sum(d is None for d in done)})")
    return done


def generate(n_runs, seed, per_batch=64, t_max=3e-9, stream=None, log=None, retries=0, draw=None):
    """n_runs runs drawn like the batched sweep (seeded), each advanced to
    saturation or t_max.  Returns (cfgs, X features, Y targets, saturated
    flags, wall seconds, failed) where failed lists (cfg, message) of runs
    the library flagged; those are left out of X and Y.

    A flagged run is one whose avalanche outgrows the grid: the electron
    cloud's space charge drives the v_x Courant number past one and the
    explicit scheme then diverges.  A smaller step only delays this (the
    step is fixed before the surface charges, Section 2 leaves it to the CFL
    conditions), so by default flagged runs are not repeated; ``retries``
    re-runs them from the start at half the step that many times.
    ``draw(seed, n)`` returns n run dictionaries (default: the batched
    sweep's distribution)."""
    draw = draw or (lambda sd, n: W.c2_instances(seed=sd, n=n))
    rng = np.random.default_rng(seed)
    todo = []
    for b0 in range(0, n_runs, per_batch):
        todo += draw(int(rng.integers(1 << 31)), min(per_batch, n_runs - b0))
    cfgs_all, xs, ys, sat, failed = [], [], [], [], []
    t0 = time.perf_counter()
    attempt = 0
    while todo:
        again = []
        # runs of similar step count share a batch, so few are left running alone
        todo.sort(key=lambda c: fk.validate(fk.make_params(c))["dt"])
        for b0 in range(0, len(todo), per_batch):
            cfgs = todo[b0:b0 + per_batch]
            # record about every picosecond of each instance's own time
            dts = [fk.validate(fk.make_params(c))["dt"] for c in cfgs]
            strides = [trace_stride(dt) for dt in dts]
            batch = fk.Batch(cfgs, stream=stream, autotune=False, trace_cap=8192, trace_stride=strides)
            try:
                done = run_to_saturation(batch, cfgs, t_max=t_max, log=log)
                for c, dt, v, d in zip(cfgs, dts, batch.views, done):
                    if d[3] != "ok":
                        if attempt < retries:
                            again.append(dict(c, dt=0.5 * dt))
                        else:
                            failed.append((c, d[3]))
                        continue
                    st = v.state()
                    prof = v.profile(NPTS)
                    cfgs_all.append(c)
                    xs.append(features([c])[0])
                    ys.append(encode(prof, st["g_pe"], st["g_see"], c["ey"]))
                    sat.append(d[0])
            finally:
                batch.close()
            if log:
                log(f"pass {attempt} batch {b0 // per_batch}: {sum(sat)} / {len(sat)} saturated, "
                    f"{len(again)} to rerun, {time.perf_counter() - t0:.1f} s")
        todo = again
        attempt += 1
    return cfgs_all, np.array(xs), np.array(ys), np.array(sat), time.perf_counter() - t0, failed


def init_params(dims, seed):
    """Normal weights scaled by 1/sqrt(fan_in), zero biases, flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(dims) - 1):
        parts.append((rng.standard_normal((dims[l + 1], dims[l])) / math.sqrt(dims[l])).ravel())
        parts.append(np.zeros(dims[l + 1]))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    """The network on the GPU plus its training loop."""

    def __init__(self, seed=0, batch=256, stream=None):
        import torch
        self.torch = torch
        self.batch = batch
        self.net = fk.MLP(DIMS, max_batch=batch, stream=stream)
        self.net.set_params(init_params(DIMS, seed))
        self.step = 0
        self.x_lo = self.x_hi = None      # box of the training inputs (encoded)

    def fit(self, X, Y, epochs=200, lr=1e-3, weight_decay=1e-4, seed=0, Xval=None, Yval=None, log=None):
        torch = self.torch
        rng = np.random.default_rng(seed)
        n = len(X)
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        self.x_lo, self.x_hi = X.min(axis=0).astype(np.float64), X.max(axis=0).astype(np.float64)
        hist = []
        m = self.batch
        self.net.take_loss()                   # start the device-side loss sum afresh
        for ep in range(epochs):
            order = rng.permutation(n)         # shuffled on the host, uploaded per epoch
            xs = torch.from_numpy(X[order]).cuda()
            ys = torch.from_numpy(Y[order]).cuda()
            for lo in range(0, n - m + 1, m):
                self.step += 1
                # cosine decay of the learning rate over the run
                frac = ep / max(1, epochs - 1)
                lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * frac)))
                # forward, loss, gradients and AdamW in one call; no per-step sync
                self.net.train_step(xs[lo:lo + m].data_ptr(), ys[lo:lo + m].data_ptr(), m, self.step, lr=lr_t,
                                    weight_decay=weight_decay)
            rec = {"epoch": ep, "train": self.net.take_loss()[0]}
            if Xval is not None and (ep % 20 == 19 or ep == epochs - 1):
                rec["val"] = float(np.mean((self.predict(Xval) - Yval) ** 2))
            hist.append(rec)
            if log and (ep % 50 == 49 or ep == epochs - 1):
                log(str(rec))
        return hist

    def predict(self, X):
        torch = self.torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.empty((len(X), DIMS[-1]), dtype=np.float32)
        for lo in range(0, len(X), self.batch):
            chunk = X[lo:lo + self.batch]
            xd = torch.from_numpy(chunk).cuda()
            yd = torch.empty((len(chunk), DIMS[-1]), dtype=torch.float32, device="cuda")
            self.net.forward(xd.data_ptr(), len(chunk), yd.data_ptr())
            out[lo:lo + len(chunk)] = yd.cpu().numpy()
        return out

    def params(self):
        return self.net.params()

    def load(self, flat, x_lo=None, x_hi=None):
        self.net.set_params(flat)
        self.x_lo, self.x_hi = x_lo, x_hi

    def save(self, path):
        """Weights and the training inputs' box, FP32 / FP64, no pickles."""
        np.savez(path, params=self.params(), dims=np.array(DIMS), x_lo=self.x_lo, x_hi=self.x_hi)

    @classmethod
    def from_file(cls, path, stream=None):
        d = np.load(path)           # plain arrays only (allow_pickle stays off)
        if list(d["dims"]) != DIMS:
            raise ValueError(f"{path}: network shape {list(d['dims'])} is not {DIMS}")
        sur = cls(stream=stream)
        sur.load(d["params"], d["x_lo"] if "x_lo" in d else None, d["x_hi"] if "x_hi" in d else None)
        return sur


FEATURE_NAMES = ("|E_y|", "delta_max", "A_max", "T_se", "L", "1/N_x", "1/N_v")


def trust_inputs(cfg, lo=None, hi=None):
    """None if every encoded input of the run lies within the training box
    [lo, hi] (default [-1, 1]: the sweep's ranges) widened by its margin,
    else the reason it does not."""
    x = features([cfg])[0].astype(np.float64)
    if not np.all(np.isfinite(x)):
        return "non-finite input"
    lo = -np.ones(len(x)) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = np.ones(len(x)) if hi is None else np.asarray(hi, dtype=np.float64)
    bad = [f"{FEATURE_NAMES[m]} encodes to {x[m]:.3f} (box [{lo[m]:.3f}, {hi[m]:.3f}])" for m in range(len(x))
           if x[m] < lo[m] - FEATURE_MARGIN[m] or x[m] > hi[m] + FEATURE_MARGIN[m]]
    return ("outside the training box: " + "; ".join(bad)) if bad else None


def warm_start(solver, cfg, surrogate):
    """Initialise a run from the surrogate's prediction for its parameters,
    or leave it at the plain cold start (f = 0, sigma = 0, the paper's
    initial state) when the inputs lie outside the training box or the
    prediction is not usable.  Returns (profile or None, reason or None)."""
    why = trust_inputs(cfg, getattr(surrogate, "x_lo", None), getattr(surrogate, "x_hi", None))
    if why is None:
        y = surrogate.predict(features([cfg]))[0]
        if not np.all(np.isfinite(y)):
            why = "non-finite prediction"
        else:
            profile, g_pe, g_see = decode(y, cfg["ey"])
            if not (np.all(np.isfinite(profile)) and np.isfinite(g_pe) and np.isfinite(g_see)):
                why = "non-finite decoded prediction"
            else:
                try:
                    solver.warm_start(profile, cfg["t_se_ev"], step=0)
                    return profile, None
                except fk.FlashkinError as e:
                    why = f"warm start refused: {e}"
    solver.write_state(None, 0.0, 0.0, 0)      # the cold start
    return None, why


def time_to_saturation(solver, window_s=50e-12, rtol=1e-3, t_max=5e-9, check_steps=500, log=None, log_every=20000):
    """Step until the Section 2 test holds; returns (saturated, steps, wall s)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while True:
        solver.step(check_steps)
        steps += check_steps
        if log and steps % log_every == 0:
            st = solver.state()
            log(f"  step {steps}: t {steps * solver.dt:.3e} s, sigma {st['sigma'] + st['sigma_lo']:.4e}, "
                f"Gamma_see/Gamma_pe {st['g_see'] / max(st['g_pe'], 1e-300):.5f}, {time.perf_counter() - t0:.1f} s")
        if solver.saturated(window_s, rtol):
            torch.cuda.synchronize()
            return True, steps, time.perf_counter() - t0
        if steps * solver.dt >= t_max:
            torch.cuda.synchronize()
            return False, steps, time.perf_counter() - t0


def _raw(cfgs):
    keys = ("ey", "delta_max", "a_max_ev", "t_se_ev", "length", "nx", "nvx", "nvy", "dt")
    return np.array([[c[k] for k in keys] for c in cfgs], dtype=np.float64)


def load_data(paths, saturated_only=True):
    """Concatenate generated .npz files; by default only the runs that
    reached the Section 2 saturation test.  The inputs are rebuilt from the
    stored raw parameters, so files written with another feature set load
    the same way."""
    ys, raws = [], []
    for p in paths:
        d = np.load(p)
        keep = d["sat"].astype(bool) if saturated_only else np.ones(len(d["Y"]), dtype=bool)
        ys.append(d["Y"][keep])
        raws.append(d["raw"][keep])
    raw = np.concatenate(raws)
    return features_raw(*raw[:, :7].T), np.concatenate(ys), raw


def profile_errors(y_pred, y_true, raw):
    """Per run: relative L2 of the decoded sigma_enc profile and relative
    errors of the two fluxes."""
    out = []
    for yp, yt, r in zip(y_pred, y_true, raw):
        pp, gp, sp = decode(yp, r[0])
        pt, gt, st = decode(yt, r[0])
        out.append((np.linalg.norm(pp - pt) / max(np.linalg.norm(pt), 1e-300), abs(gp / gt - 1), abs(sp / st - 1)))
    return np.array(out)


def train_cli(args, stream):
    X, Y, raw = load_data(args.data)
    Xv, Yv, rawv = load_data([args.val])
    print(f"train {len(X)} saturated runs, held out {len(Xv)}", flush=True)
    sur = Surrogate(seed=args.seed, stream=stream)
    t0 = time.perf_counter()
    hist = sur.fit(X, Y, epochs=args.epochs, lr=args.lr, seed=args.seed, Xval=Xv, Yval=Yv,
                   log=lambda m: print(m, flush=True))
    wall = time.perf_counter() - t0
    pv = sur.predict(Xv)
    err = profile_errors(pv, Yv, rawv)
    # the method without the network: the training set's mean target
    base = profile_errors(np.repeat(Y.mean(axis=0, keepdims=True), len(Yv), axis=0), Yv, rawv)
    rep = {"train_runs": len(X), "heldout_runs": len(Xv), "epochs": args.epochs, "train_s": wall,
           "steps": sur.step, "final_train_mse": hist[-1]["train"], "heldout_mse": float(np.mean((pv - Yv) ** 2)),
           "heldout_profile_rel_l2_median": float(np.median(err[:, 0])),
           "heldout_profile_rel_l2_p90": float(np.percentile(err[:, 0], 90)),
           "heldout_gpe_rel_median": float(np.median(err[:, 1])),
           "heldout_gsee_rel_median": float(np.median(err[:, 2])),
           "mean_predictor_profile_rel_l2_median": float(np.median(base[:, 0]))}
    sur.save(args.out)
    print(json.dumps(rep), flush=True)


def warmcold_cli(args, stream):
    cfg = W.c4()
    sur = Surrogate.from_file(args.params, stream=stream)
    res = {}
    profiles = {}
    for mode in ("cold", "warm"):
        with fk.Solver(cfg, "f32", stream=stream, trace_cap=8192,
                       trace_stride=trace_stride(fk.validate(fk.make_params(cfg))["dt"])) as s:
            if mode == "warm":
                t0 = time.perf_counter()
                prof0, why = warm_start(s, cfg, sur)
                setup = time.perf_counter() - t0
                if why:
                    print("warm start fell back to the cold start:", why, flush=True)
            else:
                setup = 0.0
            sat, steps, wall = time_to_saturation(s, t_max=args.t_max, check_steps=args.check_steps,
                                                  log=lambda m: print(m, flush=True))
            st = s.state()
            profiles[mode] = s.profile(NPTS)
            res[mode] = {"saturated": sat, "steps": steps, "sim_time_s": steps * s.dt, "wall_s": wall,
                         "setup_s": setup, "sigma": st["sigma"] + st["sigma_lo"], "g_pe": st["g_pe"],
                         "g_see": st["g_see"]}
            print(mode, json.dumps(res[mode]), flush=True)
    d = profiles["warm"] - profiles["cold"]
    res["final_profile_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(profiles["cold"]))
    res["speedup_wall"] = res["cold"]["wall_s"] / (res["warm"]["wall_s"] + res["warm"]["setup_s"])
    np.savez(args.out, cold=profiles["cold"], warm=profiles["warm"])
    print(json.dumps(res), flush=True)


def main(argv=None):
    """Command line: ``generate`` saturated runs into an .npz file, ``train``
    the network on them, ``warmcold`` compares a warm-started large run with
    a cold start."""
    import argparse
    import torch
    ap = argparse.ArgumentParser(prog="python -m paper_2303_14119_amd.surrogate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate", help="run the batched solver to saturation and store (X, Y)")
    g.add_argument("--n", type=int, required=True)
    g.add_argument("--seed", type=int, required=True)
    g.add_argument("--per-batch", type=int, default=128)
    g.add_argument("--t-max", type=float, default=3e-9)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train", help="train the network on generated runs")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--val", required=True)
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    w = sub.add_parser("warmcold", help="warm vs cold start on the 4096 x 384 x 384 run")
    w.add_argument("--params", required=True)
    w.add_argument("--t-max", type=float, default=5e-9)
    w.add_argument("--check-steps", type=int, default=500)
    w.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    if args.cmd == "generate":
        cfgs, X, Y, sat, wall, failed = generate(args.n, args.seed, per_batch=args.per_batch, t_max=args.t_max,
                                                 stream=stream, log=lambda m: print(m, flush=True))
        cells = sum(c["nx"] * c["nvx"] * c["nvy"] for c in cfgs)
        np.savez(args.out, X=X, Y=Y, sat=sat, raw=_raw(cfgs), wall=wall, n_failed=len(failed))
        print(f"generated {len(cfgs)} runs ({int(sat.sum())} saturated, {len(failed)} failed) "
              f"in {wall:.1f} s; {cells / 1e9:.2f} Gcells", flush=True)
    elif args.cmd == "train":
        train_cli(args, stream)
    else:
        warmcold_cli(args, stream)


if __name__ == "__main__":
    main()
