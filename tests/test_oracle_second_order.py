"""Pins of the oracle's second-order scheme (scheme 1), no GPU.

The paper advances Eq 2 with an explicit first-order upwind update
(Section 2).  Scheme 1 is this build's accuracy extension for coarse grids:
each 1D sweep in flux form with a minmod-limited slope (the face value of
the upwind cell moved towards the face by (1 - |c|)/2 times its slope,
slope zero in the first and last cell of every line), and the split order
x, v_x, v_y, source on even steps reversed on odd steps, so that a pair of
steps is a symmetric composition.  What fixes it:
  * exactness: where the limiter keeps the full slope (a concave monotone
    quadratic) the flux is Lax-Wendroff's, which moves a quadratic exactly;
    where every slope is clipped (alternating data) the step is the
    first-order upwind one, boundaries included;
  * accuracy: free streaming of a smooth profile converges at about second
    order (first order: ratio 2 per halving);
  * splitting: under uniform acceleration the x centroid after an even
    number of steps follows x0 + v0 t + a t^2 / 2 up to the limiter's small
    error, which falls faster than the grid; Lie splitting keeps the error
    a dt t / 2;
  * positivity at Courant numbers up to one, the particle balance in both
    orders, and the v_y mirror symmetry.
"""
import math
import os

import numpy as np
import pytest

from oracle.solver import E_CHARGE, M_E, Oracle, set_threads
from paper_2303_14119_amd import workloads as W

set_threads(min(8, os.cpu_count() or 1))


def tiny(**kw):
    base = dict(nx=64, nvx=8, nvy=6, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0, j_src=0.0,
                physics_mask=0, scheme=1)
    base.update(kw)
    return W.config(**base)


def centres(vmax, n):
    dv = 2 * vmax / n
    return (np.arange(n) + 0.5 - 0.5 * n) * dv, dv


@pytest.mark.parametrize("row", [6, 1])
def test_quadratic_moves_exactly_where_the_limiter_keeps_the_slope(row):
    """One x sweep of a concave profile that rises towards the flow's
    downwind side: every interior face takes the Lax-Wendroff flux, and
    Lax-Wendroff translates a quadratic exactly, f'(k) = f(k - c)."""
    cfg = tiny(nx=40, physics_mask=W.X, dt=2.0e-13)
    o = Oracle(cfg)
    vx, _ = centres(cfg["vmax_x"], cfg["nvx"])
    c = vx[row] * o.dt / o.dx
    k = np.arange(cfg["nx"], dtype=np.float64)
    M = 60.0 if c > 0 else -21.0         # apex outside the line: monotone, concave
    prof = lambda kk: 5000.0 - (kk - M) ** 2
    f0 = np.zeros(o.shape)
    f0[:, row, :] = prof(k)[:, None]
    o.set_state(f0, 0.0, 0)
    o.step(1)
    got = o.f()[:, row, 0]
    inner = slice(2, cfg["nx"] - 2)
    assert np.allclose(got[inner], prof(k - c)[inner], rtol=1e-13, atol=0)
    # the first-order scheme misses by the upwind diffusion c (1 - c) f'' / 2
    o1 = Oracle(dict(cfg, scheme=0))
    o1.set_state(f0, 0.0, 0)
    o1.step(1)
    miss = o1.f()[inner, row, 0] - prof(k - c)[inner]
    assert np.allclose(miss, -abs(c) * (1 - abs(c)), rtol=1e-9)


def test_clipped_slopes_give_the_first_order_step():
    """Alternating data is a local extremum in every cell, so every slope is
    zero and the step equals the first-order upwind one, with the wall
    emission row and the vacuum face included (x sweep alone, both orders)."""
    cfg = tiny(nx=30, nvx=8, nvy=4, physics_mask=W.X | W.SEE, dt=2.5e-13)
    k = np.arange(30)
    f0 = (1.0 + 0.5 * (-1.0) ** k)[:, None, None] * np.ones((1, 8, 4))
    a, b = Oracle(cfg), Oracle(dict(cfg, scheme=0))
    for o in (a, b):
        o.set_state(f0, 0.0, 0)
        o.step(3)
    assert np.allclose(a.f(), b.f(), rtol=1e-14, atol=0)


@pytest.mark.parametrize("axis", ["x", "vy"])
def test_free_streaming_converges_at_second_order(axis):
    """A Gaussian moved by free streaming (x) or uniform acceleration (v_y)
    over a fixed time: the L1 error against the exact shift falls by >= 3.3
    per halving of cells and step (minmod clips the extremum, so the ratio
    sits just under 4); first-order upwind falls by about 2."""
    ratios = {}
    for scheme in (0, 1):
        errs = []
        for n in ((200, 400, 800) if axis == "x" else (400, 800, 1600)):
            if axis == "x":
                cfg = tiny(nx=n, nvx=8, nvy=2, physics_mask=W.X, dt=0.0, cfl=0.5, ey=0.0, scheme=scheme)
                o = Oracle(cfg)
                vx, _ = centres(cfg["vmax_x"], cfg["nvx"])
                x = (np.arange(n) + 0.5) * o.dx
                L = cfg["length"]
                prof = lambda xx: np.exp(-((xx - 0.3 * L) / (0.1 * L)) ** 2)
                f0 = np.zeros(o.shape)
                f0[:, 6, 0] = prof(x)
                o.set_state(f0, 0.0, 0)
                steps = int(round(0.3 * L / vx[6] / o.dt)) // 2 * 2
                o.step(steps)
                exact = prof(x - vx[6] * steps * o.dt)
                errs.append(np.abs(o.f()[:, 6, 0] - exact).sum() * o.dx)
            else:
                vmax = 1.0e7
                cfg = tiny(nx=2, nvx=2, nvy=n, physics_mask=W.VY, vmax_x=vmax, vmax_y=vmax, ey=-2e6,
                           dt=0.4 * (2 * vmax / n) / (E_CHARGE * 2e6 / M_E), scheme=scheme)
                o = Oracle(cfg)
                vy, dvy = centres(vmax, n)
                prof = lambda v: np.exp(-((v + 0.4 * vmax) / (0.12 * vmax)) ** 2)
                f0 = np.zeros(o.shape)
                f0[:, :, :] = prof(vy)[None, None, :]
                o.set_state(f0, 0.0, 0)
                a_y = E_CHARGE * 2e6 / M_E
                steps = int(round(0.6 * vmax / a_y / o.dt)) // 2 * 2
                o.step(steps)
                exact = prof(vy - a_y * steps * o.dt)
                errs.append(np.abs(o.f()[0, 0] - exact).sum() * dvy)
        ratios[scheme] = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(1.8 < r < 2.2 for r in ratios[0]), ratios
    assert all(r >= 3.3 for r in ratios[1]), ratios


def test_split_order_centroid_under_uniform_acceleration():
    """x and v_x transport under a uniform external E_x: the exact centroid
    is x0 + v0 t + a t^2 / 2.  Lie splitting (x then v_x every step) misses
    by a dt t / 2, the same number of cells at every resolution; reversing
    the order on odd steps cancels that term after an even number of steps,
    leaving the limiter's error, which falls at least fourfold per halving."""
    errs = {0: [], 1: []}
    for scheme in (0, 1):
        for r in (1, 2, 4):
            nx, nvx = 100 * r, 32 * r
            cfg = tiny(nx=nx, nvx=nvx, nvy=2, physics_mask=W.X | W.VX, ex_external=-1.5e6, dt=2.5e-13 / r,
                       scheme=scheme)
            o = Oracle(cfg)
            vx, dvx = centres(cfg["vmax_x"], nvx)
            xk = (np.arange(nx) + 0.5) * o.dx
            f0 = np.exp(-((xk - 0.35e-3) / 0.06e-3) ** 2)[:, None, None] \
                * np.exp(-((vx - 0.25 * cfg["vmax_x"]) / (0.12 * cfg["vmax_x"])) ** 2)[None, :, None] * np.ones((1, 1, 2))
            o.set_state(f0, 0.0, 0)
            a = -E_CHARGE * cfg["ex_external"] / M_E
            m = f0.sum()
            x0 = (f0.sum(axis=(1, 2)) * xk).sum() / m
            v0 = (f0.sum(axis=(0, 2)) * vx).sum() / m
            n = 40 * r
            o.step(n)
            f = o.f()
            t = n * o.dt
            xn = (f.sum(axis=(1, 2)) * xk).sum() / f.sum()
            errs[scheme].append(abs(xn - (x0 + v0 * t + 0.5 * a * t * t)) / o.dx)
            if scheme == 0:
                assert errs[0][-1] == pytest.approx(0.5 * a * o.dt * t / o.dx, rel=1e-2)
    assert errs[1][0] < 0.25 * errs[0][0]
    assert errs[1][0] / errs[1][1] >= 4.0 and errs[1][1] / errs[1][2] >= 4.0


def test_positivity_and_balance_in_both_orders():
    """Every Courant number below one, every part of the step on, a random
    charged state: f stays non-negative and the particle balance closes to
    FP64 rounding on even (forward) and odd (reversed) steps alike."""
    cfg = W.config(nx=24, nvx=20, nvy=18, length=1e-3 * 24 / 128, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                   j_src=1e7, x_src_lo=1e-6, x_src_hi=5e-6, r_refl=0.2, r_inel=0.1, scheme=1)
    o = Oracle(cfg)
    o.set_state(W.random_state((24, 20, 18), seed=11, scale=1e3), 2e-6, 0)
    tr = o.step(40, trace=True)
    assert o.f().min() >= 0.0
    for r in tr:
        assert abs(r["resid"]) <= 1e-13 * r["n_total"], r
    assert o.cfl_max_vx() < 1.0
    # the run differs from the first-order one
    o1 = Oracle(dict(cfg, scheme=0))
    o1.set_state(W.random_state((24, 20, 18), seed=11, scale=1e3), 2e-6, 0)
    o1.step(40)
    assert np.abs(o1.f() - o.f()).max() > 1e-3 * np.abs(o.f()).max()


def test_mirror_symmetry_without_tangential_field():
    """With E_y = 0 and no one-sided source, v_y -> -v_y stays a symmetry of
    the limited step in both orders."""
    cfg = tiny(nx=16, nvx=12, nvy=10, physics_mask=W.X | W.VX | W.VY | W.SEE | W.SELF, ey=0.0)
    o = Oracle(cfg)
    f = W.random_state(o.shape, seed=9)
    f = f + f[:, :, ::-1]
    o.set_state(f, 1e-6, 0)
    o.step(41)
    g = o.f()
    assert np.allclose(g, g[:, :, ::-1], rtol=1e-13, atol=0)
