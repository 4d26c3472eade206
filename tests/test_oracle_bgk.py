"""Pins of the oracle's electron-electron collision term (Eq 3-5), no GPU.

The term is a BGK relaxation f -> n_e f~_e0 at the frequency nu_ee of Eq 4.
What fixes it independently of the oracle's own code:
  * nu_ee against the textbook electron collision time: Eq 4 is 1/(sqrt 2
    tau_e) with tau_e = 3.44e5 T_e^1.5 / (n_e lnL) s (T_e in eV, n_e in
    cm^-3, the NRL plasma formulary), so a slip in a power, in pi^1.5, in the
    eV -> J conversion or in the factor 12 fails;
  * BGK alone relaxes each plane geometrically at the rate (1 - nu_ee dt)
    per step with its density held fixed (explicit Euler of Eq 3), so a
    wrong sign, a term taken from the wrong state, or a non-conserving
    normalisation fails;
  * the fixed point of that relaxation is the Maxwellian of Eq 5 at T_e:
    log f is quadratic in v with curvature -m / T_e, so a wrong temperature
    or a dropped factor 2 in the exponent fails;
  * with every other part of the step on, the particle balance still closes,
    which holds only if the term conserves the density it is given.
"""
import math
import os

import numpy as np
import pytest

from oracle.solver import BGK, E_CHARGE, M_E, Oracle, nu_ee, set_threads
from paper_2303_14119_amd import workloads as W

set_threads(min(8, os.cpu_count() or 1))


def nrl_tau_e(n_m3, t_ev, ln_lambda):
    """Electron collision time of the NRL plasma formulary, s."""
    return 3.44e5 * t_ev ** 1.5 / (n_m3 * 1e-6 * ln_lambda)


@pytest.mark.parametrize("n,t,lnl", [(1e18, 2.0, 10.0), (3e20, 7.5, 12.0), (5e15, 0.5, 8.0)])
def test_nu_ee_is_the_textbook_rate(n, t, lnl):
    nu = nu_ee(n, t, lnl)
    # the formulary's coefficient has three significant figures
    assert nu * math.sqrt(2.0) * nrl_tau_e(n, t, lnl) == pytest.approx(1.0, abs=3e-3)


def bgk_only(nx=3, nvx=24, nvy=20, dt=2e-13, t_e=3.0):
    """BGK alone, on a velocity box of three thermal speeds at T_e (so the
    equilibrium's tails stay well above rounding)."""
    vth = math.sqrt(t_e * E_CHARGE / M_E)
    return W.config(nx=nx, nvx=nvx, nvy=nvy, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                    vmax_x=3 * vth, vmax_y=3 * vth, dt=dt, physics_mask=BGK, t_e_ev=t_e, ln_lambda=10.0,
                    j_src=0.0)


def dense_state(cfg, seed, dens):
    """Positive random f with plane densities of the order of dens (1/m^3)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.2, 1.0, (cfg["nx"], cfg["nvx"], cfg["nvy"]))
    dv2 = (2 * cfg["vmax_x"] / cfg["nvx"]) * (2 * cfg["vmax_y"] / cfg["nvy"])
    scale = np.array([dens * (1 + k) for k in range(cfg["nx"])]) / (f.sum(axis=(1, 2)) * dv2)
    return f * scale[:, None, None]


def test_bgk_alone_relaxes_geometrically_with_density_fixed():
    cfg = bgk_only()
    f0 = dense_state(cfg, 3, 2e22)
    o = Oracle(cfg)
    o.set_state(f0, 0.0, 0)
    dt = o.dt
    _, n0 = o.field()
    fs = [f0]
    for _ in range(6):
        o.step(1)
        fs.append(o.f())
    _, n1 = o.field()
    assert np.allclose(n1, n0, rtol=1e-13, atol=0)
    rates = np.array([nu_ee(n, cfg["t_e_ev"], cfg["ln_lambda"]) * dt for n in n0])
    assert rates.min() > 1e-2 and rates.max() < 0.2      # the test exercises the term
    g = [fs[m + 1] - fs[m] for m in range(len(fs) - 1)]
    for m in range(len(g) - 1):
        for k in range(cfg["nx"]):
            expect = (1.0 - rates[k]) * g[m][k]
            assert np.allclose(g[m + 1][k], expect, rtol=1e-10, atol=1e-12 * np.abs(g[m][k]).max())
    assert o.nu_dt_max() == pytest.approx(rates.max(), rel=1e-14)


def test_bgk_fixed_point_is_the_maxwellian_at_t_e():
    cfg = bgk_only(t_e=3.0)
    f0 = dense_state(cfg, 5, 1e22)
    o = Oracle(cfg)
    o.set_state(f0, 0.0, 0)
    _, n0 = o.field()
    o.step(1)
    f1 = o.f()
    dv = 2 * cfg["vmax_x"] / cfg["nvx"]
    vx = (np.arange(cfg["nvx"]) + 0.5 - 0.5 * cfg["nvx"]) * dv
    dvy = 2 * cfg["vmax_y"] / cfg["nvy"]
    vy = (np.arange(cfg["nvy"]) + 0.5 - 0.5 * cfg["nvy"]) * dvy
    for k in range(cfg["nx"]):
        rate = nu_ee(n0[k], cfg["t_e_ev"], cfg["ln_lambda"]) * o.dt
        finf = f0[k] + (f1[k] - f0[k]) / rate          # limit of the geometric series
        assert finf.min() > 0
        # log f is -m v^2 / (2 T_e) plus a constant: second differences in
        # each direction give the curvature -m dv^2 / T_e
        lf = np.log(finf)
        d2x = lf[2:, :] - 2 * lf[1:-1, :] + lf[:-2, :]
        d2y = lf[:, 2:] - 2 * lf[:, 1:-1] + lf[:, :-2]
        te = cfg["t_e_ev"] * E_CHARGE
        assert np.allclose(d2x, -M_E * dv * dv / te, rtol=1e-8)
        assert np.allclose(d2y, -M_E * dvy * dvy / te, rtol=1e-8)
        # and it holds the plane's electrons
        assert finf.sum() * dv * dvy == pytest.approx(n0[k], rel=1e-12)
        # symmetric in v (no drift)
        assert abs((finf * vx[:, None]).sum()) <= 1e-12 * (finf * np.abs(vx)[:, None]).sum()
        assert abs((finf * vy[None, :]).sum()) <= 1e-12 * (finf * np.abs(vy)[None, :]).sum()


def test_equilibrium_is_stationary():
    cfg = bgk_only()
    o = Oracle(cfg)
    dens = np.array([1e21, 3e21, 7e20])
    feq = o.feq()
    f0 = dens[:, None, None] * feq[None]
    o.set_state(f0, 0.0, 0)
    o.step(5)
    assert np.allclose(o.f(), f0, rtol=1e-12, atol=0)


def test_particle_balance_closes_with_collisions():
    """Every part of the step on but the self field (densities where nu_ee dt
    is about 1e-3 would drive the space-charge field far past the v_x
    Courant limit; a uniform E_x stands in for it), collisions included: the
    per-step balance residual stays at rounding."""
    cfg = W.config(nx=24, nvx=20, nvy=18, length=1e-3 * 24 / 128, ey=-5e6, delta_max=2.5, a_max_ev=400.0,
                   physics_mask=(W.ALL & ~W.SELF) | BGK, ex_external=2e5, t_e_ev=2.0, ln_lambda=10.0)
    f0 = dense_state(cfg, 9, 2e20)
    o = Oracle(cfg)
    o.set_state(f0, 1e-6, 0)
    tr = o.step(20, trace=True)
    assert o.nu_dt_max() > 1e-3
    for r in tr:
        assert abs(r["resid"]) <= 1e-12 * r["n_total"], r
