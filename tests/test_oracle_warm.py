"""Pins of the enclosed-charge profile and the warm-start state (oracle.warm).

Each pin fixes the oracle by something other than itself: closed forms of
simple densities, hand-computed values, and the C oracle's own field solve
(an independent routine) at the cell centres.
"""
import numpy as np
import pytest

from oracle import warm
from oracle.solver import E_CHARGE, EPS0, M_E, Oracle
from paper_2303_14119_amd import workloads as W


def test_uniform_density_gives_linear_profile():
    # n_e = n0 everywhere: sigma_enc(x) = sigma - 2 e n0 x exactly
    L, nx, n0, sigma = 2e-3, 37, 3.0e15, 4.0e-6
    prof = warm.enclosed_profile(sigma, np.full(nx, n0), L, 101)
    x = np.linspace(0.0, L, 101)
    assert np.allclose(prof, sigma - 2 * E_CHARGE * n0 * x, rtol=0, atol=1e-15)


def test_single_cell_density_by_hand():
    # four cells of width 1 m, charge only in cell 2: flat, ramp across the
    # cell, flat again
    ne = np.array([0.0, 0.0, 1.0 / E_CHARGE, 0.0])
    prof = warm.enclosed_profile(5.0, ne, 4.0, 9)   # x = 0, 0.5, ..., 4
    assert np.allclose(prof, [5, 5, 5, 5, 5, 4, 3, 3, 3], rtol=0, atol=1e-12)


def test_profile_at_centres_is_two_eps0_ex_of_the_field_solve():
    """The C oracle's E_x at cell centres (its own prefix sum, Section 2)
    equals sigma_enc / 2 eps0 there."""
    cfg = W.config(nx=24, nvx=16, nvy=18, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
    o = Oracle(cfg)
    f = W.random_state(o.shape, seed=5, scale=1e3)
    o.set_state(f, sigma=3.0e-7)
    ex, ne = o.field()
    prof = warm.enclosed_profile(3.0e-7, ne, cfg["length"], 2 * cfg["nx"] + 1)
    centres = prof[1::2]
    assert np.allclose(2 * EPS0 * ex, centres, rtol=1e-12, atol=1e-12 * abs(prof).max())
    o.close()


def test_warm_state_of_linear_profile_is_uniform_maxwellian():
    nx, nvx, nvy, L = 20, 24, 30, 1e-3
    vmx, vmy, t_ev = 1.8e7, 1.5e7, 2.0
    n0, s0 = 7.0e15, 2.0e-6
    prof = s0 - 2 * E_CHARGE * n0 * np.linspace(0.0, L, 64)
    f, sigma = warm.warm_state(prof, L, nx, nvx, nvy, vmx, vmy, t_ev)
    assert sigma == s0
    dvx, dvy = 2 * vmx / nvx, 2 * vmy / nvy
    dens = f.sum(axis=(1, 2)) * dvx * dvy
    assert np.allclose(dens, n0, rtol=1e-10)
    # Maxwellian shape: f(v) / f(0-ish) = exp(-m (v^2 - v'^2) / 2T)
    vx = (np.arange(nvx) + 0.5 - nvx / 2) * dvx
    vy = (np.arange(nvy) + 0.5 - nvy / 2) * dvy
    r = f[3, 2, 7] / f[3, 12, 15]
    want = np.exp(-M_E * (vx[2] ** 2 + vy[7] ** 2 - vx[12] ** 2 - vy[15] ** 2) / (2 * t_ev * E_CHARGE))
    assert r == pytest.approx(want, rel=1e-12)


def test_warm_state_round_trip_through_the_field_solve():
    """A piecewise-linear profile with kinks at the cell faces is recovered
    exactly by the C oracle's density of the warm state."""
    cfg = W.config(nx=16, nvx=20, nvy=22, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)
    rng = np.random.default_rng(2)
    n_true = rng.uniform(0.0, 1e16, cfg["nx"])
    s0 = 1.5e-6
    dx = cfg["length"] / cfg["nx"]
    faces = s0 - 2 * E_CHARGE * dx * np.concatenate([[0.0], np.cumsum(n_true)])
    # given at the faces (npts - 1 = nx)
    f, sigma = warm.warm_state(faces, cfg["length"], cfg["nx"], cfg["nvx"], cfg["nvy"],
                               cfg["vmax_x"], cfg["vmax_y"], cfg["t_se_ev"])
    o = Oracle(cfg)
    o.set_state(f, sigma=sigma)
    _, ne = o.field()
    assert np.allclose(ne, n_true, rtol=1e-10, atol=1e-6 * n_true.max())
    back = warm.enclosed_profile(sigma, ne, cfg["length"], cfg["nx"] + 1)
    assert np.allclose(back, faces, rtol=0, atol=1e-10 * abs(faces).max())
    o.close()


def test_rising_profile_gives_zero_density():
    # where the profile rises the implied density would be negative: clamped
    prof = np.array([0.0, 1e-6, 0.5e-6])
    f, _ = warm.warm_state(prof, 1e-3, 10, 8, 8, 1e7, 1e7, 2.0)
    dens = f.sum(axis=(1, 2))
    assert np.all(dens[:5] == 0.0)
    assert np.all(dens[5:] > 0.0)
