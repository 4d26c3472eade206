"""Seeded synthetic workloads: parameter sets and initial states.

This module holds no part of the method's arithmetic.  It only states the
inputs (grid sizes, field, SEY parameters, temperatures, extents) and draws
seeded random numbers.  Both the HIP library and the CPU oracle receive the
same dictionaries; each side turns them into its own parameter record.

Parameter keys (SI units unless the name says eV):
  nx, nvx, nvy             grid cells in x (normal to the surface), v_x, v_y
  length                   domain extent normal to the surface
  vmax_x, vmax_y           velocity-box half widths
  dt, cfl                  time step (0 selects the CFL rule) and CFL fraction
  ey                       applied tangential field (negative: cathode on the left)
  delta_max, a_max_ev, ks  SEY curve parameters (Eq 8-9)
  t_se_ev                  secondary emission temperature (Eq 15)
  j_src, x_src_lo, x_src_hi, t_src_ev   seed-electron band source (Eq 7)
  emission_norm            0 discrete, 1 continuum prefactor of Eq 15
  physics_mask             bit set of the step's parts (values below)
  ex_external              uniform E_x added to the self field
  t_e_ev, ln_lambda        temperature and Coulomb logarithm of the electron-
                           electron collision term (Eq 3-5), used with BGK
  r_refl                   elastic (specular) share of the wall reflection R_f (0: none)
  r_inel                   inelastic share of R_f, re-emitted with the secondaries' shape
  scheme                   0: first-order upwind (the paper's); 1: limited second order
                           with the split order reversed on odd steps
"""
import math

import numpy as np

# Physics-mask bits (part of the parameter interface of both sides).
X, VX, VY, SRC, SEE, SELF = 1, 2, 4, 8, 16, 32
ALL = X | VX | VY | SRC | SEE | SELF
BGK = 64   # electron-electron collisions; opt-in, not part of ALL
NOSC = 128  # with SELF: the field of the surface charge alone (no electron space charge)

_E = 1.602176634e-19
_ME = 9.1093837015e-31


def speed_of(energy_ev: float) -> float:
    """Speed of an electron of the given kinetic energy (non-relativistic)."""
    return math.sqrt(2.0 * energy_ev * _E / _ME)


VMAX_1KEV = speed_of(1000.0)

_BASE = dict(
    dt=0.0, cfl=0.9, ks=1.0, t_se_ev=2.0, j_src=1.0e5, x_src_lo=10e-6, x_src_hi=15e-6,
    t_src_ev=2.0, emission_norm=0, physics_mask=ALL, ex_external=0.0, t_e_ev=2.0, ln_lambda=10.0, r_refl=0.0,
    r_inel=0.0, scheme=0,
    vmax_x=VMAX_1KEV, vmax_y=VMAX_1KEV,
)


def config(**kw):
    c = dict(_BASE)
    c.update(kw)
    return c


def c0():
    """Plain single run: 128 x 64 x 64 over 1 mm, |E_y| = 5 MV/m, 1000 steps."""
    return config(nx=128, nvx=64, nvy=64, length=1e-3, ey=-5e6, delta_max=2.5, a_max_ev=400.0)


C0_STEPS = 1000


def c1():
    """Production size: 2048 x 256 x 256 (134M cells), |E_y| = 8 MV/m."""
    return config(nx=2048, nvx=256, nvy=256, length=1e-3, ey=-8e6, delta_max=2.2, a_max_ev=350.0)


C1_STEPS = 20000


def c4():
    """Large run: 4096 x 384 x 384 (604M cells), |E_y| = 6 MV/m."""
    return config(nx=4096, nvx=384, nvy=384, length=1e-3, ey=-6e6, delta_max=2.8, a_max_ev=450.0)


def paper_default():
    """The paper's default run (Section 2, parameter paragraph): h = 20 um,
    200 x 401 x 201 cells, dt = 5 fs, v_x box 16 v_Te wide, v_y box 40 v_Te
    wide (v_Te from T_e = 2 eV), T_fe = 4 eV."""
    vte = math.sqrt(2.0 * _E / _ME)
    return config(nx=200, nvx=401, nvy=201, length=20e-6, vmax_x=8 * vte, vmax_y=20 * vte,
                  dt=5e-15, ey=-5e6, delta_max=6.5, a_max_ev=650.0, t_src_ev=4.0)


def c2_instances(seed: int = 0, n: int = 64):
    """Batched sweep: n instances with N_x ~ U{256..1024}, N_v ~ U{64..192},
    |E_y| ~ U[1,10] MV/m, delta_max ~ U[1.5,3.5], A_max ~ U[250,600] eV,
    T_se ~ U[1,5] eV, L ~ U[0.5,5] mm."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(256, 1025))
        nv = int(rng.integers(64, 193))
        out.append(config(
            nx=nx, nvx=nv, nvy=nv,
            ey=-float(rng.uniform(1e6, 10e6)),
            delta_max=float(rng.uniform(1.5, 3.5)),
            a_max_ev=float(rng.uniform(250.0, 600.0)),
            t_se_ev=float(rng.uniform(1.0, 5.0)),
            length=float(rng.uniform(0.5e-3, 5e-3)),
        ))
    return out


def surrogate_inputs(seed: int, n: int):
    """(|E_y|, delta_max, A_max, T_se, L) drawn as for the batched sweep."""
    rng = np.random.default_rng(seed)
    return np.stack([
        rng.uniform(1e6, 10e6, n), rng.uniform(1.5, 3.5, n), rng.uniform(250.0, 600.0, n),
        rng.uniform(1.0, 5.0, n), rng.uniform(0.5e-3, 5e-3, n)], axis=1)


def random_state(shape, seed: int, scale: float = 1.0e-3, dtype=np.float64):
    """A positive, smooth-plus-noise distribution for parity tests:
    a product of random Gaussian bumps in each direction times a lognormal
    cell noise.  Values are O(scale)."""
    rng = np.random.default_rng(seed)
    nx, nvx, nvy = shape

    def bumps(n):
        x = np.linspace(-1.0, 1.0, n)
        acc = np.zeros(n)
        for _ in range(3):
            c = rng.uniform(-0.8, 0.8)
            w = rng.uniform(0.1, 0.5)
            acc += rng.uniform(0.2, 1.0) * np.exp(-((x - c) / w) ** 2)
        return acc + 0.05

    f = bumps(nx)[:, None, None] * bumps(nvx)[None, :, None] * bumps(nvy)[None, None, :]
    f = f * np.exp(0.3 * rng.standard_normal(shape))
    return (scale * f).astype(dtype)
