"""Single-particle SEEA prediction (Section 3, Eq 19-20 and the flux
estimate of Section 4).  Test infrastructure only (see ``oracle/__init__``).

A secondary electron leaves the surface with energy A0 along the normal,
is pulled back by the surface-charge field a_ex and accelerated along the
surface by a_ey; in a saturated avalanche it must return with the energy A1
at which the yield is one.  With E_x = sigma / 2 eps0 at the surface and the
cosine-averaged launch, this fixes sigma (Eq 20).  Readings: A0 = T_se and
A1 is the first normal-incidence crossover of the Eq 8-9 yield curve.
"""
import math

from scipy.optimize import brentq

from .solver import E_CHARGE, EPS0, M_E, sey


def first_crossover_ev(delta_max, a_max_ev, ks=1.0):
    """Smallest energy with yield one at normal incidence, or None when the
    curve never reaches one (delta_max <= 1: no avalanche can form)."""
    peak = a_max_ev
    if sey(delta_max, a_max_ev, ks, peak, 0.0) <= 1.0:
        return None
    return brentq(lambda a: sey(delta_max, a_max_ev, ks, a, 0.0) - 1.0, 1e-9 * peak, peak,
                  xtol=1e-14, rtol=1e-14, maxiter=500)


def sigma_saturated(ey, delta_max, a_max_ev, a0_ev, ks=1.0):
    """Eq 20: sigma = 2 eps0 |E_y| [ (A1/A0 - 1) / 2 ]^(-1/2), C/m^2."""
    a1 = first_crossover_ev(delta_max, a_max_ev, ks)
    if a1 is None or a1 <= a0_ev:
        return None
    return 2.0 * EPS0 * abs(ey) * (0.5 * (a1 / a0_ev - 1.0)) ** -0.5


def sigma_saturated_normal(ey, delta_max, a_max_ev, a0_ev, ks=1.0):
    """Eq 19 for a secondary launched along the normal, without the cosine
    average of Eq 20: the flight time 2 v0 / a_ex and the distance
    a_ey t^2 / 2 must bring the energy from A0 to A1 with a_ex / a_ey =
    E_x / E_y and E_x = sigma / 2 eps0.  Solved for sigma (C/m^2)."""
    a1 = first_crossover_ev(delta_max, a_max_ev, ks)
    if a1 is None or a1 <= a0_ev:
        return None
    # (2/m)(A1 - A0) = a_ey^2 t^2 with t = 2 v0 / a_ex and v0^2 = 2 A0 / m
    # gives (a_ey / a_ex)^2 = (A1 - A0) / (4 A0)
    ex = abs(ey) * math.sqrt(4.0 * a0_ev / (a1 - a0_ev))
    return 2.0 * EPS0 * ex


def flight_time(sigma, a0_ev):
    """Time of flight of a normally launched secondary, 2 v0 / |a_ex| with
    a_ex = e E_x / m and E_x = sigma / 2 eps0."""
    v0 = math.sqrt(2.0 * a0_ev * E_CHARGE / M_E)
    aex = E_CHARGE * (sigma / (2.0 * EPS0)) / M_E
    return 2.0 * v0 / aex


def primary_flux_saturated(sigma, a0_ev):
    """Flux estimate Gamma_pe = sigma / (e t_ef) (Section 4)."""
    return sigma / (E_CHARGE * flight_time(sigma, a0_ev))


def sigma_along(times, sigmas, v_seea, t, y):
    """Surface charge along the insulator from a 1D trace (a reading of
    Section 4: the avalanche front moves from the junction at v_seea and
    each element then charges as the 1D run did): sigma_1D(t - y / v_seea),
    piecewise linear through (0, 0) and the records, 0 ahead of the front,
    the last value after the trace ends.  Plain numpy interpolation."""
    import numpy as np
    times = np.asarray(times, dtype=np.float64)
    sigmas = np.asarray(sigmas, dtype=np.float64)
    tau = t - np.asarray(y, dtype=np.float64) / v_seea
    if times[0] > 0:
        times = np.concatenate([[0.0], times])
        sigmas = np.concatenate([[0.0], sigmas])
    out = np.interp(tau, times, sigmas, left=0.0, right=sigmas[-1])
    return np.where(tau < 0, 0.0, out)
