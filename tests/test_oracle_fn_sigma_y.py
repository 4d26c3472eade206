"""Pins of the field-emission rate (Eq 6) and of the sigma(y, t) reading,
and the library's host-only versions of both against them (no GPU).

Eq 6 is the elementary Fowler-Nordheim formula: J = (a / phi) E^2
exp(-b phi^1.5 / E) with the first and second Fowler-Nordheim constants
a = 1.541434e-6 A eV V^-2 and b = 6.830890e9 eV^-1.5 V m^-1 (the values
tabulated in the field-emission literature).  A slip in a power of e, in
pi, in the eV -> J conversion or in the square root of 2m fails against
them; the Fowler-Nordheim plot (ln J/E^2 linear in 1/E with slope
-b phi^1.5) pins the exponent's form on its own.
"""
import math

import numpy as np
import pytest

from oracle import theory
from oracle.solver import fn_current
from paper_2303_14119_amd import flashkin as fk

A_FN = 1.541434e-6
B_FN = 6.830890e9


@pytest.mark.parametrize("E,phi", [(3e9, 4.5), (5e9, 4.5), (8e9, 5.1), (2e9, 3.0)])
def test_fn_current_matches_the_fowler_nordheim_constants(E, phi):
    ref = A_FN / phi * E * E * math.exp(-B_FN * phi ** 1.5 / E)
    assert fn_current(E, phi) == pytest.approx(ref, rel=2e-5)
    # the same field reached by enhancing a lower applied one
    assert fn_current(E / 250.0, phi, beta=250.0) == pytest.approx(ref, rel=2e-5)


def test_fowler_nordheim_plot_is_a_line():
    phi = 4.5
    inv = np.linspace(1 / 9e9, 1 / 2e9, 9)
    lj = np.array([math.log(fn_current(1 / u, phi) * u * u) for u in inv])
    slope, icpt = np.polyfit(inv, lj, 1)
    assert slope == pytest.approx(-B_FN * phi ** 1.5, rel=1e-6)
    assert math.exp(icpt) == pytest.approx(A_FN / phi, rel=1e-5)
    assert np.max(np.abs(np.polyval([slope, icpt], inv) - lj)) < 1e-9


def test_fn_current_underflows_at_the_applied_field():
    """Section 2 takes E_CTJ = |E_y| (a few MV/m): the rate is zero in
    double precision, which is why the band source takes J_src as a
    parameter unless a field enhancement is given."""
    assert fn_current(-5e6, 4.5) == 0.0
    assert fk.fn_current(-5e6, 4.5) == 0.0


@pytest.mark.parametrize("E,phi,beta", [(-5e6, 4.5, 600.0), (8e6, 4.0, 400.0), (-1e7, 5.0, 350.0), (3e9, 4.5, 1.0)])
def test_library_fn_current_matches_oracle(E, phi, beta):
    assert fk.fn_current(E, phi, beta) == pytest.approx(fn_current(E, phi, beta), rel=1e-13)


def test_library_fn_current_rejects_bad_arguments():
    for args in ((1e9, 0.0, 1.0), (1e9, 4.5, 0.0), (float("nan"), 4.5, 1.0)):
        with pytest.raises(fk.FlashkinError):
            fk.fn_current(*args)


def ramp_trace():
    """sigma rising linearly to a plateau: 0 at t = 0, s1 at t1, flat after."""
    t = np.linspace(1e-12, 4e-10, 400)
    s1, t1 = 5e-5, 3e-10
    sig = np.where(t < t1, s1 * t / t1, s1)
    return t, sig


def test_sigma_along_closed_form():
    t, sig = ramp_trace()
    v = 1e7
    now = 5e-10
    y = np.linspace(0, 6e-3, 61)
    got = theory.sigma_along(t, sig, v, now, y)
    tau = now - y / v
    expect = np.where(tau < 0, 0.0, np.minimum(5e-5 * np.clip(tau, 0, None) / 3e-10, 5e-5))
    assert np.allclose(got, expect, rtol=0, atol=1e-12 * 5e-5)
    # the front: charged behind y = v t, uncharged ahead
    assert got[y < v * now - 1e-9].min() > 0 and np.all(got[y > v * now] == 0)
    # the charged length reaches the plateau behind y = v (t - t1)
    assert np.allclose(got[y <= v * (now - 3e-10)], 5e-5)


def test_library_sigma_along_matches_oracle():
    t, sig = ramp_trace()
    recs = [dict(t=a, sigma=b * 0.75, sigma_lo=b * 0.25) for a, b in zip(t, sig)]
    y = np.linspace(0, 6e-3, 97)
    for now in (1e-10, 3.3e-10, 5e-10, 9e-10):
        got = fk.sigma_along(recs, 1e7, now, y)
        ref = theory.sigma_along(t, sig, 1e7, now, y)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-20)
    with pytest.raises(fk.FlashkinError):
        fk.sigma_along(recs[::-1], 1e7, 1e-10, y)
    with pytest.raises(fk.FlashkinError):
        fk.sigma_along(recs, 0.0, 1e-10, y)
