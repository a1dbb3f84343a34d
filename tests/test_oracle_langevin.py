"""Pins for the oracle's Langevin derivatives (L(x) = coth x - 1/x, paper Sec. 2;
pole structure at i*m*pi, App. E Prop. 2)."""
from fractions import Fraction
from math import factorial

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import langevin as lg

# Values of L^(n)(0): the Taylor coefficients of coth u - 1/u times n!.
# (Textbook: coth u = 1/u + u/3 - u^3/45 + 2u^5/945 - u^7/4725 + 2u^9/93555 - ...)
CLOSED_AT_ZERO = {1: Fraction(1, 3), 3: Fraction(-2, 15), 5: Fraction(16, 63),
                  7: Fraction(-16, 15), 9: Fraction(256, 33)}


@pytest.mark.parametrize("n", list(range(0, 11)) + [12])
def test_value_at_zero(n):
    got = float(lg.langevin_deriv(n, np.array([0.0]))[0])
    want = float(CLOSED_AT_ZERO.get(n, 0))
    assert abs(got - want) <= 1e-15 * max(1.0, abs(want))


def test_textbook_coth_coefficients():
    # coth u - 1/u = u/3 - u^3/45 + 2u^5/945 - u^7/4725 + 2u^9/93555
    want = [Fraction(1, 3), Fraction(-1, 45), Fraction(2, 945), Fraction(-1, 4725),
            Fraction(2, 93555)]
    for j, w in enumerate(want, start=1):
        assert lg.taylor_coefficient(j) == pytest.approx(float(w), rel=1e-15)


def _mp_deriv(n, u):
    mpmath.mp.dps = 40
    return float(mpmath.diff(lambda x: mpmath.coth(x) - 1 / x, mpmath.mpf(u), n))


@pytest.mark.parametrize("n", range(0, 14))
def test_against_mpmath(n):
    us = np.linspace(-20.0, 20.0, 41) + 0.0137
    ref = np.array([_mp_deriv(n, u) for u in us])
    got = lg.langevin_deriv(n, us)
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    assert np.max(np.abs(got - ref) / scale) < 1e-13


@pytest.mark.parametrize("n", range(1, 14))
def test_parity(n):
    u = np.linspace(0.01, 12.0, 97)
    a = lg.langevin_deriv(n, u)
    b = lg.langevin_deriv(n, -u)
    assert np.allclose(b, (-1) ** (n + 1) * a, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", range(1, 14))
def test_large_u_asymptote(n):
    # L(u) = 1 - 1/u + O(e^{-2u}) for u -> +inf
    for u in (40.0, 60.0):
        want = (-1) ** (n + 1) * factorial(n) / u ** (n + 1)
        got = float(lg.langevin_deriv(n, np.array([u]))[0])
        assert got == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("n", range(1, 14))
def test_finite_difference(n):
    u = np.linspace(-6.0, 6.0, 49) + 0.021
    hstep = 1e-4
    fd = (lg.langevin_deriv(n - 1, u + hstep) - lg.langevin_deriv(n - 1, u - hstep)) / (2 * hstep)
    ex = lg.langevin_deriv(n, u)
    scale = np.max(np.abs(ex))
    assert np.max(np.abs(fd - ex)) < 1e-6 * scale


@pytest.mark.parametrize("n", range(1, 14))
def test_series_and_poles_agree_on_overlap(n):
    u = np.concatenate([np.linspace(0.5, 1.5, 21), -np.linspace(0.5, 1.5, 21)])
    s = lg.series(n, u)
    p = lg.poles(n, u)
    scale = np.max(np.abs(p))
    assert np.max(np.abs(s - p)) < 1e-12 * scale


@pytest.mark.parametrize("n", range(2, 9))
def test_zero_integral(n):
    # integral of L^(n) over the line = L^(n-1)(+inf) - L^(n-1)(-inf) = 0 for n >= 2
    f = lambda t: float(lg.langevin_deriv(n, np.array([t]))[0])
    left, _ = integrate.quad(f, -np.inf, 0.0, limit=400)
    right, _ = integrate.quad(f, 0.0, np.inf, limit=400)
    mag, _ = integrate.quad(lambda t: abs(f(t)), -60, 60, limit=400)
    assert abs(left + right) < 1e-8 * mag


def test_first_derivative_integral_is_two():
    f = lambda t: float(lg.langevin_deriv(1, np.array([t]))[0])
    val = integrate.quad(f, -np.inf, 0.0)[0] + integrate.quad(f, 0.0, np.inf)[0]
    assert val == pytest.approx(2.0, rel=1e-9)


def test_reference_values():
    # high-precision values (mpmath, 50 digits) at a few points
    mpmath.mp.dps = 50
    assert float(lg.langevin_deriv(1, np.array([0.4]))[0]) == pytest.approx(0.3229316216312544, rel=1e-14)
    assert float(lg.langevin_deriv(1, np.array([0.8]))[0]) == pytest.approx(0.2946426019, rel=1e-9)
    assert float(lg.langevin_deriv(12, np.array([3.0]))[0]) == pytest.approx(-2.28595049335416, rel=1e-13)
