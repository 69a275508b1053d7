"""Pins of the oracle's sparse kernel, Eq. (8) under reading R1.

Every expected value below is fixed by mathematics, not by re-running the
oracle's formula: closed-form values at special radii, the integral of f over
[0, 1], the behaviour at both ends of the support and the leading term of the
expansion at the support edge.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

PI = math.pi


@pytest.mark.parametrize("r,expected", [
    (0.0, 1.0),                                  # k(0) = sigma0
    (0.25, 0.5 + 1 / (2 * PI)),                  # cos(pi/2) = 0, sin(pi/2) = 1
    (1 / 3, 1 / 3 + math.sqrt(3) / (4 * PI)),    # cos(2pi/3) = -1/2, sin = sqrt3/2
    (0.5, 1 / 6),                                # cos(pi) = -1, sin(pi) = 0
    (2 / 3, 1 / 6 - math.sqrt(3) / (4 * PI)),    # cos(4pi/3) = -1/2, sin = -sqrt3/2
    (0.75, 1 / 6 - 1 / (2 * PI)),                # cos(3pi/2) = 0, sin = -1
    (1.0, 0.0),                                  # support edge (reading R2: d < l)
    (1.5, 0.0),
    (7.0, 0.0),
])
def test_kernel_closed_form_values(r, expected):
    assert float(oracle.kernel_f(r)) == pytest.approx(expected, rel=1e-14, abs=1e-15)


def test_kernel_integral_is_one_third():
    # int_0^1 (2 + cos 2pi r)(1 - r)/3 dr = 1/3 ; int_0^1 sin(2 pi r) dr = 0 ;
    # int_0^1 r cos(2 pi r) dr = 0  =>  int_0^1 f = 1/3.
    val, err = integrate.quad(lambda r: float(oracle.kernel_f(r)), 0.0, 1.0, epsabs=1e-13,
                              epsrel=1e-13, limit=200)
    assert val == pytest.approx(1 / 3, rel=1e-11)


def test_kernel_flat_at_both_ends_and_continuous_at_l():
    h = 1e-5
    # f'(0) = 0 (even to third order): symmetric difference
    f = oracle.kernel_f
    assert abs((f(h) - f(0.0)) / h) < 1e-4
    # continuity and zero slope at r = 1 (reading R1; the literal printed
    # bracket would jump from 2/3 to 0 here)
    assert float(f(1 - 1e-9)) < 1e-40
    assert abs((f(1.0) - f(1 - h)) / h) < 1e-15


def test_kernel_edge_expansion_leading_term():
    # f(1 - s) = (2pi)^4 s^5 / 180 - (2pi)^6 s^7 / 3780 + O(s^9)
    for s in (1e-1, 3e-2, 1e-2):
        lead = (2 * PI) ** 4 * s ** 5 / 180 - (2 * PI) ** 6 * s ** 7 / 3780
        assert float(oracle.kernel_f(1 - s)) == pytest.approx(lead, rel=3 * (2 * PI * s) ** 4 / 100)


def test_kernel_monotone_and_bounded():
    r = np.linspace(0.0, 1.0, 4001)
    f = oracle.kernel_f(r)
    assert np.all(np.diff(f) <= 1e-15)
    assert f.min() >= 0.0 and f.max() <= 1.0


def test_kernel_derivative_matches_central_differences():
    r = np.linspace(0.01, 0.99, 99)
    h = 1e-6
    fd = (oracle.kernel_f(r + h) - oracle.kernel_f(r - h)) / (2 * h)
    np.testing.assert_allclose(oracle.kernel_df(r), fd, rtol=1e-7, atol=1e-9)
    # closed forms: f'(1/4) = -(2pi/3)(3/4) - 2/3 ; f'(1/2) = -4/3
    assert float(oracle.kernel_df(0.25)) == pytest.approx(-(2 * PI / 3) * 0.75 - 2 / 3, rel=1e-14)
    assert float(oracle.kernel_df(0.5)) == pytest.approx(-4 / 3, rel=1e-14)
    assert float(oracle.kernel_df(0.0)) == 0.0 and float(oracle.kernel_df(1.0)) == 0.0
