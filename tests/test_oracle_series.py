"""Pins for the truncated divided difference of Lemma 2.2 (eqs. taylor, D2-1).

The oracle's f_S and G2^S are checked against the exact divided difference of
Phi evaluated in 50-digit arithmetic, within the truncation bound of the series.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import scheme

mpmath.mp.dps = 50


def exact_f(x, s):
    """f(x, s) = [(x+s) ln(x+s) - (x-s) ln(x-s)] / (2s) in 50 digits (Lemma 2.2)."""
    x = mpmath.mpf(x)
    s = mpmath.mpf(s)
    return ((x + s) * mpmath.log(x + s) - (x - s) * mpmath.log(x - s)) / (2 * s)


def exact_dd(a1, a0):
    """[Phi(a1) - Phi(a0)]/(a1 - a0) in 50 digits (eq. D2)."""
    a1 = mpmath.mpf(a1)
    a0 = mpmath.mpf(a0)
    Phi = lambda z: z * mpmath.log(z) + (1 - z) * mpmath.log(1 - z)
    return (Phi(a1) - Phi(a0)) / (a1 - a0)


def tail_bound(r, S):
    # sum_{m>S} r^{2m}/((2m+1)2m) <= r^{2S+2} / ((2S+3)(2S+2)(1-r^2))
    return r ** (2 * S + 2) / ((2 * S + 3) * (2 * S + 2) * (1 - r * r))


@pytest.mark.parametrize("x,s", [(0.5, 0.01), (0.3, 0.1), (0.2, 0.15), (0.7, 0.35), (0.05, 0.04)])
@pytest.mark.parametrize("S", [1, 3, 10])
def test_f_series_matches_exact_minus_constant(x, s, S):
    got = float(scheme.f_series(np.float64(x), np.float64(s), S))
    want = float(exact_f(x, s) - 1)
    r = s / x
    assert abs(got - want) <= tail_bound(r, S) * (1 + 1e-9) + 4e-16 * (1 + abs(want))


@pytest.mark.parametrize("a1,a0", [(0.52, 0.48), (0.31, 0.29), (0.9, 0.6), (0.15, 0.45), (0.02, 0.06),
                                   (0.5 + 1e-9, 0.5)])
def test_g2_series_matches_exact_divided_difference(a1, a0):
    S = 10
    got = float(scheme.g2_series(np.float64(a1), np.float64(a0), S))
    want = float(exact_dd(a1, a0))
    zeta = 0.5 * (a1 + a0)
    sig = abs(0.5 * (a1 - a0))
    bound = tail_bound(sig / zeta, S) + tail_bound(sig / (1 - zeta), S)
    assert abs(got - want) <= bound * (1 + 1e-9) + 1e-14


def test_printed_plus_sign_would_be_wrong():
    """The printed phi^S = f_S(z,s) + f_S(1-z,-s) tends to ln z + ln(1-z), not Phi'(z):
    at z = 0.3 the two readings differ by O(1); the minus reading matches eq. D2."""
    a1, a0 = 0.31, 0.29
    z, s = 0.3, 0.01
    plus = float(scheme.f_series(z, s, 10) + scheme.f_series(1 - z, -s, 10))
    want = float(exact_dd(a1, a0))
    assert abs(plus - want) > 0.5
    assert abs(float(scheme.g2_series(a1, a0, 10)) - want) < 1e-14


def test_series_limit_is_phi_prime():
    """As sigma -> 0, G2^S -> Phi'(zeta) = ln zeta - ln(1-zeta)."""
    for z in [0.1, 0.37, 0.5, 0.93]:
        got = float(scheme.g2_series(np.float64(z), np.float64(z), 10))
        assert abs(got - (math.log(z) - math.log(1 - z))) < 1e-15


def test_truncation_error_decreases_with_S():
    a1, a0 = 0.6, 0.3
    want = float(exact_dd(a1, a0))
    errs = [abs(float(scheme.g2_series(a1, a0, S)) - want) for S in (1, 2, 4, 8, 10)]
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
