"""Pins of the exact CPU oracle F_m(x) (the definition, Eq. fn) to things other than itself.

Each check would fail for a plausible slip in the oracle: a wrong series term or index,
a wrong sign in the incomplete-gamma recurrence, a mis-set crossover between the two
branches, or a mixed-up m.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as orc

XS = np.array([1e-12, 1e-8, 1e-4, 0.01, 0.3, 0.5, 1.0, 2.0, 3.7, 7.3, 12.0, 20.0, 29.5, 30.5,
               35.0, 41.0, 49.9, 50.1, 57.0, 63.0, 75.0, 80.0, 93.0, 100.0, 250.0, 1e3, 1e4])
MS = [0, 1, 2, 3, 5, 8, 13, 16, 20, 27, 36]


def _val(hi, lo, m, i):
    return mp.mpf(hi[m, i]) + mp.mpf(lo[m, i])


def test_value_at_zero_is_one_over_2m_plus_1():
    # Eq. fn at x = 0: int_0^1 t^2m dt = 1/(2m+1)
    hi, lo = orc.exact(np.zeros(1), 40)
    for m in range(41):
        assert hi[m, 0] == 1.0 / (2 * m + 1)
        assert abs(Fraction_err(hi[m, 0], lo[m, 0], 2 * m + 1)) < 1e-31


def Fraction_err(hi, lo, d):
    from fractions import Fraction
    return float((Fraction(hi) + Fraction(lo)) * d - 1)


def test_f0_is_the_error_function():
    # n = 0 reduces to erf: F_0(x) = sqrt(pi) erf(sqrt x) / (2 sqrt x)
    x = np.concatenate([np.logspace(-10, 4, 400), np.linspace(0.01, 120, 400)])
    hi, lo = orc.exact(x, 0)
    ref = np.array([math.sqrt(math.pi) * math.erf(math.sqrt(v)) / (2 * math.sqrt(v)) for v in x])
    assert np.max(np.abs(hi[0] / ref - 1)) < 2e-15


def test_against_incomplete_gamma_library():
    # library routine: F_m(x) = gamma(m+1/2, x) / (2 x^(m+1/2)), mpmath at 50 digits
    hi, lo = orc.exact(XS, max(MS))
    with mp.workdps(50):
        for i, x in enumerate(XS):
            xm = mp.mpf(x)
            for m in MS:
                s = mp.mpf(m) + mp.mpf(1) / 2
                ref = mp.gammainc(s, 0, xm) / (2 * xm ** s)
                got = _val(hi, lo, m, i)
                assert abs(got / ref - 1) < mp.mpf(10) ** -29, (x, m, got, ref)


def test_against_quadrature_of_the_definition():
    # brute force: integrate t^2m exp(-x t^2) over [0, 1] (tanh-sinh, 40 digits)
    xs = [1e-8, 1e-3, 0.5, 1.0, 7.3, 20.0, 50.0, 100.0]
    ms = [0, 1, 4, 9, 16, 25, 36]
    hi, lo = orc.exact(np.array(xs), max(ms))
    with mp.workdps(40):
        for i, x in enumerate(xs):
            for m in ms:
                f = lambda t: t ** (2 * m) * mp.exp(-mp.mpf(x) * t * t)
                # split near the peak of the integrand for large x
                pts = [0, min(1, 1 / mp.sqrt(x)) if x > 1 else mp.mpf(1) / 2, 1]
                ref = mp.quad(f, pts)
                got = _val(hi, lo, m, i)
                assert abs(got / ref - 1) < mp.mpf(10) ** -26, (x, m)


def test_downward_recursion_identity():
    # Eq. r, with the divisor 2m-1 that integration by parts of Eq. fn gives (the paper
    # prints 2m+1): F_{m-1} = (2x F_m + exp(-x)) / (2m-1); the oracle computes each m on
    # its own, so this ties neighbouring orders together
    x = np.concatenate([np.logspace(-6, 3, 60), [29.99, 30.01, 40.0, 60.0, 92.0]])
    hi, lo = orc.exact(x, 37)
    with mp.workdps(40):
        for i, xv in enumerate(x):
            xm = mp.mpf(xv)
            e = mp.exp(-xm)
            for m in range(1, 38):
                lhs = _val(hi, lo, m - 1, i)
                rhs = (2 * xm * _val(hi, lo, m, i) + e) / (2 * m - 1)
                assert abs(lhs / rhs - 1) < mp.mpf(10) ** -29, (xv, m)


def test_long_range_limit():
    # Eq. limf1: x^(m+1/2) F_m(x) / c_m -> 1, with c_m = Gamma(m+1/2)/2
    x = np.array([2e3, 1e4, 1e6])
    hi, lo = orc.exact(x, 36)
    with mp.workdps(40):
        for i, xv in enumerate(x):
            for m in range(37):
                s = mp.mpf(m) + mp.mpf(1) / 2
                r = _val(hi, lo, m, i) * mp.mpf(xv) ** s / (mp.gamma(s) / 2)
                assert abs(r - 1) < mp.mpf(10) ** -29


def test_branch_crossover_is_continuous():
    # both branches agree across X_m = max(30, 2m+20), to second order in the step d:
    # F_m(X+d) - F_m(X) = -F_{m+1}(X) d + F_{m+2}(X) d^2/2 + O(d^3)  (dF_m/dx = -F_{m+1})
    for m in (0, 4, 5, 16, 36):
        X = max(30.0, 2.0 * m + 20.0)
        d = 2.0 ** -30
        x = np.array([X, X + d])
        hi, lo = orc.exact(x, m + 2)
        with mp.workdps(40):
            f0 = _val(hi, lo, m, 0)
            f1 = _val(hi, lo, m, 1)
            dm = mp.mpf(d)
            taylor = -_val(hi, lo, m + 1, 0) * dm + _val(hi, lo, m + 2, 0) * dm * dm / 2
            resid = (f1 - f0) - taylor
            assert abs(resid / f0) < mp.mpf(10) ** -28, (m, resid / f0)


def test_special_inputs():
    x = np.array([-1.0, float("nan"), float("inf"), -0.0])
    hi, lo = orc.exact(x, 3)
    assert np.all(np.isnan(hi[:, 0])) and np.all(np.isnan(hi[:, 1]))
    assert np.all(hi[:, 2] == 0)
    assert np.all(hi[:, 3] == 1.0 / (2 * np.arange(4) + 1))


def test_scipy_cross_check_many_points():
    # a second library (double precision): scipy's regularised incomplete gamma
    sp = pytest.importorskip("scipy.special")
    g = np.random.default_rng(11)
    x = np.exp(g.uniform(np.log(1e-3), np.log(300), 2000))
    hi, lo = orc.exact(x, 20)
    for m in (0, 3, 11, 20):
        s = m + 0.5
        ref = sp.gamma(s) * sp.gammainc(s, x) / (2 * x ** s)
        assert np.max(np.abs(hi[m] / ref - 1)) < 1e-12
