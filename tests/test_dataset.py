"""Pins of the coefficient dataset and of the approximant part of the oracle.

The dataset (paper_2504_07637_amd/data/boys_coeffs.txt) plays the role of the paper's
supplementary coefficient file, which is not available: it was re-fitted offline.  These
tests tie it, and the oracle's evaluation of it, to what the paper and the mathematics fix:
the closed forms of Eqs. q0, q1, aq, bq and c_n, the cut-off definition, the gathering rule
and no pole on x >= 0, and the exact-arithmetic error E_n of Table 1.

The third class, fp32x (binary64 coefficients of approximants fitted to at least 28 bits
for binary32 outputs computed in binary64, cut-off z_{n,28}), has no table in the paper:
its pins are the same closed forms, the cut-off definition with b = 28, the structure,
and an exact-arithmetic error of at least 28 bits measured here against the exact oracle.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as orc

NMAX = 36
CLASSES = ("fp64", "fp32")
ALL_CLASSES = ("fp64", "fp32", "fp32x")


def _recs():
    return orc.dataset()


def test_dataset_has_every_order_with_table1_N(table1):
    recs = _recs()
    for cls in CLASSES:
        for n in range(NMAX + 1):
            r = recs[(cls, n)]
            assert r.N == table1[n][cls]["N"], (cls, n)
            f = r.fields
            deg_u = len(f["ug"]) + 2 * (len(f["uq"]) // 2) + len(f["ul"])
            deg_v = len(f["vg"]) + 2 * (len(f["vq"]) // 2) + len(f["vl"])
            # Eqs. pz, qz: u has degree N-1, v degree N
            assert deg_u == r.N - 1 and deg_v == r.N, (cls, n, deg_u, deg_v)


def _q_from_F(n, x, F):
    """Invert Eq. fq: Q = ((c/F)^(1/s) - x) e^x)^(1/s)."""
    s = mp.mpf(2 * n + 1) / 2
    c = mp.gamma(s) / 2
    W = (c / F) ** (1 / s) - x
    return (W * mp.exp(x)) ** (1 / s)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 11, 16, 20, 27, 36])
def test_q0_q1_from_the_exact_function(n):
    # Q_n(0) and Q'_n(0) of Eqs. q0, q1 recovered from the exact oracle via Eq. fq
    h = 1e-7
    x = np.array([0.0, h, 2 * h])
    hi, lo = orc.exact_one(x, n)
    with mp.workdps(40):
        Q = [_q_from_F(n, mp.mpf(x[i]), mp.mpf(hi[i]) + mp.mpf(lo[i])) for i in range(3)]
        d0 = (4 * Q[1] - Q[2] - 3 * Q[0]) / (2 * mp.mpf(h))
        for cls in ALL_CLASSES:
            r = orc.record(cls, n)
            tol = 2.0 ** -23 if cls == "fp32" else 2.0 ** -52
            assert abs(float(Q[0]) / r["q0"] - 1) <= tol, (cls, n)
            assert abs(float(d0) / r["q1"] - 1) < 1e-9 + tol, (cls, n, float(d0), r["q1"])
            # the 40-digit values too
            assert abs(Q[0] - mp.mpf(r["q0x"].numerator) / r["q0x"].denominator) < 1e-30
            assert abs(d0 - mp.mpf(r["q1x"].numerator) / r["q1x"].denominator) < 1e-12


@pytest.mark.parametrize("cls", ALL_CLASSES)
def test_asymptote_constraints_alpha_beta_and_q2(cls):
    # Eqs. qa, qb, aq, bq: the expanded rational P/D (Eq. qr) tends to alpha x + beta, and
    # q2 = alpha - q1 follows from the leading coefficients of P - (q0 + q1 x) D
    with mp.workdps(40):
        for n in range(NMAX + 1):
            r = orc.record(cls, n)
            A = [mp.mpf(a.numerator) / a.denominator for a in r["A"]]
            B = [mp.mpf(b.numerator) / b.denominator for b in r["B"]]
            N = r.N
            s = mp.mpf(2 * n + 1) / 2
            c_next = mp.gamma(s + 1) / 2
            alpha = (2 * c_next) ** (mp.mpf(-2) / (2 * n + 1))
            beta = mp.mpf(2 * n - 1) / (2 * n + 1) * alpha
            assert abs(A[N + 1] / B[N] / alpha - 1) < 1e-30
            b_fit = (A[N] * B[N] - A[N + 1] * B[N - 1]) / B[N] ** 2
            assert abs(b_fit - beta) < 1e-30 * (1 + abs(beta))
            q1 = mp.mpf(r["q1x"].numerator) / r["q1x"].denominator
            q2 = mp.mpf(r["q2x"].numerator) / r["q2x"].denominator
            assert abs(q2 - (alpha - q1)) < 1e-30
            assert B[0] == 1 and B[N] > 0   # solutions with B_N < 0 are rejected


def test_c_n_and_c0():
    with mp.workdps(40):
        for cls in ALL_CLASSES:
            for n in range(NMAX + 1):
                r = orc.record(cls, n)
                # c_n = (2n)! sqrt(pi) / (n! 2^(2n+1)), rounded to binary64
                exact = mp.factorial(2 * n) * mp.sqrt(mp.pi) / (mp.factorial(n) * 2 ** (2 * n + 1))
                assert r["c"] == float(exact)
                assert r["c0"] == float(mp.sqrt(mp.pi) / 2)


@pytest.mark.parametrize("cls,b", [("fp64", 53), ("fp32", 24), ("fp32x", 28)])
def test_cutoff_definition(cls, b):
    # z_nb solves z^(n+1/2) F_n(z) / c_n = 1 - 2^-b (the printed 1 - 2^b read with -b)
    for n in range(NMAX + 1):
        r = orc.record(cls, n)
        z = r["z"]
        hi, lo = orc.exact_one(np.array([z]), n)
        with mp.workdps(40):
            s = mp.mpf(2 * n + 1) / 2
            ratio = (mp.mpf(hi[0]) + mp.mpf(lo[0])) * mp.mpf(z) ** s / (mp.gamma(s) / 2)
            gap = -mp.log(1 - ratio, 2)
            assert abs(gap - b) < 1e-6, (cls, n, float(gap))


@pytest.mark.parametrize("cls", ALL_CLASSES)
def test_factor_structure(cls):
    # gathered factors have all-positive coefficients (roots with negative real parts,
    # the remark after Eq. qz); v has no zero on x >= 0; quadratic factors have a > 0
    for n in range(NMAX + 1):
        f = orc.record(cls, n).fields
        assert all(c > 0 for c in f["ug"] + f["vg"]), (cls, n)
        for side in ("u", "v"):
            q = f[side + "q"]
            assert all(q[2 * k] >= 0 and q[2 * k + 1] > 0 for k in range(len(q) // 2))
            assert all(y >= 0 for y in f[side + "l"])
            ys = [q[2 * k] for k in range(len(q) // 2)]
            assert ys == sorted(ys)
        assert not f["vl"], (cls, n)


@pytest.mark.parametrize("cls", ALL_CLASSES)
def test_factored_form_equals_expanded_rational(cls):
    # Eq. pqz with Eqs. pz, qz is the same function as Eq. qr: compare F~_n from the
    # oracle's binary128 factored evaluation with F~_n from P/D in mpmath
    g = np.random.default_rng(3)
    for n in (0, 1, 6, 13, 16, 25, 36):
        r = orc.record(cls, n)
        x = np.sort(g.uniform(0, r["z"], 12))
        hi, lo = orc.approx_exact_n(x, n, cls)
        with mp.workdps(45):
            A = [mp.mpf(a.numerator) / a.denominator for a in r["A"]]
            B = [mp.mpf(b.numerator) / b.denominator for b in r["B"]]
            s = mp.mpf(2 * n + 1) / 2
            c = mp.gamma(s) / 2
            for i, xv in enumerate(x):
                xm = mp.mpf(xv)
                Q = mp.polyval(A[::-1], xm) / mp.polyval(B[::-1], xm)
                F = c / (xm + Q ** s * mp.exp(-xm)) ** s
                got = mp.mpf(hi[i]) + mp.mpf(lo[i])
                assert abs(got / F - 1) < 1e-28, (cls, n, xv)


def exact_arith_bits(cls, n, k=1 << 13, fields=None):
    r = orc.record(cls, n)
    x = (np.arange(k) * (r["z"] / k))[1:]
    fh, fl = orc.approx_exact_n(x, n, cls, fields)
    eh, el = orc.exact_one(x, n)
    rel = ((fh - eh) + (fl - el)) / eh
    return orc.bits(rel)


@pytest.mark.parametrize("cls", CLASSES)
def test_exact_arithmetic_error_matches_table1(cls, table1):
    # Table 1, column epsilon_n: -log2 max |F~_n/F_n - 1| with exact arithmetic, measured
    # here on 2^13 evenly spaced points of [0, z_nb) in binary128
    worst = []
    for n in range(NMAX + 1):
        got = exact_arith_bits(cls, n)
        want = table1[n][cls]["en"]
        worst.append((abs(got - want), n, got, want))
        assert abs(got - want) <= 0.3 + 1e-9, (cls, n, got, want)


def test_fp32x_sets_reach_28_bits_with_the_smallest_N():
    # the binary32-output class computed in binary64: every order reaches 28 bits in
    # exact arithmetic over [0, z_{n,28}) (measured against the exact oracle), agrees with
    # the error recorded by the fit, and uses no more terms than the binary64 set of Table 1
    for n in range(NMAX + 1):
        r = orc.record("fp32x", n)
        got = exact_arith_bits("fp32x", n)
        assert got >= 28.0 - 0.02, (n, got)
        assert abs(got - r["eps"][0]) <= 0.3, (n, got, r["eps"])
        assert 4 <= r.N <= orc.record("fp64", n).N, n


def test_pin_detects_a_wrong_q1_or_a_dropped_term():
    # the E_n pin is sensitive: a slip in q1 or losing the q2 term costs many bits
    r = orc.record("fp64", 16)
    base = exact_arith_bits("fp64", 16, 1 << 11)
    bad_q1 = exact_arith_bits("fp64", 16, 1 << 11, {"q1x": r["q1x"] * Fraction(1001, 1000)})
    no_q2 = exact_arith_bits("fp64", 16, 1 << 11, {"q2x": Fraction(0)})
    assert base > 48.5 and bad_q1 < base - 10 and no_q2 < 10
