"""Pins of the oracle's finite-precision evaluation of the approximant.

Table 1 prints, for binary64 and binary32 arithmetic, the largest relative errors of F_0,
F_{n-1} (from the downward recursion) and F_n (from the approximant) over ~2^20 evenly
spaced points of [0, z_nb).  The oracle's binary64 evaluation, with re-fitted
coefficients, must land within one bit of those numbers; a dropped term, a wrong index in
the recursion or a wrong cut-off moves them by far more.  The mixed class (binary32
rational and recursion, binary64 power) has no column of its own in the paper; it is held
to the binary32 columns minus one bit.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc

GRID = 1 << 16
NS = list(range(37))   # every order of Table 1


def ebar(cls, n, rec=None, k=GRID):
    r = rec if rec is not None else orc.record(cls, n)
    x = np.arange(k) * (r["z"] / k)
    A = orc.approx_f64(x, n, rec) if cls == "fp64" else orc.approx_mixed(x, n, rec)
    A = A.astype(np.float64)
    out = {}
    for key, m in (("eb0", 0), ("ebn1", n - 1), ("ebn", n)):
        if m < 0:
            continue
        hi, lo = orc.exact_one(x, m)
        out[key] = orc.bits(orc.rel_err(A[m], hi, lo))
    return out


@pytest.mark.parametrize("n", NS)
def test_binary64_finite_precision_error_matches_table1(n, table1):
    got = ebar("fp64", n)
    want = table1[n]["fp64"]
    for key, v in got.items():
        if want[key] is None:
            continue
        assert abs(v - want[key]) <= 1.0, (n, key, v, want[key])


@pytest.mark.parametrize("n", NS)
def test_mixed_class_at_least_the_binary32_columns(n, table1):
    got = ebar("fp32", n)
    want = table1[n]["fp32"]
    for key, v in got.items():
        if want[key] is None:
            continue
        assert v >= want[key] - 1.0, (n, key, v, want[key])


def test_kappa_is_the_rounded_root_of_c_n():
    # F_n = c_n / G^(n+1/2) = (kappa_n / G)^(n+1/2): kappa_n = c_n^(1/(n+1/2)), c_n =
    # Gamma(n+1/2)/2 (the x -> inf limit of Eq. fn), rounded once to binary32; checked at
    # 50 digits against both neighbouring binary32 values
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    for n in NS:
        s = mpmath.mpf(n) + mpmath.mpf(1) / 2
        exact = (mpmath.gamma(s) / 2) ** (1 / s)
        k = np.float32(orc.kappa32(n))
        lo, hi = np.nextafter(k, np.float32(0)), np.nextafter(k, np.float32(np.inf))
        d = abs(mpmath.mpf(float(k)) - exact)
        assert d <= abs(mpmath.mpf(float(lo)) - exact) and d <= abs(mpmath.mpf(float(hi)) - exact), n


@pytest.mark.parametrize("n", NS)
def test_all_binary32_evaluation_matches_table1(n, table1):
    # Table 1's binary32 columns are all-binary32 arithmetic: the oracle's evaluation of the
    # binary32 sets in binary32 (F_n = (kappa_n / G)^(n+1/2)) lands within one bit of them
    r = orc.record("fp32", n)
    x = np.arange(GRID) * (r["z"] / GRID)
    A = orc.approx_single(x, n).astype(np.float64)
    want = table1[n]["fp32"]
    for key, m in (("eb0", 0), ("ebn1", n - 1), ("ebn", n)):
        if m < 0 or want[key] is None:
            continue
        hi, lo = orc.exact_one(x, m)
        ok = np.abs(hi) >= 1.1754943508222875e-38
        got = orc.bits(orc.rel_err(A[m][ok], hi[ok], lo[ok]))
        assert abs(got - want[key]) <= 1.0, (n, key, got, want[key])


def test_value_at_zero():
    # F~_m(0) must be 1/(2m+1) to the accuracy of the approximant
    for n in (0, 5, 16, 36):
        F = orc.approx_f64(np.zeros(1), n)[:, 0]
        want = 1.0 / (2 * np.arange(n + 1) + 1)
        assert np.max(np.abs(F / want - 1)) < 2.0 ** -40


def test_special_inputs():
    x = np.array([-1.0, np.nan, np.inf, -0.0, 0.0])
    for n in (0, 9):
        F = orc.approx_f64(x, n)
        G = orc.approx_mixed(x, n)
        H = orc.approx_single(x, n)
        assert np.all(np.isnan(H[:, :2])) and np.all(H[:, 2] == 0)
        assert np.array_equal(H[:, 3], H[:, 4])
        assert np.all(np.isnan(F[:, :2])) and np.all(np.isnan(G[:, :2]))
        assert np.all(F[:, 2] == 0) and np.all(G[:, 2] == 0)
        assert np.array_equal(F[:, 3], F[:, 4]) and np.array_equal(G[:, 3], G[:, 4])


@pytest.mark.parametrize("cls,b", [("fp64", 53), ("fp32", 24)])
def test_past_the_cutoff_and_large_arguments(cls, b):
    # above z_nb every order is the long-range limit (Eq. limf1), accurate to about 2^-b
    # plus the rounding of the upward product; far above, nothing under- or overflows early
    for n in (0, 4, 16, 36):
        z = orc.record(cls, n)["z"]
        x = np.concatenate([np.nextafter(z, np.inf) * np.array([1.0, 1.0001, 1.5, 3.0]),
                            [1e4, 1e8, 1e12, 1e30]])
        A = (orc.approx_f64(x, n) if cls == "fp64" else orc.approx_mixed(x, n)).astype(float)
        hi, lo = orc.exact(x, n)
        for m in range(n + 1):
            ok = np.abs(hi[m]) >= (2.2250738585072014e-308 if cls == "fp64"
                                   else 1.1754943508222875e-38)
            e = orc.rel_err(A[m][ok], hi[m][ok], lo[m][ok])
            assert orc.bits(e) >= (b - 6), (cls, n, m, orc.bits(e))
        assert A[0, -1] > 0  # F_0(1e30) = sqrt(pi)/2e15 is not lost to underflow


@pytest.mark.parametrize("n", NS)
def test_fp32x_class_within_half_a_binary32_ulp(n):
    # binary32 outputs computed in binary64 from the ~28-bit approximant: every normal
    # value within half a binary32 ulp plus 2^-27.5 relative of the exact F_m, below and
    # above the cut-off z_{n,28}; subnormal outputs within half the subnormal spacing plus
    # 2^-27.5 of FLT_MIN
    r = orc.record("fp32x", n)
    k = 1 << 14
    x = np.concatenate([np.arange(k) * (r["z"] / k),
                        r["z"] * (1.0 + np.arange(1, 257) / 64.0), [1e3, 1e6, 1e12]])
    A = orc.approx_f32x(x, n)
    hi, lo = orc.exact(x, n)
    fmin = 1.1754943508222875e-38
    for m in range(n + 1):
        F = hi[m] + lo[m]
        err = np.abs(A[m].astype(np.float64) - hi[m] - lo[m])
        half_ulp = 0.5 * np.spacing(np.abs(F).astype(np.float32)).astype(np.float64)
        tol = half_ulp + 2.0 ** -27.5 * np.maximum(np.abs(F), fmin)
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, (n, m, x[bad[:3]], err[bad[:3]], tol[bad[:3]])


@pytest.mark.parametrize("n,nbar", [(36, 0), (36, 16), (20, 4), (16, 8), (16, 15)])
def test_two_approximation_option_improves_the_low_orders(n, nbar, table1):
    # over [0, 1.2 z_n): rows above nbar are the order-n evaluation's; every row up to nbar
    # is within the Table 1 bounds of row nbar; rows up to nbar-2 are never worse than
    # the order-n recursion leaves them, and F_0 gains when the recursion saved is long.
    # (F_nbar itself carries the order-nbar approximant's own error, the weakest column
    # of Table 1, which can be below what a longer recursion recovers: measured 44.4 vs
    # 46.7 bits at n = 36, nbar = 16.)
    k = 1 << 14
    z = orc.record("fp64", n)["z"]
    x = np.arange(k) * (1.2 * z / k)
    S = orc.approx_split(x, n, nbar)
    P = orc.approx_f64(x, n)
    assert np.array_equal(S[nbar + 1:], P[nbar + 1:])
    t = table1[nbar]["fp64"]
    ebn1 = t["ebn1"] if t["ebn1"] is not None else t["eb0"]
    bounds = [min(t["eb0"], ebn1) - 1.0] * (nbar + 1)
    if nbar >= 1:
        bounds[nbar - 1] = ebn1 - 1.0
    bounds[nbar] = t["ebn"] - 1.0
    gain0 = None
    for m in range(nbar + 1):
        hi, lo = orc.exact_one(x, m)
        bs = orc.bits(orc.rel_err(S[m], hi, lo))
        bp = orc.bits(orc.rel_err(P[m], hi, lo))
        assert bs >= bounds[m], (n, nbar, m, bs, bounds[m])
        if m <= nbar - 2:
            assert bs >= bp - 0.25, (n, nbar, m, bs, bp)
        if m == 0:
            gain0 = bs - bp
    if n - nbar >= 8:
        assert gain0 > 0.5, (n, nbar, gain0)


def test_pin_detects_planted_mistakes():
    # a wrong q1, or swapping the gathered factors of u and v, breaks the Table 1 pin
    r = orc.record("fp64", 16)
    ok = ebar("fp64", 16, r, k=1 << 12)
    bad = orc.Record("fp64", 16, r.N)
    bad.fields = dict(r.fields)
    bad.fields["q1"] = r["q1"] * 1.0001
    got = ebar("fp64", 16, bad, k=1 << 12)
    assert got["ebn"] < ok["ebn"] - 8
    swap = orc.Record("fp64", 16, r.N)
    swap.fields = dict(r.fields)
    swap.fields["ug"], swap.fields["vg"] = r["vg"], r["ug"]
    got = ebar("fp64", 16, swap, k=1 << 12)
    assert got["ebn"] < 20


def _w_binary32(x, r, n):
    """W = Q~^n sqrt(Q~) e of the mixed class, recomputed here in numpy binary32 from the
    record's binary32 coefficients (Eqs. pqz, pz, qz, fq; left to right as written), with
    e = RN32(RN64(exp(-x))) taken from mpmath at 50 digits."""
    mpmath = pytest.importorskip("mpmath")
    f32 = np.float32
    xf = x.astype(f32)
    with mpmath.workdps(50):
        e = np.array([float(mpmath.exp(-mpmath.mpf(float(v)))) for v in x]).astype(f32)

    def fac(g, q, l):
        p = np.ones_like(xf)
        for gk in reversed(g):
            p = p * xf + f32(gk)
        for k in range(len(q) // 2):
            d = xf - f32(q[2 * k])
            p = p * (d * d + f32(q[2 * k + 1]))
        for lk in l:
            p = p * (xf - f32(lk))
        return p

    u = fac(r["ug"], r["uq"], r["ul"])
    v = fac(r["vg"], r["vq"], r["vl"])
    Q = (f32(r["q0"]) + f32(r["q1"]) * xf) + ((f32(r["q2"]) * (u / v)) * xf) * xf
    P = np.ones_like(Q) if n == 0 else Q.copy()
    if n > 0:
        for b in range(int(n).bit_length() - 2, -1, -1):
            P = P * P
            if (n >> b) & 1:
                P = P * Q
    return (P * np.sqrt(Q)) * e


@pytest.mark.parametrize("n", [0, 1, 4, 8, 16, 20, 27, 36])
def test_mixed_class_binary64_stage(n):
    # The mixed class takes G = x + W and c_n / G^(n+1/2) (Eq. fq) in binary64, on the
    # binary64 argument: with W as binary32 arithmetic leaves it, F_n must be the exact
    # c_n / (x + W)^(n+1/2) rounded to binary32, within one binary32 ulp.  In binary32
    # (G = RN32(x) + W, or (kappa_n / G)^(n+1/2)) the power amplifies a rounding of G by
    # n + 1/2: several ulps from n = 4 on, which this catches.
    mpmath = pytest.importorskip("mpmath")
    r = orc.record("fp32", n)
    g = np.random.default_rng(1000 + n)
    x = np.concatenate([np.sort(g.uniform(0.0, r["z"], 1500)),
                        np.exp(g.uniform(np.log(1e-6), np.log(1.0), 300))])
    W = _w_binary32(x, r, n)
    got = orc.approx_mixed(x, n)[n]
    s = mpmath.mpf(n) + mpmath.mpf(1) / 2
    with mpmath.workdps(50):
        c = mpmath.gamma(s) / 2
        want = np.array([float(c / (mpmath.mpf(float(xi)) + mpmath.mpf(float(wi))) ** s)
                         for xi, wi in zip(x, W)]).astype(np.float32)
    d = np.abs(got.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
    assert d.max() <= 1, (n, x[np.argmax(d)], int(d.max()))


@pytest.mark.parametrize("n", [8, 12, 16, 24, 36])
def test_mixed_class_beats_all_binary32_in_the_recursion(n):
    # The binary64 power is what sets the mixed class apart from Table 1's all-binary32
    # arithmetic: on Table 1's grid its F_m gain at least half a bit at some mid order.
    r = orc.record("fp32", n)
    x = np.arange(1 << 14) * (r["z"] / (1 << 14))
    A = orc.approx_mixed(x, n).astype(np.float64)
    S = orc.approx_single(x, n).astype(np.float64)
    gains = []
    for m in range(n // 4, 3 * n // 4 + 1):
        hi, lo = orc.exact_one(x, m)
        ok = np.abs(hi) >= 1.1754943508222875e-38
        gains.append(orc.bits(orc.rel_err(A[m][ok], hi[ok], lo[ok]))
                     - orc.bits(orc.rel_err(S[m][ok], hi[ok], lo[ok])))
    assert max(gains) >= 0.5, (n, gains)


def _horner(c, x):
    p = np.zeros_like(x) + c[-1]
    for a in c[-2::-1]:
        p = p * x + a
    return p


@pytest.mark.parametrize("n,gain", [(16, 0.5), (20, 2.0), (36, 5.0)])
def test_factored_form_beats_the_expanded_rational_in_binary64(n, gain):
    # The paper's remark in section "Computations": in finite precision the expanded
    # rational of Eq. qr loses accuracy at higher n that the root-factored form of
    # Eqs. pqz, pz, qz keeps.  Here the expanded numerator and denominator (the record's
    # coefficients rounded once to binary64) go through Horner's rule, then Eq. fq in
    # binary64; the oracle's factored evaluation must be the more accurate F_n.
    r = orc.record("fp64", n)
    x = np.arange(GRID) * (r["z"] / GRID)
    A = [float(a) for a in r["A"]]
    B = [float(b) for b in r["B"]]
    Q = _horner(A, x) / _horner(B, x)
    e = orc.exp_neg(x)
    Qn = np.ones_like(x)
    for _ in range(n):
        Qn = Qn * Q
    G = x + Qn * np.sqrt(Q) * e
    Gn = np.ones_like(x)
    for _ in range(n):
        Gn = Gn * G
    F = r["c"] / (Gn * np.sqrt(G))
    hi, lo = orc.exact_one(x, n)
    expanded = orc.bits(orc.rel_err(F, hi, lo))
    factored = ebar("fp64", n)["ebn"]
    assert factored >= expanded + gain, (n, factored, expanded)
