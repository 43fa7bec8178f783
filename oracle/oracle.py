"""Python face of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads ``liboracle.so`` (plain C, built from ``boys_oracle.c`` by
``build()`` below) and reads the coefficient dataset with its own parser.  It shares
no code with the GPU library or its Python binding.

Functions
---------
exact(x, mmax)            F_m(x), m = 0..mmax, from the definition (Eq. fn), as
                          double-double (hi, lo) arrays of shape (mmax+1, len(x)).
exact_one(x, m)           the same for one order m, arrays of shape (len(x),).
approx_f64(x, n)          the binary64 approximant (Eqs. fq, pqz, pz, qz, r, limf1),
                          shape (n+1, len(x)), float64.
approx_mixed(x, n)        the mixed binary32/binary64 class, shape (n+1, len(x)), float32.
approx_single(x, n)       the all-binary32 evaluation (Table 1's binary32 arithmetic), float32.
approx_f32x(x, n)         the binary32-output class computed in binary64 (the ~28-bit
                          approximant, each value rounded once), shape (n+1, len(x)), float32.
approx_split(x, n, nbar)  the two-approximation option: rows 0..nbar of approx_f64(x, nbar)
                          over rows nbar+1..n of approx_f64(x, n).
eri_ssss(...)             a consumer of F_m: contracted (ss|ss)^(m) integrals of s Gaussians.
approx_exact_n(x, n)      F~_n in binary128 from the 40-digit coefficients, as (hi, lo).
exp_neg(x)                correctly rounded exp(-x) as both approximants use it.
load_dataset(path)        the parsed coefficient dataset.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "boys_oracle.c")
DATASET = os.path.join(REPO, "paper_2504_07637_amd", "data", "boys_coeffs.txt")


NATIVE_LIB_PATH = os.path.join(HERE, "liboracle_native.so")


def build(force: bool = False, native: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE arithmetic, no contraction).  native: the
    same source at -O3 -march=native for the host it runs on (the timed CPU baseline; the
    same IEEE operations, since nothing is contracted)."""
    path = NATIVE_LIB_PATH if native else LIB_PATH
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        tmp = f"{path}.tmp{os.getpid()}"  # concurrent builders each write their own file
        cmd = ["gcc", *opt, "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, SRC, "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


_lib = None


def use_native_build():
    """Build the same source at -O3 -march=native for this host and route every later
    call through it (the CPU-baseline timing)."""
    global _lib
    _lib = _load(build(force=True, native=True))


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


def _load(path):
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64 = ctypes.c_int64
    L.oracle_boys_exact.argtypes = [dp, i64, ctypes.c_int, dp, dp]
    L.oracle_boys_exact_one.argtypes = [dp, i64, ctypes.c_int, dp, dp]
    L.oracle_boys_approx_f64.argtypes = [dp, i64, dp, ctypes.c_int, dp, i64]
    L.oracle_boys_approx_mixed.argtypes = [dp, i64, dp, ctypes.c_int, fp, i64]
    L.oracle_boys_approx_f64r.argtypes = [dp, i64, dp, ctypes.c_int, dp, i64]
    L.oracle_boys_approx_f64r.restype = ctypes.c_int
    L.oracle_boys_approx_single.argtypes = [dp, i64, dp, ctypes.c_int, fp, i64]
    L.oracle_boys_approx_single.restype = ctypes.c_int
    L.oracle_kappa32.argtypes = [ctypes.c_int]
    L.oracle_kappa32.restype = ctypes.c_float
    L.oracle_boys_approx_q.argtypes = [dp, i64, dp, dp, dp]
    L.oracle_exp_neg.argtypes = [dp, i64, dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    L.oracle_eri_ssss.argtypes = [dp, ctypes.c_int, dp, i64, ip, ctypes.c_int32, dp, i64, ip,
                                  ctypes.c_int32, dp, i64]
    L.oracle_eri_ssss.restype = ctypes.c_int
    L.oracle_eri_prefactor.argtypes = []
    L.oracle_eri_prefactor.restype = ctypes.c_double
    for f in (L.oracle_boys_exact, L.oracle_boys_exact_one, L.oracle_boys_approx_f64, L.oracle_boys_approx_mixed,
              L.oracle_boys_approx_q, L.oracle_exp_neg):
        f.restype = ctypes.c_int
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


# ------------------------------------------------------------------------------------
# dataset


class Record:
    """One (precision class, n) approximant.  Fields hold Python floats (hex-exact)
    and, with suffix ``x``, Fractions of the 40-digit decimal values."""

    def __init__(self, cls, n, N):
        self.cls, self.n, self.N = cls, n, N
        self.fields = {}

    def __getitem__(self, k):
        return self.fields[k]


def _parse_hex_list(tok, pairs=False):
    k = int(tok[0])
    vals = [float.fromhex(t) for t in tok[1:]]
    if len(vals) != (2 * k if pairs else k):
        raise ValueError("bad count in dataset line")
    return vals


def _parse_dec_list(tok, pairs=False):
    k = int(tok[0])
    vals = [Fraction(t) for t in tok[1:]]
    if len(vals) != (2 * k if pairs else k):
        raise ValueError("bad count in dataset line")
    return vals


def load_dataset(path: str = DATASET):
    recs = {}
    c0 = None
    cur = None
    with open(path) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            key = tok[0]
            if key == "format":
                if tok[1:] != ["boys-coeffs", "1"]:
                    raise ValueError("unknown dataset format")
            elif key == "c0":
                c0 = float.fromhex(tok[1])
            elif key == "record":
                cur = Record(tok[1], int(tok[2]), int(tok[3]))
            elif key == "end":
                cur.fields["c0"] = c0
                recs[(cur.cls, cur.n)] = cur
                cur = None
            elif key in ("c", "z", "q0", "q1", "q2"):
                cur.fields[key] = float.fromhex(tok[1])
                cur.fields[key + "x"] = Fraction(tok[2])
            elif key in ("ug", "ul", "vg", "vl"):
                cur.fields[key] = _parse_hex_list(tok[1:])
            elif key in ("uq", "vq"):
                cur.fields[key] = _parse_hex_list(tok[1:], pairs=True)
            elif key in ("ugx", "ulx", "vgx", "vlx"):
                cur.fields[key] = _parse_dec_list(tok[1:])
            elif key in ("uqx", "vqx"):
                cur.fields[key] = _parse_dec_list(tok[1:], pairs=True)
            elif key in ("A", "B"):
                cur.fields[key] = _parse_dec_list(tok[1:])
            elif key == "eps":
                cur.fields["eps"] = (float(tok[1]), float(tok[2]))
            else:
                raise ValueError(f"unknown dataset key {key!r}")
    return recs


_DATA = None


def dataset():
    global _DATA
    if _DATA is None:
        _DATA = load_dataset()
    return _DATA


def record(cls: str, n: int) -> Record:
    return dataset()[(cls, n)]


def flat_record(r: Record) -> np.ndarray:
    """The rec[] layout of boys_oracle.c."""
    f = r.fields
    out = [float(r.n), f["c"], f["z"], f["q0"], f["q1"], f["q2"], f["c0"]]
    for side in ("u", "v"):
        g, q, l = f[side + "g"], f[side + "q"], f[side + "l"]
        out += [float(len(g))] + g + [float(len(q) // 2)] + q + [float(len(l))] + l
    return np.array(out, dtype=np.float64)


def _dd(fr: Fraction):
    hi = float(fr)
    lo = float(fr - Fraction(hi))
    return [hi, lo]


def flat_record_ext(r: Record, fields=None) -> np.ndarray:
    """The recx[] layout of boys_oracle.c (double-double coefficients)."""
    f = dict(r.fields)
    if fields:
        f.update(fields)
    out = [float(r.n)]
    for k in ("q0x", "q1x", "q2x"):
        out += _dd(f[k])
    for side in ("u", "v"):
        g, q, l = f[side + "gx"], f[side + "qx"], f[side + "lx"]
        out += [float(len(g))]
        for v in g:
            out += _dd(v)
        out += [float(len(q) // 2)]
        for v in q:
            out += _dd(v)
        out += [float(len(l))]
        for v in l:
            out += _dd(v)
    return np.array(out, dtype=np.float64)


# ------------------------------------------------------------------------------------
# evaluators


def exact(x, mmax: int):
    x = np.ascontiguousarray(x, dtype=np.float64)
    hi = np.empty((mmax + 1, x.size))
    lo = np.empty((mmax + 1, x.size))
    rc = lib().oracle_boys_exact(_dp(x), x.size, mmax, _dp(hi), _dp(lo))
    if rc:
        raise ValueError("oracle_boys_exact rejected its arguments")
    return hi, lo


def exact_one(x, m: int):
    """F_m(x) for one order m, as (hi, lo)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    hi = np.empty(x.size)
    lo = np.empty(x.size)
    rc = lib().oracle_boys_exact_one(_dp(x), x.size, m, _dp(hi), _dp(lo))
    if rc:
        raise ValueError("oracle_boys_exact_one rejected its arguments")
    return hi, lo


def approx_f64(x, n: int, rec: Record | None = None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = rec if rec is not None else record("fp64", n)
    fr = flat_record(r)
    out = np.empty((n + 1, x.size))
    rc = lib().oracle_boys_approx_f64(_dp(x), x.size, _dp(fr), fr.size, _dp(out), x.size)
    if rc:
        raise ValueError("oracle_boys_approx_f64 rejected its arguments")
    return out


def approx_mixed(x, n: int, rec: Record | None = None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = rec if rec is not None else record("fp32", n)
    fr = flat_record(r)
    out = np.empty((n + 1, x.size), dtype=np.float32)
    rc = lib().oracle_boys_approx_mixed(_dp(x), x.size, _dp(fr), fr.size, _fp(out), x.size)
    if rc:
        raise ValueError("oracle_boys_approx_mixed rejected its arguments")
    return out


def approx_single(x, n: int, rec: Record | None = None):
    """The all-binary32 evaluation of the binary32 sets (the arithmetic of Table 1's
    binary32 columns), float32 (n+1, len(x))."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = rec if rec is not None else record("fp32", n)
    fr = flat_record(r)
    out = np.empty((n + 1, x.size), dtype=np.float32)
    rc = lib().oracle_boys_approx_single(_dp(x), x.size, _dp(fr), fr.size, _fp(out), x.size)
    if rc:
        raise ValueError("oracle_boys_approx_single rejected its arguments")
    return out


def kappa32(n: int) -> float:
    """c_n^(1/(n+1/2)) rounded to binary32, as the oracle computes it."""
    return float(lib().oracle_kappa32(n))


def approx_f32x(x, n: int, rec: Record | None = None):
    """The binary64 evaluation of the ~28-bit approximant (the steps of approx_f64 with the
    record's own cut-off, each recursion step a multiplication by RN(1/(2m-1))), each
    value rounded to nearest binary32 once at the end."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = rec if rec is not None else record("fp32x", n)
    fr = flat_record(r)
    out = np.empty((n + 1, x.size))
    rc = lib().oracle_boys_approx_f64r(_dp(x), x.size, _dp(fr), fr.size, _dp(out), x.size)
    if rc:
        raise ValueError("oracle_boys_approx_f64r rejected its arguments")
    return out.astype(np.float32)


def approx_split(x, n: int, nbar: int):
    """The two-approximation option of section "Computations": F_0..F_nbar as the
    order-nbar evaluation gives them, F_{nbar+1}..F_n as the order-n evaluation does."""
    if not 0 <= nbar < n:
        raise ValueError("need 0 <= nbar < n")
    lo = approx_f64(x, nbar)
    hi = approx_f64(x, n)
    return np.concatenate([lo, hi[nbar + 1:]], axis=0)


def eri_prefactor() -> float:
    """2 pi^(5/2) rounded to binary64, as the (ss|ss) oracle uses it."""
    return float(lib().oracle_eri_prefactor())


def eri_ssss(bra, bstart, ket, kstart, n: int):
    """Contracted (ss|ss)^(m), m = 0..n (see boys_oracle.c, item 5): bra, ket are (5, k)
    float64 arrays of (p, Px, Py, Pz, w); bstart, kstart int32 CSR offsets.  Returns
    (n+1, n_bra * n_ket)."""
    bra = np.ascontiguousarray(bra, dtype=np.float64)
    ket = np.ascontiguousarray(ket, dtype=np.float64)
    bstart = np.ascontiguousarray(bstart, dtype=np.int32)
    kstart = np.ascontiguousarray(kstart, dtype=np.int32)
    nb, nk = bstart.size - 1, kstart.size - 1
    fr = flat_record(record("fp64", n))
    out = np.empty((n + 1, nb * nk))
    ip = ctypes.POINTER(ctypes.c_int32)
    rc = lib().oracle_eri_ssss(_dp(fr), fr.size, _dp(bra), bra.shape[1],
                               bstart.ctypes.data_as(ip), nb, _dp(ket), ket.shape[1],
                               kstart.ctypes.data_as(ip), nk, _dp(out), max(1, nb * nk))
    if rc:
        raise ValueError("oracle_eri_ssss rejected its arguments")
    return out


def approx_exact_n(x, n: int, cls: str = "fp64", fields=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    fr = flat_record_ext(record(cls, n), fields)
    hi = np.empty(x.size)
    lo = np.empty(x.size)
    lib().oracle_boys_approx_q(_dp(x), x.size, _dp(fr), _dp(hi), _dp(lo))
    return hi, lo


def exp_neg(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.size)
    lib().oracle_exp_neg(_dp(x), x.size, _dp(out))
    return out


def rel_err(approx, hi, lo):
    """(approx - F) / F with F = hi + lo, elementwise, in binary64."""
    a = np.asarray(approx, dtype=np.float64)
    return ((a - hi) - lo) / hi


def bits(e) -> float:
    """-log2 of the largest |e|."""
    m = float(np.max(np.abs(e)))
    return float("inf") if m == 0 else -np.log2(m)
