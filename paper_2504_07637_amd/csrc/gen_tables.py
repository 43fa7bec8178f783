"""Generate boys_tables.inc for the HIP library from the coefficient dataset.

The header holds, as hexadecimal floating-point literals:
  * per (precision class, n) the root-factored approximant of Eqs. pqz, pz, qz
    (F64Set: binary64, F32Set: binary32 values, F32xSet: the ~28-bit sets, binary64):
    c_n, the cut-off z_nb, q0, q1, q2 and the factor lists of u and v;
  * the binary64 sets once more as one runtime-indexed table (RtSet headers and one
    flat coefficient array), for the two-approximation option whose lower order is a
    launch argument;
  * c_0 = sqrt(pi)/2 for the long-range limit past the cut-off (Eq. limf1),
    2 pi^(5/2) for the (ss|ss) integrals of the consumer kernel, and kappa_n =
    c_n^(1/(n+1/2)) in binary32 for the all-binary32 class;
  * the tables of the correctly rounded exponential: 2^(j/256) for j = 0..255 as
    double-double pairs, and ln2/256 split into three parts for an exact reduction.

Run by the build step; the output is not edited by hand.
"""
from __future__ import annotations

import os
import sys

import mpmath as mp

HERE = os.path.dirname(os.path.abspath(__file__))
DATASET = os.path.join(os.path.dirname(HERE), "data", "boys_coeffs.txt")
OUT = os.path.join(HERE, "boys_tables.inc")


def read_dataset(path):
    recs = {}
    c0 = None
    cur = None
    with open(path) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].split()
            if not line:
                continue
            key, rest = line[0], line[1:]
            if key == "format":
                assert rest == ["boys-coeffs", "1"], rest
            elif key == "c0":
                c0 = rest[0]
            elif key == "record":
                cur = {"cls": rest[0], "n": int(rest[1]), "N": int(rest[2])}
            elif key == "end":
                recs[(cur["cls"], cur["n"])] = cur
                cur = None
            elif key in ("c", "z", "q0", "q1", "q2"):
                cur[key] = rest[0]
            elif key in ("ug", "ul", "vg", "vl"):
                k = int(rest[0])
                vals = rest[1:]
                assert len(vals) == k
                cur[key] = vals
            elif key in ("uq", "vq"):
                k = int(rest[0])
                vals = rest[1:]
                assert len(vals) == 2 * k
                cur[key] = vals
            # extended-precision and expanded entries are not used by the kernels
    return c0, recs


def lit(h: str, single: bool) -> str:
    v = float.fromhex(h)
    if single:
        # the dataset stores binary32 values for this class; keep them exact
        import struct
        assert struct.unpack("f", struct.pack("f", v))[0] == v, h
        return float.hex(v) + "f"
    return float.hex(v)


def arr(name, vals, single):
    ty = "float" if single else "double"
    body = ", ".join(lit(v, single) for v in vals) if vals else ("0.0f" if single else "0.0")
    size = max(1, len(vals))
    return f"  static constexpr int {name}_n = {len(vals) // (2 if name.endswith('q') else 1)};\n" \
           f"  static constexpr {ty} {name}[{size}] = {{{body}}};\n"


def emit_record(r):
    single = r["cls"] == "fp32"
    name = {"fp32": "F32Set", "fp64": "F64Set", "fp32x": "F32xSet"}[r["cls"]]
    s = f"template <> struct {name}<{r['n']}> {{\n"
    s += f"  static constexpr int N = {r['N']};\n"
    s += f"  static constexpr double c = {lit(r['c'], False)};\n"
    s += f"  static constexpr double z = {lit(r['z'], False)};\n"
    ty = "float" if single else "double"
    for k in ("q0", "q1", "q2"):
        s += f"  static constexpr {ty} {k} = {lit(r[k], single)};\n"
    for k in ("ug", "uq", "ul", "vg", "vq", "vl"):
        s += arr(k, r[k], single)
    s += "};\n"
    return s


def emit_runtime(recs, cls, nmax):
    """RtSet headers and the flat coefficient array (per set: ug, uq, ul, vg, vq, vl)."""
    heads, coefs = [], []
    for n in range(nmax + 1):
        r = recs[(cls, n)]
        cnt = [len(r["ug"]), len(r["uq"]) // 2, len(r["ul"]),
               len(r["vg"]), len(r["vq"]) // 2, len(r["vl"])]
        heads.append("  {" + ", ".join(lit(r[k], False) for k in ("c", "z", "q0", "q1", "q2"))
                     + ", " + ", ".join(str(c) for c in cnt) + f", {len(coefs)}}},")
        for k in ("ug", "uq", "ul", "vg", "vq", "vl"):
            coefs += r[k]
    out = ["// the binary64 sets, indexed at run time",
           "struct RtSet {",
           "  double c, z, q0, q1, q2;",
           "  int ug_n, uq_n, ul_n, vg_n, vq_n, vl_n;  // factor counts (uq, vq: pairs)",
           "  int off;                                 // first coefficient in kRtCoef64",
           "};",
           f"constexpr RtSet kRt64[{nmax + 1}] = {{"] + heads + ["};",
           f"constexpr double kRtCoef64[{len(coefs)}] = {{"]
    for i in range(0, len(coefs), 4):
        out.append("  " + ", ".join(lit(v, False) for v in coefs[i:i + 4]) + ",")
    out.append("};")
    return out


def exp_tables():
    mp.mp.prec = 300
    ln2 = mp.log(2)
    step = ln2 / 256
    # L1 keeps 36 significant bits so that k * L1 is exact for |k| < 2^17
    e = mp.floor(mp.log(step, 2))
    scale = mp.mpf(2) ** (35 - e)
    L1 = mp.floor(step * scale + mp.mpf(1) / 2) / scale
    L2 = mp.mpf(float(step - L1))
    L3 = mp.mpf(float(step - L1 - L2))
    inv = 256 / ln2
    tab = []
    for j in range(256):
        t = mp.mpf(2) ** (mp.mpf(j) / 256)
        hi = float(t)
        lo = float(t - mp.mpf(hi))
        tab += [hi, lo]
    return float(L1), float(L2), float(L3), float(inv), tab


def exp_coeffs():
    """1/k! as double-double (k = 2..4 need the low part) and doubles for the tail."""
    mp.mp.prec = 300
    out = {}
    for k in range(2, 12):
        v = 1 / mp.factorial(k)
        hi = float(v)
        lo = float(v - mp.mpf(hi))
        out[k] = (hi, lo)
    return out


def main(dataset=DATASET, out=OUT):
    c0, recs = read_dataset(dataset)
    def top(cls):
        ns = sorted(n for (c, n) in recs if c == cls)
        ok = [n for n in ns if all(k in ns for k in range(n + 1))]
        return max(ok) if ok else -1
    max64, max32, max32x = top("fp64"), top("fp32"), top("fp32x")
    L1, L2, L3, inv, tab = exp_tables()
    fac = exp_coeffs()
    lines = ["// Generated by gen_tables.py from data/boys_coeffs.txt. Do not edit.",
             "#pragma once",
             "namespace boys_tab {",
             "// The coefficient arrays of the binary64 and fp32x sets have internal linkage: the",
             "// device compiler then treats them as ordinary constants and an element read at a",
             "// fixed index becomes an immediate operand.  Static constexpr arrays with external",
             "// linkage are emitted as externally initialised device constants, read from memory",
             "// with scalar loads; the binary32 sets stay that way (one load fetches several",
             "// coefficients into SGPRs, which their kernels run slightly faster with).  Inside a",
             "// loop over many inlined sets (the persistent batched kernel) those loads are hoisted",
             "// and held live, so the binary64 sets, the largest part, are immediates.",
             "template <int n> struct F32Set;",
             "namespace {",
             f"constexpr int kMaxN64 = {max64};",
             f"constexpr int kMaxN32 = {max32};",
             f"constexpr int kMaxN32x = {max32x};",
             f"constexpr double kC0 = {lit(c0, False)};  // sqrt(pi)/2",
             "template <int n> struct F64Set;",
             "template <int n> struct F32xSet;"]
    for n in range(max64 + 1):
        lines.append(emit_record(recs[("fp64", n)]))
    lines.append("}  // namespace")
    for n in range(max32 + 1):
        lines.append(emit_record(recs[("fp32", n)]))
    lines.append("namespace {")
    for n in range(max32x + 1):
        lines.append(emit_record(recs[("fp32x", n)]))
    lines += emit_runtime(recs, "fp64", max64)
    lines.append("constexpr double kCut64[] = {" + ", ".join(
        lit(recs[("fp64", n)]["z"], False) for n in range(max64 + 1)) + "};")
    lines.append("constexpr double kCut32[] = {" + ", ".join(
        lit(recs[("fp32", n)]["z"], False) for n in range(max32 + 1)) + "};")
    lines.append("constexpr double kCut32x[] = {" + (", ".join(
        lit(recs[("fp32x", n)]["z"], False) for n in range(max32x + 1)) or "0.0") + "};")
    mp.mp.prec = 300
    lines.append(f"constexpr double kTwoPi52 = {float.hex(float(2 * mp.pi ** 2.5))};"
                 "  // 2 pi^(5/2), the (ss|ss) prefactor")
    # kappa_n = c_n^(1/(n+1/2)) rounded once to binary32: F_n = (kappa_n / G)^(n+1/2)
    # keeps the all-binary32 class in range (c_n itself exceeds binary32 beyond n = 27)
    import numpy as np
    kap = []
    for n in range(max32 + 1):
        c = mp.gamma(n + mp.mpf(1) / 2) / 2
        kap.append(float(np.float32(float(c ** (1 / (n + mp.mpf(1) / 2))))))
    lines.append("constexpr float kKappa32[] = {" + ", ".join(float.hex(v) + "f" for v in kap) + "};")
    lines.append("// exp(a) = 2^m 2^(j/256) exp(r), a = k ln2/256 + r, k = 256 m + j")
    lines.append(f"constexpr double kInvLn2x256 = {float.hex(inv)};")
    lines.append(f"constexpr double kLn2d256_1 = {float.hex(L1)};  // 36 significant bits")
    lines.append(f"constexpr double kLn2d256_2 = {float.hex(L2)};")
    lines.append(f"constexpr double kLn2d256_3 = {float.hex(L3)};")
    for k, (hi, lo) in fac.items():
        lines.append(f"constexpr double kInvFact{k}_hi = {float.hex(hi)};")
        lines.append(f"constexpr double kInvFact{k}_lo = {float.hex(lo)};")
    lines.append("// 2^(j/256) as (hi, lo) pairs")
    lines.append("alignas(16) constexpr double kExp2Tab[512] = {")
    for i in range(0, 512, 4):
        lines.append("  " + ", ".join(float.hex(v) for v in tab[i:i + 4]) + ",")
    lines.append("};")
    lines.append("}  // namespace")
    lines.append("}  // namespace boys_tab")
    text = "\n".join(lines) + "\n"
    tmp = out + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(text)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    main(*sys.argv[1:])
