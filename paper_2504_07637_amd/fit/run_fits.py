"""Fit every (precision class, n) approximant and write the coefficient dataset.

Usage:  python -m paper_2504_07637_amd.fit.run_fits [--nmax 36] [--jobs 7] [--out PATH]

The orders N follow Table 1 of the paper (blank cells read as repeats of the cell
above): binary64 N = 10 (n = 0-1), 11 (2-6), 12 (7-10), 13 (11-17), 14 (18-36);
binary32 N = 4 (0-1), 5 (2-9), 6 (10-36).  The cut-off z_nb uses b = 53 for the
binary64 class and b = 24 for the binary32 class.  The class fp32x (binary32 results
rounded from binary64 arithmetic) uses b = 28 and, per n, the smallest N whose fit
reaches 28 bits; its coefficients are binary64 values.

Dataset format (text, one token list per line, '#' starts a comment):

    format boys-coeffs 1
    c0 <hex>                         c_0 = sqrt(pi)/2 in binary64
    record <fp64|fp32|fp32x> <n> <N>
    c  <hex> <dec>                   c_n (binary64)
    z  <hex> <dec>                   z_nb (binary64)
    q0 <hex> <dec>                   Q_n(0)        } working precision of the class
    q1 <hex> <dec>                   Q'_n(0)       } (binary32 values for fp32)
    q2 <hex> <dec>                   alpha_n - q1  }
    ug <k> <hex>*k                   gathered monic factor of u, ascending, leading 1 implied
    uq <k> (<hex y> <hex a>)*k       factors (x - y)^2 + a of u, ascending y
    ul <k> <hex>*k                   factors (x - y) of u
    vg / vq / vl                     the same for v
    ugx / uqx / ulx / vgx / vqx / vlx   the same values with 40 significant decimal digits
    A <N+2> <dec>*                   expanded numerator of Eq. qr
    B <N+1> <dec>*                   expanded denominator of Eq. qr (B_0 = 1)
    eps <exact coefficients> <rounded coefficients>   -log2 max|F~/F-1| on [0, z_nb)
    end
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mproc
import os
import sys
import time

import mpmath as mp

from . import boys_fit as bf

DATA_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "data")
DEFAULT_OUT = os.path.join(DATA_DIR, "boys_coeffs.txt")
REPORT = os.path.join(DATA_DIR, "fit_report.json")


def table1_N(cls: str, n: int) -> int:
    if cls == "fp64":
        return 10 if n <= 1 else 11 if n <= 6 else 12 if n <= 10 else 13 if n <= 17 else 14
    return 4 if n <= 1 else 5 if n <= 9 else 6


# the binary32-output class evaluated in binary64 (section "Computations": full 24-bit
# binary32 values by rounding binary64 results of about 28-bit approximants): cut-off
# b = 28 and the smallest N whose fit reaches EPS_FP32X bits
B_FP32X = 28
EPS_FP32X = 28.0


def class_b(cls: str) -> int:
    return {"fp64": 53, "fp32": 24, "fp32x": B_FP32X}[cls]


def _record_from(cls, n, N, b, A, B, z, t0, extra=None):
    cn = bf.consts(n)
    f = bf.factor(cn, A, B)
    # no pole on [0, inf): every linear factor of v must have a negative root
    if f.vl:
        raise RuntimeError(f"v has real non-negative roots {f.vl}")
    if B[-1] <= 0:
        raise RuntimeError("B_N <= 0 (rejected, as in the paper)")
    for y, a in f.uq + f.vq:
        if a <= 0:
            raise RuntimeError("non-positive a in a quadratic factor")
    fr = bf.round_factored(f, cls == "fp32")  # fp32x coefficients are binary64 values
    eps_x = bf.dense_error(n, f, z, npts=1500)
    eps_r = bf.dense_error(n, fr, z, npts=1500)
    to_hex = bf.to_f32_hex if cls == "fp32" else (lambda v: bf.hexf(float(v)))  # fp32x: binary64
    rec = {
        "cls": cls, "n": n, "N": N, "b": b,
        "c": (bf.hexf(float(cn.c)), bf.decs(cn.c)),
        "z": (bf.hexf(float(z)), bf.decs(z)),
        "q0": (to_hex(f.q0), bf.decs(f.q0)),
        "q1": (to_hex(f.q1), bf.decs(f.q1)),
        "q2": (to_hex(f.q2), bf.decs(f.q2)),
        "ug": [to_hex(c) for c in f.ug], "ugx": [bf.decs(c) for c in f.ug],
        "uq": [(to_hex(y), to_hex(a)) for y, a in f.uq],
        "uqx": [(bf.decs(y), bf.decs(a)) for y, a in f.uq],
        "ul": [to_hex(y) for y in f.ul], "ulx": [bf.decs(y) for y in f.ul],
        "vg": [to_hex(c) for c in f.vg], "vgx": [bf.decs(c) for c in f.vg],
        "vq": [(to_hex(y), to_hex(a)) for y, a in f.vq],
        "vqx": [(bf.decs(y), bf.decs(a)) for y, a in f.vq],
        "vl": [to_hex(y) for y in f.vl], "vlx": [bf.decs(y) for y in f.vl],
        "A": [bf.decs(a) for a in A], "B": [bf.decs(b_) for b_ in B],
        "eps_exact": eps_x, "eps_rounded": eps_r, "seconds": time.time() - t0,
    }
    if extra:
        rec.update(extra)
    return rec


def _fit_one(job):
    """Lawson-SK fit from scratch, then the Remez polish."""
    cls, n = job
    if cls == "fp32x":
        return _fit_adaptive(n)
    mp.mp.prec = bf.PREC
    b = class_b(cls)
    N = table1_N(cls, n)
    t0 = time.time()
    attempts = [(500 if cls == "fp64" else 300, 1.0), (800, 1.0), (800, 1.1)]
    last_err = None
    for M, xs in attempts:
        try:
            r = bf.fit(n, N, b, M=M, iters=600 if cls == "fp64" else 300, X_scale=xs)
            A, B = r.A, r.B
            try:
                A2, B2, _ = bf.remez_polish(n, N, b, A, B)
                A, B = A2, B2
            except Exception:
                pass
            rec = _record_from(cls, n, N, b, A, B, r.z, t0,
                               {"eps_sampled": r.err_sampled, "iterations": r.iterations})
            break
        except Exception as exc:  # try the next sampling
            last_err = exc
            rec = None
    if rec is None:
        return {"cls": cls, "n": n, "N": N, "error": repr(last_err)}
    print(f"[fit] {cls} n={n} N={N} eps={rec['eps_exact']:.2f} (rounded {rec['eps_rounded']:.2f}) "
          f"{time.time() - t0:.0f}s", flush=True)
    return rec


def _fit_adaptive(n: int):
    """fp32x: the smallest N (from 4 up) whose polished fit reaches EPS_FP32X bits."""
    mp.mp.prec = bf.PREC
    cls, b = "fp32x", B_FP32X
    t0 = time.time()
    last = None
    for N in range(4, 11):
        try:
            r = bf.fit(n, N, b, M=300, iters=300)
            A, B = r.A, r.B
            try:
                A, B, _ = bf.remez_polish(n, N, b, A, B, M=1500, iters=40)
            except Exception:
                pass
            rec = _record_from(cls, n, N, b, A, B, r.z, t0)
        except Exception as exc:
            last = {"cls": cls, "n": n, "N": N, "error": repr(exc)}
            continue
        last = rec
        if rec["eps_exact"] >= EPS_FP32X:
            break
    if "error" not in last:
        print(f"[fit] {cls} n={n} N={last['N']} eps={last['eps_exact']:.2f} "
              f"(rounded {last['eps_rounded']:.2f}) {time.time() - t0:.0f}s", flush=True)
    return last


def _polish_one(job):
    """Remez polish of an existing dataset entry; keeps the better of the two."""
    cls, n, N, A, B, eps_old = job
    mp.mp.prec = bf.PREC
    b = class_b(cls)
    t0 = time.time()
    z = bf.cutoff(n, b)
    A = [mp.mpf(a) for a in A]
    B = [mp.mpf(v) for v in B]
    best = None
    try:
        A2, B2, _ = bf.remez_polish(n, N, b, A, B, M=2000, iters=60)
        best = _record_from(cls, n, N, b, A2, B2, z, t0)
    except Exception as exc:
        print(f"[polish] {cls} n={n} failed: {exc!r}", flush=True)
    if best is None or best["eps_exact"] < eps_old:
        best = _record_from(cls, n, N, b, A, B, z, t0)
    print(f"[polish] {cls} n={n} N={N} eps {eps_old:.2f} -> {best['eps_exact']:.2f} "
          f"(rounded {best['eps_rounded']:.2f}) {time.time() - t0:.0f}s", flush=True)
    return best


def read_expanded(path):
    """(cls, n) -> (N, A decimal strings, B decimal strings, eps) from a dataset file."""
    out = {}
    cur = None
    with open(path) as fh:
        for raw in fh:
            tok = raw.split("#", 1)[0].split()
            if not tok:
                continue
            if tok[0] == "record":
                cur = {"cls": tok[1], "n": int(tok[2]), "N": int(tok[3])}
            elif tok[0] in ("A", "B") and cur is not None:
                cur[tok[0]] = tok[2:]
            elif tok[0] == "eps" and cur is not None:
                cur["eps"] = float(tok[1])
            elif tok[0] == "end":
                out[(cur["cls"], cur["n"])] = cur
                cur = None
    return out


def _line(tag, vals):
    return tag + " " + str(len(vals)) + ("" if not vals else " " + " ".join(vals))


def _pairs(tag, pairs):
    return f"{tag} {len(pairs)}" + "".join(f" {a} {b}" for a, b in pairs)


def read_blocks(path):
    """[(cls, n, text)] of the record blocks of an existing dataset file."""
    out, cur, lines = [], None, []
    with open(path) as fh:
        for raw in fh:
            tok = raw.split()
            if tok and tok[0] == "record":
                cur, lines = (tok[1], int(tok[2])), [raw.rstrip("\n")]
            elif cur is not None:
                lines.append(raw.rstrip("\n"))
                if tok and tok[0] == "end":
                    out.append((cur[0], cur[1], "\n".join(lines)))
                    cur = None
    return out


def write_dataset(records, path, kept_blocks=()):
    mp.mp.prec = bf.PREC
    c0 = mp.sqrt(mp.pi) / 2
    out = ["# Boys-function approximant coefficients (root-factored form of Eqs. pqz, pz, qz)",
           "# written by paper_2504_07637_amd.fit.run_fits; see that module for the format",
           "format boys-coeffs 1",
           f"c0 {bf.hexf(float(c0))}"]
    for r in sorted(records, key=lambda r: (r["cls"], r["n"])):
        out.append(f"record {r['cls']} {r['n']} {r['N']}")
        for k in ("c", "z", "q0", "q1", "q2"):
            out.append(f"{k} {r[k][0]} {r[k][1]}")
        for side in ("u", "v"):
            out.append(_line(side + "g", r[side + "g"]))
            out.append(_pairs(side + "q", r[side + "q"]))
            out.append(_line(side + "l", r[side + "l"]))
        for side in ("u", "v"):
            out.append(_line(side + "gx", r[side + "gx"]))
            out.append(_pairs(side + "qx", r[side + "qx"]))
            out.append(_line(side + "lx", r[side + "lx"]))
        out.append(_line("A", r["A"]))
        out.append(_line("B", r["B"]))
        out.append(f"eps {r['eps_exact']:.3f} {r['eps_rounded']:.3f}")
        out.append("end")
    out.extend(kept_blocks)
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nmax", type=int, default=36)
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--classes", default="fp64,fp32")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--report", default=REPORT)
    ap.add_argument("--polish", action="store_true",
                    help="polish the existing dataset at --out instead of fitting afresh")
    ap.add_argument("--merge", action="store_true",
                    help="keep the records of other classes already in --out")
    args = ap.parse_args(argv)
    classes = args.classes.split(",")
    if args.polish:
        old = read_expanded(args.out)
        jobs = [(c, n, old[(c, n)]["N"], old[(c, n)]["A"], old[(c, n)]["B"], old[(c, n)]["eps"])
                for c in classes for n in range(args.nmax + 1)]
        jobs.sort(key=lambda j: -j[2])
        with mproc.Pool(args.jobs) as pool:
            recs = pool.map(_polish_one, jobs, chunksize=1)
    else:
        # long binary64 fits first so the pool drains evenly
        jobs = [(c, n) for c in classes for n in range(args.nmax + 1)]
        jobs.sort(key=lambda j: (j[0] != "fp64", -bf_cost(j)))
        with mproc.Pool(args.jobs) as pool:
            recs = pool.map(_fit_one, jobs, chunksize=1)
    bad = [r for r in recs if "error" in r]
    good = [r for r in recs if "error" not in r]
    if args.merge and os.path.exists(args.out):
        kept = [blk for blk in read_blocks(args.out) if blk[0] not in classes]
        write_dataset(good, args.out, kept_blocks=[b for _, _, b in kept])
        if os.path.exists(args.report):
            old_rep = [r for r in json.load(open(args.report)) if r["cls"] not in classes]
            recs = old_rep + recs
    else:
        write_dataset(good, args.out)
    with open(args.report, "w") as fh:
        json.dump([{k: r[k] for k in r if k in ("cls", "n", "N", "eps_exact", "eps_rounded",
                                                "eps_sampled", "iterations", "seconds", "error")}
                   for r in recs], fh, indent=1)
    for r in bad:
        print("[fit] FAILED", r, file=sys.stderr)
    return 1 if bad else 0


def bf_cost(job):
    cls, n = job
    return table1_N(cls, n)


if __name__ == "__main__":
    sys.exit(main())
