"""Offline fitter for the rational approximants of the Boys-function closed form.

Laikov (arXiv 2504.07637, section "Methodology", Eq. fq) writes the Boys function as

    F_n(x) = c_n / (x + Q_n(x)^(n+1/2) exp(-x))^(n+1/2),   c_n = Gamma(n+1/2)/2,

which turns F_n into a smooth, almost linear function Q_n.  This module fits, for one
order n and one target precision (b = 53 or 24 bits), the rational function of Eq. qr

    Q~_n(x) = (sum_{k=0}^{N+1} A_k x^k) / (1 + sum_{k=1}^{N} B_k x^k)

that minimises the largest relative error of F~_n (Eq. e) on [0, z_nb], with the four
constraints of Eqs. q0, q1, qa/aq and qb/bq built into the parametrisation:

    A_0 = Q_n(0),  A_1 = Q'_n(0) + Q_n(0) B_1,  A_{N+1} = alpha_n B_N,
    A_N = alpha_n B_{N-1} + beta_n B_N.

The paper's own optimiser and its 547 solutions are not available, so the coefficients
are re-fitted here.  The method is Lawson's iteratively reweighted least squares on the
Sanathanan-Koerner linearisation, in 256-bit arithmetic (mpmath), on Chebyshev points.
The fitted rational is then rewritten in the root-factored form of Eqs. pqz, pz, qz,

    Q~_n = q0 + q1 x + q2 x^2 u(x)/v(x),

with monic u (degree N-1) and v (degree N).  Factors whose roots have negative real
parts are gathered into one polynomial with positive coefficients (the remark after
Eq. qz); the others stay as quadratic factors (x-y)^2 + a or linear factors (x-y).

The exact Q_n used as the fitting target comes from the regularised incomplete gamma
function: F_n(x) = c_n P(n+1/2, x) / x^(n+1/2), so x + W = x P^(-1/s) and
Q = (W e^x)^(1/s) with s = n + 1/2.

This is an offline tool.  Nothing on the evaluation path imports it; it writes the
coefficient dataset that the evaluators read.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import mpmath as mp

PREC = 256


def _mpf(v):
    return mp.mpf(v)


@dataclass
class Consts:
    n: int
    s: mp.mpf
    c: mp.mpf          # c_n = (2n)! sqrt(pi) / (n! 2^(2n+1)) = Gamma(n+1/2)/2
    q0: mp.mpf         # Q_n(0), Eq. q0
    q1: mp.mpf         # Q'_n(0), Eq. q1
    alpha: mp.mpf      # Eq. aq
    beta: mp.mpf       # Eq. bq


def consts(n: int) -> Consts:
    """The closed-form constants of section "Methodology" (Eqs. c_n, q0, q1, aq, bq)."""
    s = _mpf(2 * n + 1) / 2
    c = mp.gamma(s) / 2
    k = (2 * n + 1) * c
    q0 = k ** (_mpf(4) / (2 * n + 1) ** 2)
    q1 = 2 * q0 / (2 * n + 1) * (_mpf(2 * n + 5) / (2 * n + 3) - k ** (_mpf(-2) / (2 * n + 1)))
    c_next = s * c  # c_{n+1} = Gamma(n+3/2)/2
    alpha = (2 * c_next) ** (_mpf(-2) / (2 * n + 1))
    beta = _mpf(2 * n - 1) / (2 * n + 1) * alpha
    return Consts(n, s, c, q0, q1, alpha, beta)


def upper_q(s, x):
    """Regularised upper incomplete gamma Gamma(s, x)/Gamma(s)."""
    return mp.gammainc(s, x, mp.inf, regularized=True)


def lower_p(s, x):
    """Regularised lower incomplete gamma gamma(s, x)/Gamma(s)."""
    return mp.gammainc(s, 0, x, regularized=True)


def cutoff(n: int, b: int):
    """z_nb: the x where x^(n+1/2) F_n(x) / c_n = 1 - 2^-b (section "Methodology").

    The printed right-hand side reads 1 - 2^b; the sign of the exponent is taken as
    negative, the only reading for which a solution exists.  Since
    x^s F_n / c_n = P(s, x), this is Q(s, z) = 2^-b for the regularised upper gamma.
    """
    s = _mpf(2 * n + 1) / 2
    target = -b * mp.log(2)

    def f(z):
        return mp.log(upper_q(s, z)) - target

    lo = s
    hi = s + 10
    while f(hi) > 0:
        lo = hi
        hi = hi * 1.5
    # bisection to a bracket of 1e-6 relative, then secant polish
    for _ in range(60):
        mid = (lo + hi) / 2
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-8 * hi:
            break
    return mp.findroot(f, (lo, hi), solver="anderson")


def exact_WQ(cn: Consts, x):
    """W_n(x) and Q_n(x) from the incomplete gamma function (x > 0)."""
    s = cn.s
    if x < s:
        P = lower_p(s, x)
        W = x * (P ** (-1 / s) - 1)
    else:
        q = upper_q(s, x)
        W = x * mp.expm1(-mp.log1p(-q) / s)
    Q = mp.exp((mp.log(W) + x) / s)
    return W, Q


def exact_F(n: int, x):
    """F_n(x) = gamma(n+1/2, x) / (2 x^(n+1/2)) (for x > 0), 1/(2n+1) at 0."""
    if x == 0:
        return _mpf(1) / (2 * n + 1)
    s = _mpf(2 * n + 1) / 2
    return mp.gammainc(s, 0, x) / (2 * x ** s)


# ----------------------------------------------------------------------------------
# parametrisation


class Param:
    """Affine map from the 2N-2 free parameters to the coefficients of P and D.

    Works in the scaled variable t = x / X so that the basis stays well scaled:
    P(t) = sum Ph_k t^k, D(t) = 1 + sum Dh_k t^k with Ph_k = A_k X^k, Dh_k = B_k X^k.
    Free parameters: Ph_2 .. Ph_{N-1}, then Dh_1 .. Dh_N.
    """

    def __init__(self, cn: Consts, N: int, X):
        self.N = N
        self.X = X
        K = 2 * N - 2
        self.K = K
        nP, nD = N + 2, N + 1
        self.Pa = [_mpf(0)] * nP
        self.Db = [_mpf(0)] * nD
        self.PM = [[_mpf(0)] * K for _ in range(nP)]
        self.DL = [[_mpf(0)] * K for _ in range(nD)]
        iA = {k: k - 2 for k in range(2, N)}          # parameter index of Ph_k
        iB = {k: (N - 2) + (k - 1) for k in range(1, N + 1)}  # parameter index of Dh_k
        aX = cn.alpha * X
        # D
        self.Db[0] = _mpf(1)
        for k in range(1, N + 1):
            self.DL[k][iB[k]] = _mpf(1)
        # P_0 = q0
        self.Pa[0] = cn.q0
        # P_1 = q1 X + q0 Dh_1
        self.Pa[1] = cn.q1 * X
        self.PM[1][iB[1]] += cn.q0
        # P_k free for 2..N-1
        for k in range(2, N):
            self.PM[k][iA[k]] = _mpf(1)
        # P_N = alpha X Dh_{N-1} + beta Dh_N   (Dh_0 = 1 when N-1 == 0, not reached: N >= 2)
        self.PM[N][iB[N - 1]] += aX
        self.PM[N][iB[N]] += cn.beta
        # P_{N+1} = alpha X Dh_N
        self.PM[N + 1][iB[N]] += aX

    def coeffs(self, p):
        P = [self.Pa[k] + mp.fdot(self.PM[k], p) for k in range(self.N + 2)]
        D = [self.Db[k] + mp.fdot(self.DL[k], p) for k in range(self.N + 1)]
        return P, D

    def unscaled(self, p):
        """A_k and B_k of Eq. qr."""
        P, D = self.coeffs(p)
        A = [P[k] / self.X ** k for k in range(len(P))]
        B = [D[k] / self.X ** k for k in range(len(D))]
        return A, B


def _horner(c, t):
    r = _mpf(0)
    for a in reversed(c):
        r = r * t + a
    return r


def cheb_points(M: int, X):
    return [X * (1 - mp.cos(mp.pi * j / (M - 1))) / 2 for j in range(M)]


@dataclass
class FitResult:
    n: int
    N: int
    b: int
    z: mp.mpf
    X: mp.mpf
    A: list
    B: list
    err_sampled: float          # -log2 max |F~/F - 1| on the fitting points
    iterations: int
    history: list = field(default_factory=list)


def rel_err_F(cn: Consts, x, Qt, W):
    """F~/F - 1 where F~ uses Q~ = Qt and F uses the exact W (Eq. fq)."""
    if Qt <= 0:
        return mp.inf
    Wt = mp.exp(cn.s * mp.log(Qt) - x)
    # (x+W)/(x+Wt) raised to s, minus 1
    return mp.expm1(cn.s * mp.log1p((W - Wt) / (x + Wt)))


def fit(n: int, N: int, b: int, M: int = 500, iters: int = 400, verbose: bool = False,
        X_scale: float = 1.0, init_B=None) -> FitResult:
    """Lawson-SK fit; init_B (expanded denominator B_0..B_N of another fit, e.g. of a
    neighbouring n) seeds the first linearisation instead of D = 1."""
    mp.mp.prec = PREC
    cn = consts(n)
    z = cutoff(n, b)
    X = z * _mpf(X_scale)
    xs = cheb_points(M, X)
    xs = xs[1:]  # x = 0 is exact by construction (Q~(0) = Q(0))
    ts = [x / X for x in xs]
    WQ = [exact_WQ(cn, x) for x in xs]
    Ws = [w for w, _ in WQ]
    Qs = [q for _, q in WQ]
    s2 = cn.s * cn.s
    wts = [s2 * W / ((x + W) * Q) for x, W, Q in zip(xs, Ws, Qs)]
    par = Param(cn, N, X)
    K = par.K
    Mn = len(xs)
    # powers of t
    tp = []
    for t in ts:
        row = [_mpf(1)]
        for _ in range(N + 1):
            row.append(row[-1] * t)
        tp.append(row)
    # row pieces independent of the iteration: phi.PM, phi.Pa, phi_D.DL, phi_D.Db
    PMt = [list(col) for col in zip(*par.PM)]  # K x nP
    DLt = [list(col) for col in zip(*par.DL)]
    base_P = []
    base_D = []
    for i in range(Mn):
        row = tp[i]
        bp = [mp.fdot(PMt[j], row[: N + 2]) for j in range(K)]
        bd = [mp.fdot(DLt[j], row[: N + 1]) for j in range(K)]
        base_P.append((bp, mp.fdot(par.Pa, row[: N + 2])))
        base_D.append((bd, mp.fdot(par.Db, row[: N + 1])))
    if init_B is not None:
        Dprev = [_horner([mp.mpf(bk) for bk in init_B], x) for x in xs]
        if any(d <= 0 for d in Dprev):
            Dprev = [_mpf(1)] * Mn
    else:
        Dprev = [_mpf(1)] * Mn
    lam = [_mpf(1) / Mn] * Mn
    best = None
    hist = []
    p = None
    for it in range(iters):
        J = []
        r0 = []
        for i in range(Mn):
            sc = wts[i] / Dprev[i]
            bp, ap = base_P[i]
            bd, ad = base_D[i]
            Q = Qs[i]
            J.append([sc * (bp[j] - Q * bd[j]) for j in range(K)])
            r0.append(sc * (ap - Q * ad))
        # normal equations of min sum lam (J p + r0)^2
        Jl = [[lam[i] * J[i][j] for i in range(Mn)] for j in range(K)]  # K x M
        A = mp.matrix(K, K)
        rhs = mp.matrix(K, 1)
        Jc = [[J[i][j] for i in range(Mn)] for j in range(K)]
        for a in range(K):
            for c in range(a, K):
                v = mp.fdot(Jl[a], Jc[c])
                A[a, c] = v
                A[c, a] = v
            rhs[a] = -mp.fdot(Jl[a], r0)
        try:
            sol = mp.lu_solve(A, rhs)
        except ZeroDivisionError:
            break
        p = [sol[j] for j in range(K)]
        P, D = par.coeffs(p)
        errs = []
        ok = True
        newD = []
        for i in range(Mn):
            Pv = _horner(P, ts[i])
            Dv = _horner(D, ts[i])
            newD.append(Dv)
            if Dv <= 0:
                ok = False
                errs.append(mp.mpf(1))
                continue
            Qt = Pv / Dv
            errs.append(rel_err_F(cn, xs[i], Qt, Ws[i]))
        emax = max(abs(e) for e in errs)
        if ok and D[-1] > 0 and (best is None or emax < best[0]):
            best = (emax, p)
        hist.append(float(-mp.log(emax, 2)) if emax > 0 else 99.0)
        if verbose and (it % 20 == 0 or it == iters - 1):
            print(f"n={n} N={N} b={b} it={it} eps={hist[-1]:.3f} best={float(-mp.log(best[0], 2)) if best else None}",
                  flush=True)
        Dprev = [d if d > 0 else _mpf(1) for d in newD]
        # Lawson update
        tot = _mpf(0)
        for i in range(Mn):
            lam[i] = lam[i] * abs(errs[i])
            tot += lam[i]
        if tot == 0:
            break
        lam = [l / tot for l in lam]
        # floor the weights so no point is dropped for good
        fl = _mpf(1e-30) / Mn
        lam = [l if l > fl else fl for l in lam]
        if len(hist) > 60 and abs(hist[-1] - hist[-41]) < 2e-4 and best is not None:
            break
    if best is None:
        raise RuntimeError(f"no admissible fit for n={n} N={N} b={b}")
    A_, B_ = par.unscaled(best[1])
    return FitResult(n, N, b, z, X, A_, B_, float(-mp.log(best[0], 2)), len(hist), hist)


def _alternation(err, nref):
    """Indices of nref alternating extrema of err (one per sign run, extras pruned)."""
    runs = []
    i = 0
    M = len(err)
    while i < M:
        if err[i] == 0:
            i += 1
            continue
        sgn = err[i] > 0
        best = i
        j = i
        while j < M and (err[j] > 0) == sgn and err[j] != 0:
            if abs(err[j]) > abs(err[best]):
                best = j
            j += 1
        runs.append(best)
        i = j
    if len(runs) < nref:
        return None
    while len(runs) > nref:
        k = min(range(len(runs)), key=lambda t: abs(err[runs[t]]))
        if k == 0 or k == len(runs) - 1:
            runs.pop(k)
        elif len(runs) - nref == 1:
            # drop the smaller end instead, which keeps the alternation
            runs.pop(0 if abs(err[runs[0]]) < abs(err[runs[-1]]) else len(runs) - 1)
        else:
            nb = k - 1 if abs(err[runs[k - 1]]) < abs(err[runs[k + 1]]) else k + 1
            for t in sorted((k, nb), reverse=True):
                runs.pop(t)
    return runs


def remez_polish(n: int, N: int, b: int, A0, B0, M: int = 3000, iters: int = 25,
                 verbose: bool = False):
    """Polish a fit by Newton steps on the equioscillation conditions.

    On a fixed dense grid of [0, z], take the 2N-1 alternating extrema of
    err(x) = F~/F - 1 and solve err(x_i; p + dp) = (-1)^i E for dp and E (2N-1 unknowns:
    the 2N-2 free parameters and the levelled error), with the derivative of err taken
    through Q~.  Keeps the iterate with the smallest grid maximum.
    """
    mp.mp.prec = PREC
    cn = consts(n)
    z = cutoff(n, b)
    X = z
    par = Param(cn, N, X)
    K = par.K
    # free parameters from the expanded coefficients
    p = [_mpf(0)] * K
    for k in range(2, N):
        p[k - 2] = A0[k] * X ** k
    for k in range(1, N + 1):
        p[(N - 2) + (k - 1)] = B0[k] * X ** k
    xs = [X * (1 - mp.cos(mp.pi * (j + mp.mpf(1) / 2) / M)) / 2 for j in range(M)]
    ts = [x / X for x in xs]
    WQ = [exact_WQ(cn, x) for x in xs]
    Ws = [w for w, _ in WQ]
    PMt = [list(col) for col in zip(*par.PM)]
    DLt = [list(col) for col in zip(*par.DL)]
    s = cn.s

    def errors(p):
        P, D = par.coeffs(p)
        out = []
        der = []
        for i, x in enumerate(xs):
            Dv = _horner(D, ts[i])
            if Dv <= 0:
                return None, None
            Qt = _horner(P, ts[i]) / Dv
            if Qt <= 0:
                return None, None
            Wt = mp.exp(s * mp.log(Qt) - x)
            e = mp.expm1(s * mp.log1p((Ws[i] - Wt) / (x + Wt)))
            out.append(e)
            der.append((-s * s * (1 + e) * Wt / ((x + Wt) * Qt), Dv, Qt))
        return out, der

    err, der = errors(p)
    if err is None:
        raise RuntimeError("starting point has a pole")
    best = (max(abs(e) for e in err), list(p))
    for it in range(iters):
        idx = _alternation(err, K + 1)
        if idx is None:
            # one alternation short (the last extremum is pushed against z, where the
            # weight vanishes): level the K extrema that exist, minimum-norm step
            idx = _alternation(err, K)
            if idx is None:
                break
        nr = len(idx)
        sig = 1 if err[idx[0]] > 0 else -1
        Mx = mp.matrix(nr, K + 1)
        rhs = mp.matrix(nr, 1)
        for r_, i in enumerate(idx):
            dq, Dv, Qt = der[i]
            row = [ts[i] ** k for k in range(N + 2)]
            for j in range(K):
                dP = mp.fdot(PMt[j], row[: N + 2])
                dD = mp.fdot(DLt[j], row[: N + 1])
                Mx[r_, j] = dq * (dP - Qt * dD) / Dv
            Mx[r_, K] = -sig * (-1) ** r_
            rhs[r_] = -err[i]
        if nr == K + 1:
            try:
                sol = mp.lu_solve(Mx, rhs)
            except ZeroDivisionError:
                break
            step = [sol[j] for j in range(K)]
            # damped Newton: the step length with the smallest grid maximum
            cand = None
            lam = _mpf(1)
            for _ in range(5):
                trial = [p[j] + lam * step[j] for j in range(K)]
                e2, d2 = errors(trial)
                if e2 is not None:
                    m2 = max(abs(e) for e in e2)
                    if cand is None or m2 < cand[0]:
                        cand = (m2, trial, e2, d2)
                lam /= 2
            if cand is None:
                break
            _, trial, e2, d2 = cand
        else:
            # K extrema for K parameters: level them at a target E below the current
            # level (square system in dp) and keep the target that lowers the grid max
            level = sum(abs(err[i]) for i in idx) / nr
            Msq = mp.matrix(nr, K)
            for r_ in range(nr):
                for j in range(K):
                    Msq[r_, j] = Mx[r_, j]
            cand = None
            for f in (0.97, 0.93, 0.85, 0.99, 0.75):
                rh = mp.matrix(nr, 1)
                for r_ in range(nr):
                    rh[r_] = rhs[r_] - Mx[r_, K] * level * f
                try:
                    sol = mp.lu_solve(Msq, rh)
                except ZeroDivisionError:
                    continue
                trial = [p[j] + sol[j] for j in range(K)]
                e2, d2 = errors(trial)
                if e2 is None:
                    continue
                m2 = max(abs(e) for e in e2)
                if cand is None or m2 < cand[0]:
                    cand = (m2, trial, e2, d2, f)
            if cand is None:
                break
            _, trial, e2, d2, f = cand
            sol = [_mpf(0)] * K + [level * f]
        p, err, der = trial, e2, d2
        emax = max(abs(e) for e in err)
        if verbose:
            print(f"remez n={n} N={N} b={b} it={it} eps={float(-mp.log(emax, 2)):.4f} "
                  f"E={float(-mp.log(abs(sol[K]), 2)):.4f}", flush=True)
        if emax < best[0]:
            best = (emax, list(p))
        elif it > 3 and emax > best[0] * 1.5:
            break
        if abs(emax / abs(sol[K]) - 1) < 1e-4:
            break  # levelled
    A, B = par.unscaled(best[1])
    return A, B, float(-mp.log(best[0], 2))


# ----------------------------------------------------------------------------------
# root-factored form


@dataclass
class Factored:
    q0: mp.mpf
    q1: mp.mpf
    q2: mp.mpf
    ug: list   # gathered monic factor of u, ascending coefficients without the leading 1
    uq: list   # [(y, a)] quadratic factors (x-y)^2 + a with y >= 0
    ul: list   # [y] linear factors (x-y) with y >= 0
    vg: list
    vq: list
    vl: list


def _poly_mul(a, b):
    r = [mp.mpc(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            r[i + j] += x * y
    return r


def _split_roots(coeffs_asc):
    """Roots of a real polynomial, grouped into the factor classes of Eqs. pz/qz."""
    deg = len(coeffs_asc) - 1
    if deg == 0:
        return [], [], []
    lead = coeffs_asc[-1]
    monic_desc = [c / lead for c in reversed(coeffs_asc)]
    roots = mp.polyroots(monic_desc, maxsteps=2000, extraprec=2 * PREC)
    reals, cplx = [], []
    for r in roots:
        r = mp.mpc(r)
        if abs(r.imag) <= mp.mpf(2) ** (-PREC // 2) * (1 + abs(r)):
            reals.append(mp.re(r))
        elif r.imag > 0:
            cplx.append(r)
    if len(reals) + 2 * len(cplx) != deg:
        raise RuntimeError("root classification failed")
    neg_roots = []   # gathered (Re < 0)
    quad = []
    lin = []
    for r in reals:
        if r < 0:
            neg_roots.append(mp.mpc(r))
        else:
            lin.append(r)
    for r in cplx:
        if r.real < 0:
            neg_roots.append(r)
            neg_roots.append(mp.conj(r))
        else:
            quad.append((mp.re(r), mp.im(r) ** 2))
    g = [mp.mpc(1)]
    for r in neg_roots:
        g = _poly_mul(g, [-r, mp.mpc(1)])
    g = [mp.re(c) for c in g]
    # ascending, monic: drop the leading 1
    gathered = g[:-1]
    quad.sort(key=lambda t: t[0])
    lin.sort()
    return gathered, quad, lin


def factor(cn: Consts, A: list, B: list) -> Factored:
    """Rewrite P/D of Eq. qr as q0 + q1 x + q2 x^2 u/v (Eqs. pqz, pz, qz)."""
    N = len(B) - 1
    # R = P - (q0 + q1 x) D ; R_0 = R_1 = 0 by the built-in constraints
    R = list(A)
    for k in range(N + 1):
        R[k] -= cn.q0 * B[k]
        R[k + 1] -= cn.q1 * B[k]
    U = R[2:]                # degree N-1
    lead_u = U[-1]
    q2 = lead_u / B[N]
    ug, uq, ul = _split_roots(U)
    vg, vq, vl = _split_roots(B)
    return Factored(cn.q0, cn.q1, q2, ug, uq, ul, vg, vq, vl)


def eval_factored(f: Factored, x):
    """Q~ by Eq. pqz in the working precision of mpmath (for checks)."""
    u = _mpf(1)
    for c in reversed(f.ug):
        pass
    # Horner for the monic gathered factor
    u = _mpf(1)
    for c in reversed(f.ug):
        u = u * x + c
    for y, a in f.uq:
        u = u * ((x - y) ** 2 + a)
    for y in f.ul:
        u = u * (x - y)
    v = _mpf(1)
    for c in reversed(f.vg):
        v = v * x + c
    for y, a in f.vq:
        v = v * ((x - y) ** 2 + a)
    for y in f.vl:
        v = v * (x - y)
    return f.q0 + f.q1 * x + f.q2 * (u / v) * x * x


def dense_error(n: int, f: Factored, z, npts: int = 2000, refine: int = 6):
    """-log2 of max |F~/F - 1| over [0, z) on an even grid, then refined near the worst points."""
    cn = consts(n)
    xs = [z * j / npts for j in range(1, npts)]
    vals = []
    for x in xs:
        W, Q = exact_WQ(cn, x)
        vals.append(abs(rel_err_F(cn, x, eval_factored(f, x), W)))
    order = sorted(range(len(xs)), key=lambda i: -vals[i])[:refine]
    emax = max(vals)
    h = z / npts
    for i in order:
        # golden-section search for a local max in [x-h, x+h]
        a, bb = xs[i] - h, xs[i] + h
        if a <= 0:
            a = h / 1000
        g = (mp.sqrt(5) - 1) / 2

        def e(x):
            W, Q = exact_WQ(cn, x)
            return abs(rel_err_F(cn, x, eval_factored(f, x), W))
        c1 = bb - g * (bb - a)
        c2 = a + g * (bb - a)
        f1, f2 = e(c1), e(c2)
        for _ in range(25):
            if f1 > f2:
                bb, c2, f2 = c2, c1, f1
                c1 = bb - g * (bb - a)
                f1 = e(c1)
            else:
                a, c1, f1 = c1, c2, f2
                c2 = a + g * (bb - a)
                f2 = e(c2)
        emax = max(emax, f1, f2)
    return float(-mp.log(emax, 2))


def round_factored(f: Factored, to_float: bool) -> Factored:
    """Round every coefficient to binary64 or binary32 (correctly, by mpmath)."""
    if to_float:
        def r(v):
            return mp.mpf(_to_f32(v))
    else:
        def r(v):
            return mp.mpf(float(v))
    return Factored(r(f.q0), r(f.q1), r(f.q2),
                    [r(c) for c in f.ug], [(r(y), r(a)) for y, a in f.uq], [r(y) for y in f.ul],
                    [r(c) for c in f.vg], [(r(y), r(a)) for y, a in f.vq], [r(y) for y in f.vl])


def _to_f32(v) -> float:
    """Correctly rounded binary32 value of an mpf, returned as a Python float."""
    with mp.workprec(24):
        w = +mp.mpf(v)
    out = float(w)
    if abs(out) > 3.4028234663852886e38:
        raise OverflowError("value out of binary32 range")
    if out != 0 and abs(out) < 1.1754943508222875e-38:
        raise ValueError("binary32 subnormal coefficient")
    return out


def hexf(v: float) -> str:
    return float.hex(float(v))


def decs(v) -> str:
    return mp.nstr(v, 40, min_fixed=1, max_fixed=0)


def to_f32_hex(v) -> str:
    return float.hex(_to_f32(v))


def math_check_consts(n: int) -> None:
    """Numerically confirm Eqs. q0, q1, aq, bq against the incomplete-gamma Q_n."""
    mp.mp.prec = PREC
    cn = consts(n)
    h = mp.mpf(10) ** -20
    _, Qh = exact_WQ(cn, h)
    _, Q2h = exact_WQ(cn, 2 * h)
    d0 = (4 * Qh - Q2h - 3 * cn.q0) / (2 * h)
    assert abs(Qh - cn.q0) < 1e-15, (n, Qh, cn.q0)
    assert abs(d0 - cn.q1) < 1e-15 * (1 + abs(cn.q1)), (n, d0, cn.q1)
    X = mp.mpf(10) ** 6
    _, QX = exact_WQ(cn, X)
    assert abs(QX - cn.alpha * X - cn.beta) < 1e-4, (n, QX - cn.alpha * X, cn.beta)
