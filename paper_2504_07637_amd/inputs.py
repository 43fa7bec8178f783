"""Seeded synthetic argument generators (shared by the tests, the benchmark and the checks).

This module holds no Boys-function arithmetic: it only draws arguments x >= 0 with the
shapes and distributions of the workloads below.  The paper evaluates on evenly spaced
grids over [0, z_nb) (section "Computations"); the integral-engine-like distributions
stand in for the arguments that a Gaussian-basis integral code produces.

    uniform_mix(n)      1/4 exact zeros, 1/4 U[0,1], 1/4 log-U[1,50], 1/4 log-U[50,1e4],
                        then shuffled (the small latency workload, 65,536 arguments).
    integral_args(n)    x = rho |PQ|^2 with rho = ab/(a+b), a, b log-uniform in
                        [0.05, 5e4], PQ a 3-D normal vector with sigma = 2.0 bohr per axis,
                        and exactly round(0.01 n) exact zeros at random positions.
    table1_grid(z, k)   the evenly spaced grid x_j = j z / k, j = 0..k-1.
    batch_plan(count)   lengths log-uniform in [32, 65536] (rounded), n_max uniform in
                        {0..16}, precision alternating binary64 / binary32 by index.
    serving_requests()  Poisson arrivals; lengths log-uniform in [64, 262144], n_max
                        uniform in {0..20}, precision binary64 or binary32 at 50/50.
    s_basis()           s-type shells on atoms of a jittered cubic grid (2.6 bohr spacing,
                        0.3 bohr jitter), 1..max_prim primitives per shell, exponents
                        log-uniform in [0.05, 5e4], coefficients U[0.1, 1].
    shell_pairs()       the Gaussian products of shell pairs (a seeded subset, or all
                        s1 <= s2): per primitive pair p = a + b, P = (aA + bB)/p and the
                        weight c_a c_b exp(-ab/p |AB|^2), as (5, n) rows (p, Px, Py, Pz, w)
                        with int32 offsets per contracted pair.  This is how a Gaussian
                        integral code prepares the pair data whose x = rho |PQ|^2 reaches
                        the Boys functions; it is input preparation, not Boys arithmetic.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _log_uniform(g, lo, hi, size):
    return np.exp(g.uniform(np.log(lo), np.log(hi), size))


def uniform_mix(n: int = 65536, seed: int = 1) -> np.ndarray:
    g = rng(seed)
    q = n // 4
    parts = [np.zeros(q),
             g.uniform(0.0, 1.0, q),
             _log_uniform(g, 1.0, 50.0, q),
             _log_uniform(g, 50.0, 1e4, n - 3 * q)]
    x = np.concatenate(parts)
    return x[g.permutation(n)].copy()


def integral_args(n: int = 1 << 26, seed: int = 2, chunk: int = 1 << 22) -> np.ndarray:
    g = rng(seed)
    x = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        k = min(chunk, n - s)
        a = _log_uniform(g, 0.05, 5e4, k)
        b = _log_uniform(g, 0.05, 5e4, k)
        pq = g.normal(0.0, 2.0, (k, 3))
        x[s:s + k] = (a * b / (a + b)) * np.einsum("ij,ij->i", pq, pq)
    nz = int(round(0.01 * n))
    if nz:
        x[g.choice(n, nz, replace=False)] = 0.0
    return x


def table1_grid(z: float, k: int = 1 << 20) -> np.ndarray:
    return np.arange(k, dtype=np.float64) * (z / k)


def batch_plan(count: int = 8192, seed: int = 4, max_len: int = 65536, min_len: int = 32,
               nmax_hi: int = 16):
    """[(length, n_max, precision)] with precision 0 = binary64, 1 = binary32."""
    g = rng(seed)
    lens = np.rint(_log_uniform(g, min_len, max_len, count)).astype(np.int64)
    nmax = g.integers(0, nmax_hi + 1, count)
    prec = np.arange(count) % 2
    return [(int(l), int(m), int(p)) for l, m, p in zip(lens, nmax, prec)]


def serving_requests(rate: float = 20000.0, duration: float = 1.0, seed: int = 5,
                     min_len: int = 64, max_len: int = 262144, nmax_hi: int = 20):
    """[(arrival_time_s, length, n_max, precision)] for a Poisson stream."""
    g = rng(seed)
    t = 0.0
    out = []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append((t, int(np.rint(_log_uniform(g, min_len, max_len, 1))[0]),
                    int(g.integers(0, nmax_hi + 1)), int(g.integers(0, 2))))
    return out


def s_basis(n_atoms: int = 32, shells_per_atom: int = 8, max_prim: int = 3, seed: int = 6,
            fixed_prim: bool = True):
    """(centres (S, 3), [exponents per shell], [coefficients per shell]); every shell has
    max_prim primitives when fixed_prim, else 1..max_prim."""
    g = rng(seed)
    side = int(np.ceil(n_atoms ** (1.0 / 3.0)))
    grid = np.array([(i, j, k) for i in range(side) for j in range(side) for k in range(side)],
                    dtype=np.float64)[:n_atoms]
    atoms = 2.6 * grid + g.normal(0.0, 0.3, (n_atoms, 3))
    centres, exps, coefs = [], [], []
    for a in range(n_atoms):
        for _ in range(shells_per_atom):
            k = max_prim if fixed_prim else int(g.integers(1, max_prim + 1))
            centres.append(atoms[a])
            exps.append(np.sort(_log_uniform(g, 0.05, 5e4, k))[::-1].copy())
            coefs.append(g.uniform(0.1, 1.0, k))
    return np.array(centres), exps, coefs


def shell_pairs(centres, exps, coefs, max_pairs: int | None = None, seed: int = 7):
    """(pairs (5, n_prim_pairs) float64, start (count+1,) int32) for the shell pairs."""
    S = len(centres)
    allp = [(i, j) for i in range(S) for j in range(i, S)]
    if max_pairs is not None and max_pairs < len(allp):
        g = rng(seed)
        pick = np.sort(g.choice(len(allp), max_pairs, replace=False))
        allp = [allp[k] for k in pick]
    cols, start = [], [0]
    for i, j in allp:
        A, B = centres[i], centres[j]
        ab2 = float(np.sum((A - B) ** 2))
        for a, ca in zip(exps[i], coefs[i]):
            for b, cb in zip(exps[j], coefs[j]):
                p = a + b
                P = (a * A + b * B) / p
                cols.append((p, P[0], P[1], P[2], ca * cb * np.exp(-a * b / p * ab2)))
        start.append(len(cols))
    pairs = np.array(cols, dtype=np.float64).T.copy() if cols else np.zeros((5, 0))
    return pairs, np.array(start, dtype=np.int32)

