"""Pins of the oracle's consumer of F_m: contracted (ss|ss)^(m) auxiliary integrals.

For s-type Gaussians the integral of m = 0 is the Coulomb energy of two Gaussian charge
clouds, a closed form independent of the Boys-function code:
    (ss|ss)^(0) = w_a w_b (pi/p)^(3/2) (pi/q)^(3/2) erf(sqrt(rho) R) / R,  R = |P - Q|,
(its R -> 0 limit 2 sqrt(rho/pi)); for m > 0 the prefactor times the exact F_m(T).  The
contraction is a plain sum, checked against a brute-force sum of exact terms.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_07637_amd import inputs


def _one_pair(p, P, w):
    return np.array([[p], [P[0]], [P[1]], [P[2]], [w]]), np.array([0, 1], dtype=np.int32)


def test_prefactor_is_two_pi_to_the_five_halves():
    with mp.workdps(50):
        assert orc.eri_prefactor() == float(2 * mp.pi ** mp.mpf(2.5))


@pytest.mark.parametrize("p,q,R", [(0.3, 0.7, 0.0), (1.5, 40.0, 0.8), (1e3, 2e4, 0.05),
                                    (0.11, 0.09, 6.0), (12.0, 0.4, 2.2), (3.0, 5.0, 30.0)])
def test_m0_is_the_coulomb_energy_of_two_gaussian_clouds(p, q, R):
    bra, bs = _one_pair(p, (0.1, -0.2, 0.3), 0.8)
    ket, ks = _one_pair(q, (0.1 + R, -0.2, 0.3), 1.3)
    got = orc.eri_ssss(bra, bs, ket, ks, 0)[0, 0]
    with mp.workdps(40):
        pm, qm = mp.mpf(p), mp.mpf(q)
        Rm = mp.mpf(ket[1, 0]) - mp.mpf(bra[1, 0])  # the distance the oracle sees
        rho = pm * qm / (pm + qm)
        charges = mp.mpf(0.8) * mp.mpf(1.3) * (mp.pi / pm) ** 1.5 * (mp.pi / qm) ** 1.5
        want = charges * (mp.erf(mp.sqrt(rho) * Rm) / Rm if Rm != 0 else 2 * mp.sqrt(rho / mp.pi))
        assert abs(got / float(want) - 1) < 2.0 ** -45, (got, float(want))


@pytest.mark.parametrize("n", [1, 4, 16, 36])
def test_every_m_is_the_prefactor_times_the_exact_function(n, table1):
    g = np.random.default_rng(n)
    k = 64
    bra = np.vstack([g.uniform(0.1, 50, k), g.normal(0, 2, (3, k)), g.uniform(0.5, 1, k)])
    ket = np.vstack([g.uniform(0.1, 50, 1), g.normal(0, 2, (3, 1)), [1.0]])
    bs = np.arange(k + 1, dtype=np.int32)
    ks = np.array([0, 1], dtype=np.int32)
    got = orc.eri_ssss(bra, bs, ket, ks, n).reshape(n + 1, k)
    p, q = bra[0], ket[0, 0]
    rho = p * q / (p + q)
    T = rho * np.sum((bra[1:4] - ket[1:4, :1]) ** 2, axis=0)
    pref = bra[4] * (2 * math.pi ** 2.5 / (p * q * np.sqrt(p + q)))
    hi, lo = orc.exact(T, n)
    bound = min(table1[n]["fp64"]["eb0"], table1[n]["fp64"]["ebn"]) - 2.0
    for m in range(n + 1):
        rel = np.abs(got[m] / (pref * (hi[m] + lo[m])) - 1)
        assert orc.bits(rel) >= bound, (n, m, orc.bits(rel))


def test_contraction_is_the_sum_over_primitive_quartets():
    c, e, w = inputs.s_basis(4, 2, 3, seed=11, fixed_prim=False)
    pairs, start = inputs.shell_pairs(c, e, w)
    n = 6
    got = orc.eri_ssss(pairs, start, pairs, start, n)
    nc = start.size - 1
    K = 2 * math.pi ** 2.5
    for i in range(nc):
        for j in range(nc):
            acc = np.zeros(n + 1)
            for a in range(start[i], start[i + 1]):
                for b in range(start[j], start[j + 1]):
                    p, q = pairs[0, a], pairs[0, b]
                    d = pairs[1:4, a] - pairs[1:4, b]
                    T = p * q / (p + q) * float(d @ d)
                    hi, lo = orc.exact(np.array([T]), n)
                    acc += pairs[4, a] * pairs[4, b] * K / (p * q * math.sqrt(p + q)) * (hi[:, 0] + lo[:, 0])
            assert np.allclose(got[:, i * nc + j], acc, rtol=2.0 ** -42, atol=0), (i, j)


def test_empty_and_primitive_free_pairs():
    bra, bs = _one_pair(1.0, (0, 0, 0), 1.0)
    empty = np.zeros((5, 0))
    assert orc.eri_ssss(bra, bs, empty, np.array([0], dtype=np.int32), 3).shape == (4, 0)
    # a contracted pair without primitive pairs contributes nothing
    ket = np.array([[2.0], [0.5], [0.0], [0.0], [1.0]])
    ks = np.array([0, 0, 1], dtype=np.int32)
    out = orc.eri_ssss(bra, bs, ket, ks, 3)
    assert np.all(out[:, 0] == 0.0) and np.all(out[:, 1] > 0)
