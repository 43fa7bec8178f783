"""GPU: the consumer kernel (contracted (ss|ss)^(m) integrals, F_m kept in registers)
against the oracle, bit for bit: both sum the same terms in the same order, each term from
the same binary64 Boys evaluation."""
import sys

import numpy as np
import pytest

from gpu_common import report_mismatch, require_gpu
from oracle import oracle as orc
from paper_2504_07637_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, pairs, start):
    return (torch.from_numpy(np.ascontiguousarray(pairs)).to("cuda"),
            torch.from_numpy(np.ascontiguousarray(start, dtype=np.int32)).to("cuda"))


def test_identical_to_the_oracle_every_order_ragged_primitives():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    c, e, w = inputs.s_basis(8, 3, 4, seed=12, fixed_prim=False)
    bra, bs = inputs.shell_pairs(c, e, w, max_pairs=150, seed=1)
    ket, ks = inputs.shell_pairs(c, e, w, max_pairs=97, seed=2)
    B, K = _dev(torch, bra, bs), _dev(torch, ket, ks)
    for n in range(boys.max_nmax("fp64") + 1):
        _say(f"[eri] n_max={n} bra={bs.size - 1} ket={ks.size - 1}")
        got = boys.boys_eri_ssss(*B, *K, n)
        torch.cuda.synchronize()
        msg = report_mismatch(f"eri n_max={n}", got.cpu().numpy(),
                              orc.eri_ssss(bra, bs, ket, ks, n))
        assert not msg, msg


def test_empty_lists_and_primitive_free_pairs():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    bra = np.array([[1.0, 3.0], [0.0, 0.1], [0.0, 0.0], [0.0, 0.2], [1.0, 0.5]])
    bs = np.array([0, 2], dtype=np.int32)
    ket = np.array([[2.0], [0.5], [0.0], [0.0], [1.0]])
    ks = np.array([0, 0, 1, 1], dtype=np.int32)  # pairs 0 and 2 have no primitives
    got = boys.boys_eri_ssss(*_dev(torch, bra, bs), *_dev(torch, ket, ks), 5)
    torch.cuda.synchronize()
    want = orc.eri_ssss(bra, bs, ket, ks, 5)
    assert np.array_equal(got.cpu().numpy(), want)
    assert np.all(want[:, [0, 2]] == 0) and np.all(want[:, 1] > 0)
    none = np.zeros((5, 0))
    out = boys.boys_eri_ssss(*_dev(torch, bra, bs), *_dev(torch, none, np.array([0])), 5)
    torch.cuda.synchronize()
    assert out.shape == (6, 0)


@pytest.mark.parametrize("n,nrows", [(16, 22), (22, 6), (36, 6)])
def test_full_size_workload_sampled(n, nrows):
    # the benchmark's 2048 x 2048 contracted pairs (9 primitive pairs each): sampled bra
    # rows in full against the oracle, at n_max = 16 (the benchmark's order) and at two
    # orders of the streaming form (22, 36)
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    c, e, w = inputs.s_basis()
    pairs, start = inputs.shell_pairs(c, e, w, max_pairs=2048)
    nc = start.size - 1
    _say(f"[eri] full {nc} x {nc}, n_max={n}")
    got = boys.boys_eri_ssss(*_dev(torch, pairs, start), *_dev(torch, pairs, start), n)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, nc - 1],
                                     np.random.default_rng(9 + n).integers(0, nc, nrows)]))
    for i in rows:
        sub = pairs[:, start[i]:start[i + 1]]
        want = orc.eri_ssss(sub, np.array([0, sub.shape[1]], dtype=np.int32), pairs, start, n)
        g = got[:, i * nc:(i + 1) * nc].cpu().numpy()
        msg = report_mismatch(f"eri row {i} n_max={n}", g, want)
        assert not msg, msg


def _ragged_list(rng, count, max_prim, centre):
    """count contracted pairs of 1..max_prim primitive pairs each; centre(k) gives the
    product centre of primitive pair k."""
    sizes = rng.integers(1, max_prim + 1, count)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(start[-1])
    P = np.array([centre(k) for k in range(n)], dtype=np.float64).reshape(n, 3)
    pairs = np.stack([rng.uniform(0.3, 6.0, n), P[:, 0], P[:, 1], P[:, 2],
                      rng.uniform(0.1, 1.0, n)])
    return pairs, start


@pytest.mark.parametrize("n", [0, 7, 16, 36])
def test_every_argument_below_the_cut_off(n):
    # coincident centres: every T is 0, so every lane of every wave-step lies below the
    # cut-off and queues its argument; a window then holds one step and the next step is
    # carried into the following window
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    rng = np.random.default_rng(31 + n)
    bra, bs = _ragged_list(rng, 37, 5, lambda k: (0.25, -1.0, 2.0))
    ket, ks = _ragged_list(rng, 53, 4, lambda k: (0.25, -1.0, 2.0))
    _say(f"[eri] all below the cut-off, n_max={n}, {bs.size - 1} x {ks.size - 1}")
    got = boys.boys_eri_ssss(*_dev(torch, bra, bs), *_dev(torch, ket, ks), n)
    torch.cuda.synchronize()
    msg = report_mismatch(f"eri all-below n_max={n}", got.cpu().numpy(),
                          orc.eri_ssss(bra, bs, ket, ks, n))
    assert not msg, msg


@pytest.mark.parametrize("n", [3, 16, 30])
def test_lanes_on_both_sides_in_blocks(n):
    # kets alternate in runs between coincident centres (every argument below the cut-off)
    # and distant ones (every argument past it), with ragged primitive counts, so that
    # windows fill, carry and mix lanes of both sides and of different lengths
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    rng = np.random.default_rng(77 + n)
    bra, bs = _ragged_list(rng, 29, 6, lambda k: (0.0, 0.0, 0.0))
    far = rng.uniform(40.0, 80.0, 4000)  # T >= 0.15 * 40^2, past every cut-off
    ket, ks = _ragged_list(rng, 150, 7,
                           lambda k: (0.0, 0.0, 0.0) if (k // 23) % 2 else (far[k], 0.0, 0.0))
    _say(f"[eri] mixed sides, n_max={n}, {bs.size - 1} x {ks.size - 1}")
    got = boys.boys_eri_ssss(*_dev(torch, bra, bs), *_dev(torch, ket, ks), n)
    torch.cuda.synchronize()
    want = orc.eri_ssss(bra, bs, ket, ks, n)
    msg = report_mismatch(f"eri mixed sides n_max={n}", got.cpu().numpy(), want)
    assert not msg, msg


@pytest.mark.parametrize("n", [5, 16])
def test_special_pair_values(n):
    # zero and negative exponents (T = 0, T < 0: NaN), infinite and NaN centres and weights,
    # mixed into ordinary pairs: every output equals the oracle's, NaN for NaN
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    rng = np.random.default_rng(5 + n)
    bra, bs = _ragged_list(rng, 21, 4, lambda k: (0.1 * k, 0.0, 0.3))
    ket, ks = _ragged_list(rng, 67, 3, lambda k: (0.0, 0.05 * k, -0.2))
    bra[0, 3], bra[0, 7] = 0.0, -1.5
    bra[1, 11], bra[4, 13] = np.inf, np.nan
    ket[0, 5], ket[2, 9], ket[3, 17] = -0.25, -np.inf, np.nan
    ket[4, 21] = np.inf
    _say(f"[eri] special values, n_max={n}")
    got = boys.boys_eri_ssss(*_dev(torch, bra, bs), *_dev(torch, ket, ks), n)
    torch.cuda.synchronize()
    want = orc.eri_ssss(bra, bs, ket, ks, n)
    assert np.isnan(want).any() and np.isfinite(want).any()
    msg = report_mismatch(f"eri special n_max={n}", got.cpu().numpy(), want)
    assert not msg, msg
