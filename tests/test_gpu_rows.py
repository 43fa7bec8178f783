"""GPU: boys_eval_rows, the evaluation that stores only selected orders.

Every stored row must equal, bit for bit, the oracle's row of the same order (and so
boys_eval's), whatever the selection; rows not selected are not written; the full
2^26-argument integral workload with rows {0, 16} (the store-reduced measurement) is
checked on sampled arguments against the oracle.
"""
import sys

import numpy as np
import pytest

from gpu_common import report_mismatch, require_gpu, same_bits
from oracle import oracle as orc
from paper_2504_07637_amd import inputs

pytestmark = pytest.mark.gpu

CLASSES = ["fp64", "fp32", "fp64plus", "fp32x", "fp32s"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle(x, n, prec):
    if prec == "fp64":
        return orc.approx_f64(x, n)
    if prec == "fp32":
        return orc.approx_mixed(x, n)
    if prec == "fp32x":
        return orc.approx_f32x(x, n)
    if prec == "fp32s":
        return orc.approx_single(x, n)
    return orc.approx_f64(x, n + 1)[: n + 1]


def _masks(n, g):
    out = [[0], [n], sorted({0, n}), list(range(n + 1))]
    for _ in range(3):
        k = int(g.integers(1, n + 2))
        out.append(sorted(g.choice(n + 1, k, replace=False).tolist()))
    return out


@pytest.mark.parametrize("prec", CLASSES)
def test_selected_rows_identical_to_the_oracle(prec):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    g = np.random.default_rng(31)
    x = np.concatenate([inputs.uniform_mix(4096, seed=31),
                        inputs.integral_args(20000 + 77, seed=32),
                        [0.0, -0.0, np.inf, -1.0, np.nan, 1e300, 74.5, 47.6]])
    xd = torch.from_numpy(x).to("cuda")
    top = boys.max_nmax(prec)
    for n in sorted({0, 1, 4, 11, 16, 20, top}):
        want = _oracle(x, n, prec)
        for rows in _masks(n, g):
            _say(f"[rows] {prec} n_max={n} rows={rows}")
            # a padded output: the window beyond n and below the selected rows stays as is
            dt = torch.float32 if want.dtype == np.float32 else torch.float64
            buf = torch.full((len(rows) + 1, x.size + 40), -7.0, dtype=dt, device="cuda")
            out = buf[: len(rows), : x.size]
            boys.boys_eval_rows(xd, n, rows, prec, out=out)
            torch.cuda.synchronize()
            b = buf.cpu().numpy()
            msg = report_mismatch(f"{prec} n_max={n} rows={rows}", b[: len(rows), : x.size],
                                  want[rows])
            assert not msg, msg
            assert np.all(b[:, x.size:] == -7.0) and np.all(b[len(rows)] == -7.0)


def test_store_reduced_workload_full_size():
    # the benchmark's store-reduced configuration: 2^26 integral arguments, n_max = 16, only
    # F_0 and F_16 stored, binary64 and the mixed class; 2^16 sampled arguments plus both
    # ends against the oracle
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    n_args = 1 << 26
    x = inputs.integral_args(n_args, seed=2)
    xd = torch.from_numpy(x).to("cuda")
    g = np.random.default_rng(7)
    idx = np.unique(np.concatenate([g.choice(n_args, 1 << 16, replace=False),
                                    np.arange(64), np.arange(n_args - 64, n_args)]))
    ti = torch.from_numpy(idx).to("cuda")
    for prec in ("fp64", "fp32"):
        _say(f"[rows] full workload {prec}, rows 0 and 16")
        out = boys.boys_eval_rows(xd, 16, [0, 16], prec)
        got = out[:, ti].cpu().numpy()
        want = _oracle(x[idx], 16, prec)[[0, 16]]
        assert same_bits(got, want).all(), prec
        del out
    del xd
    torch.cuda.empty_cache()
