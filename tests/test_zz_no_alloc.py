"""GPU: boys_eval_batched_noalloc, the allocation-free batched entry point, through the C
ABI: its results equal those of boys_eval_batched bit for bit, on two calls in a row (the
second with a smaller batch, so the fixed scratch array holds stale tables from the
first), and a sample equals the CPU oracle."""
import sys

import numpy as np
import pytest

from gpu_common import require_gpu
from oracle import oracle as orc
from paper_2504_07637_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(torch, count, seed, max_len, nmax_hi):
    spec = inputs.batch_plan(count, seed=seed, max_len=max_len, nmax_hi=nmax_hi)
    total = sum(l for l, _, _ in spec)
    x = inputs.integral_args(total, seed=seed + 1)
    xd = torch.from_numpy(x).to("cuda")
    xs, hs, off = [], [], 0
    for l, _, _ in spec:
        xs.append(xd[off:off + l])
        hs.append(x[off:off + l])
        off += l
    nm = [m for _, m, _ in spec]
    names = ("fp64", "fp32", "fp64plus", "fp32x", "fp32s")
    # every class, orders up to nmax_hi (fp64plus one less)
    pr = [names[k % 5] for k in range(count)]
    nm = [min(m, 35) if p == "fp64plus" else m for m, p in zip(nm, pr)]
    return xs, hs, nm, pr


def _bits(t):
    import torch
    return t.view(torch.int64 if t.dtype == torch.float64 else torch.int32)


def _noalloc(boys, xs, nm, pr):
    """Through the C ABI: marshal, call boys_eval_batched_noalloc, check the status."""
    from paper_2504_07637_amd import _lib
    import torch
    arr, outs = boys._arrays(xs, nm, pr, None)
    for o in outs:
        o.fill_(-7.0)
    st = _lib.lib().boys_eval_batched_noalloc(arr, len(xs),
                                              torch.cuda.current_stream().cuda_stream)
    assert st == _lib.OK, _lib.status_string(st)
    return outs


@pytest.mark.parametrize("first,second", [((700, 3, 65536, 36), (90, 13, 4096, 20))])
def test_noalloc_equals_batched_twice(first, second):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    for call, (count, seed, max_len, nmax_hi) in enumerate((first, second)):
        xs, hs, nm, pr = _batch(torch, count, seed, max_len, nmax_hi)
        _say(f"[noalloc] call {call}: {count} arrays, {sum(x.numel() for x in xs)} arguments")
        got = _noalloc(boys, xs, nm, pr)
        want = boys.boys_eval_batched(xs, nm, pr)
        torch.cuda.synchronize()
        for k, (g, w) in enumerate(zip(got, want)):
            assert torch.equal(_bits(g), _bits(w)), f"call {call}, array {k} ({pr[k]}, n_max {nm[k]})"
        for k in range(0, count, 29):
            if pr[k] == "fp64":
                want_o = orc.approx_f64(hs[k], nm[k])
            elif pr[k] == "fp32":
                want_o = orc.approx_mixed(hs[k], nm[k])
            else:
                continue
            g = got[k].cpu().numpy()
            assert np.array_equal(g.view(np.int64 if g.dtype == np.float64 else np.int32),
                                  want_o.view(np.int64 if want_o.dtype == np.float64
                                              else np.int32)), f"call {call}, array {k} vs the oracle"


def test_noalloc_empty_and_too_large():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    from paper_2504_07637_amd import _lib
    x = torch.zeros(0, dtype=torch.float64, device="cuda")
    outs = boys.boys_eval_batched_noalloc([x, x], [2, 5], ["fp64", "fp32"])
    assert [tuple(o.shape) for o in outs] == [(3, 0), (6, 0)]
    assert _lib.lib().boys_eval_batched_noalloc(None, 0, None) == _lib.OK
    # more tiles than the fixed array holds: refused on the host, nothing launched
    big = torch.empty(1, dtype=torch.float64, device="cuda")
    arr = (_lib.BoysArray * 1)()
    arr[0].x = arr[0].out = big.data_ptr()
    arr[0].n = arr[0].ld_out = 1 << 30
    arr[0].n_max, arr[0].precision = 0, _lib.FP64
    assert _lib.lib().boys_eval_batched_noalloc(arr, 1, None) == _lib.ERR_TOO_LARGE
