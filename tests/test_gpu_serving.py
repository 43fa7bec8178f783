"""GPU: the serving loop (boys_server_*) under a Poisson stream of requests.

Each checked request's result in the mix equals, bit for bit, boys_eval on the same
arguments alone and, for a sample, the CPU oracle (the tolerance is 0: the batched launch
runs the same kernels); every request completes; the device budget is respected; a small
budget makes requests wait; a result fetched and released at once, without any
synchronisation, is intact even when later requests reuse its memory.
"""
import sys

import numpy as np
import pytest

from gpu_common import require_gpu, same_bits
from oracle import oracle as orc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("budget_mb,streams", [(2048, 4), (64, 2)])
def test_serving_results_equal_solo(budget_mb, streams):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    from paper_2504_07637_amd import inputs, serving
    pool = serving.argument_pool(1 << 22, seed=5)
    P = pool.numel()
    reqs = inputs.serving_requests(rate=20000.0, duration=0.15, seed=55)
    # every fourth request in the order n+1 option or the binary32-output class computed
    # in binary64, and some mixed-class requests all in binary32, so all five classes share
    # the batches
    reqs = [(t, ln, nm, (2 if pr == 0 else 3) if i % 4 == 0 else 4 if i % 4 == 2 and pr == 1
             else pr) for i, (t, ln, nm, pr) in enumerate(reqs)]
    checked = []
    bad = []
    oracle_bad = []
    srv = None

    def check(i, rid):
        # every 17th request: compare with a solo evaluation before it is released
        if i % 17:
            return
        ta, ln, nm, pr = reqs[i]
        off = (i * 1000003) % (P - ln)
        x = pool[off:off + ln].to("cuda")
        solo = boys.boys_eval(x, nm, pr)
        got = srv.fetch(rid)
        torch.cuda.synchronize()
        checked.append(i)
        if not torch.equal(got, solo):
            bad.append((i, ln, nm, pr))
        if i % 51 == 0:
            # directly against the oracle too
            xh = pool[off:off + ln].numpy()
            if not same_bits(got.cpu().numpy(), _oracle(xh, nm, pr)).all():
                oracle_bad.append((i, ln, nm, pr))

    _say(f"[serving] {len(reqs)} requests, budget {budget_mb} MiB, {streams} streams")
    with serving.Server(budget_bytes=budget_mb << 20, streams=streams) as srv:
        res = serving.run_poisson(srv, reqs, pool, on_done=check)
        st = srv.stats()
        _say(f"[serving] {serving.summarize(res)}")
        assert st["completed"] == len(reqs) and st["device_errors"] == 0
        assert st["max_bytes_in_use"] <= budget_mb << 20
        if budget_mb == 64:
            assert st["max_queued"] > 0
        assert len(checked) == len(range(0, len(reqs), 17)) and not bad, bad[:5]
        assert not oracle_bad, oracle_bad[:5]
        assert st["bytes_in_use"] == 0 and st["failed"] == 0


def _oracle(x, n, code):
    return (orc.approx_f64(x, n) if code == 0 else orc.approx_mixed(x, n) if code == 1
            else orc.approx_f64(x, n + 1)[: n + 1] if code == 2 else orc.approx_f32x(x, n)
            if code == 3 else orc.approx_single(x, n))


def test_fetch_then_release_without_synchronisation():
    # Every completed request is fetched (a copy enqueued on the current stream) and
    # released at once, with no synchronisation, under a budget so small that later
    # requests reuse the same memory while the copies may still be pending; every 7th
    # fetched copy is checked against the oracle at the end.
    torch = require_gpu()
    from paper_2504_07637_amd import inputs, serving
    pool = serving.argument_pool(1 << 21, seed=6)
    P = pool.numel()
    reqs = inputs.serving_requests(rate=20000.0, duration=0.1, seed=66)
    reqs = [(t, min(ln, 1 << 16), nm, pr) for t, ln, nm, pr in reqs]
    fetched = {}
    srv = None

    def grab(i, rid):
        if i % 7 == 0:
            fetched[i] = srv.fetch(rid)

    _say(f"[serving] fetch+release, {len(reqs)} requests, 24 MiB budget")
    with serving.Server(budget_bytes=24 << 20, streams=2) as srv:
        serving.run_poisson(srv, reqs, pool, on_done=grab)
        st = srv.stats()
    torch.cuda.synchronize()
    assert st["max_queued"] > 0 and st["failed"] == 0 and st["bytes_in_use"] == 0
    bad = []
    for i, got in fetched.items():
        _, ln, nm, pr = reqs[i]
        off = (i * 1000003) % (P - ln)
        if not same_bits(got.cpu().numpy(), _oracle(pool[off:off + ln].numpy(), nm, pr)).all():
            bad.append(i)
    assert len(fetched) == len(range(0, len(reqs), 7)) and not bad, bad[:5]


def test_serving_refuses_what_can_never_fit():
    torch = require_gpu()
    from oracle import oracle as orc
    from paper_2504_07637_amd import serving
    from paper_2504_07637_amd._lib import BoysError
    with serving.Server(budget_bytes=16 << 20, streams=1) as srv:
        x = torch.zeros(1 << 20, dtype=torch.float64).pin_memory()
        with pytest.raises(BoysError):
            srv.submit(x, 20, "fp64")          # 176 MB of output > 16 MB budget
        with pytest.raises(BoysError):
            srv.submit(x[:10], 99, "fp64")     # unsupported n_max
        rid = srv.submit(x[:1000], 3, "fp32")
        srv.drain(10.0)
        assert srv.poll() == [rid]
        out = srv.fetch(rid)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), orc.approx_mixed(np.zeros(1000), 3))
        srv.release(rid)
