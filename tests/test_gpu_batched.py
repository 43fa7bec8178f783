"""GPU: the persistent batched launch and its plans (HIP graph replay, update, autotune).

Invariant: every array's result in a batch is bit for bit the result of boys_eval on that
array alone (the batched kernel runs the same unrolled bodies), and for a sample of arrays
also identical to the CPU oracle.
"""
import sys

import numpy as np
import pytest

from gpu_common import report_mismatch, require_gpu, same_bits
from oracle import oracle as orc
from paper_2504_07637_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(torch, count, seed, max_len=65536, nmax_hi=16):
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
    pr = ["fp64" if p == 0 else "fp32" for _, _, p in spec]
    return xs, hs, nm, pr


def _solo(boys, xs, nm, pr):
    return [boys.boys_eval(x, m, p) for x, m, p in zip(xs, nm, pr)]


def test_batched_equals_solo_and_oracle():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    xs, hs, nm, pr = _batch(torch, 600, 40)
    _say(f"[batched] 600 arrays, {sum(x.numel() for x in xs)} arguments")
    outs = boys.boys_eval_batched(xs, nm, pr)
    solo = _solo(boys, xs, nm, pr)
    torch.cuda.synchronize()
    for k, (o, s) in enumerate(zip(outs, solo)):
        msg = report_mismatch(f"array {k}", o.cpu().numpy(), s.cpu().numpy())
        assert not msg, msg
    for k in range(0, 600, 37):
        want = orc.approx_f64(hs[k], nm[k]) if pr[k] == "fp64" else orc.approx_mixed(hs[k], nm[k])
        assert same_bits(outs[k].cpu().numpy(), want).all(), k


def test_plan_graph_replays_and_update():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    xs, hs, nm, pr = _batch(torch, 300, 50, nmax_hi=20)
    solo = [s.cpu().numpy() for s in _solo(boys, xs, nm, pr)]
    plan = boys.Plan(xs, nm, pr, tuning={"tile": 1024, "block": 256, "grid_per_cu": 2})
    for rep in range(4):
        _say(f"[plan] replay {rep}")
        for o in plan.outs:
            o.fill_(-1.0)
        plan.execute()
        # eager work and a synchronisation between replays
        torch.ones(1 << 20, device="cuda").sum().item()
        torch.cuda.synchronize()
        for k, o in enumerate(plan.outs):
            assert same_bits(o.cpu().numpy(), solo[k]).all(), (rep, k)
    # new argument and output buffers with the same shapes
    xs2 = [x.flip(0).contiguous() for x in xs]
    outs2 = [torch.empty_like(o) for o in plan.outs]
    plan.update(xs2, outs2)
    plan.execute()
    torch.cuda.synchronize()
    solo2 = _solo(boys, xs2, nm, pr)
    for k, (o, s) in enumerate(zip(plan.outs, solo2)):
        assert same_bits(o.cpu().numpy(), s.cpu().numpy()).all(), k
    plan.close()


def test_full_batched_workload_equals_solo():
    # the 8,192-array workload (lengths log-uniform in [32, 65536], n_max 0..16,
    # binary64 and binary32 alternating) in one launch
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    xs, hs, nm, pr = _batch(torch, 8192, 4)
    _say(f"[batched] 8192 arrays, {sum(x.numel() for x in xs)} arguments")
    plan = boys.Plan(xs, nm, pr)
    plan.execute()
    torch.cuda.synchronize()
    for k in range(0, 8192, 1):
        s = boys.boys_eval(xs[k], nm[k], pr[k])
        # bit patterns, so that a NaN on one side and a number on the other differ
        ib = torch.int64 if s.dtype == torch.float64 else torch.int32
        if not torch.equal(plan.outs[k].view(ib), s.view(ib)):
            pytest.fail(f"array {k} differs from its solo evaluation")
    # a sample of the arrays straight against the oracle
    for k in range(0, 8192, 97):
        want = orc.approx_f64(hs[k], nm[k]) if pr[k] == "fp64" else orc.approx_mixed(hs[k], nm[k])
        assert same_bits(plan.outs[k].cpu().numpy(), want).all(), f"array {k} vs the oracle"
    plan.close()


@pytest.mark.parametrize("tuning", [
    {"schedule": 0, "tile": 256, "block": 256, "grid_per_cu": 4, "order": 0},
    {"schedule": 0, "tile": 256, "block": 64, "grid_per_cu": 16, "order": 1},
    {"schedule": 0, "tile": 256, "block": 128, "grid_per_cu": 1, "order": 2},
    {"schedule": 1, "tile": 256, "block": 256, "grid_per_cu": 1, "order": 2},
    {"schedule": 1, "tile": 512, "block": 128, "grid_per_cu": 1, "order": 0},
    {"schedule": 1, "tile": 256, "block": 64, "grid_per_cu": 1, "order": 1},
    {"schedule": 2, "tile": 256, "block": 256, "grid_per_cu": 1, "order": 1},
    {"schedule": 2, "tile": 256, "block": 64, "grid_per_cu": 1, "order": 0},
    {"schedule": 2, "tile": 256, "block": 128, "grid_per_cu": 1, "order": 2},
    {"schedule": 2, "tile": 256, "block": 256, "grid_per_cu": 1, "order": 1, "split_nmax": 8},
    {"schedule": 2, "tile": 256, "block": 64, "grid_per_cu": 1, "order": 0, "split_nmax": 1},
    {"schedule": 2, "tile": 256, "block": 128, "grid_per_cu": 1, "order": 2, "split_nmax": 40}])
def test_every_schedule_equals_solo(tuning):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    xs, hs, nm, pr = _batch(torch, 300, 70, nmax_hi=35)
    # every third array in the binary64 class with the order n+1 option, every fifth
    # in the binary32-output class computed in binary64, every seventh all in binary32
    pr = ["fp64plus" if k % 3 == 0 else "fp32x" if k % 5 == 0 else "fp32s" if k % 7 == 0
          else p for k, p in enumerate(pr)]
    _say(f"[schedule] {tuning}")
    plan = boys.Plan(xs, nm, pr, tuning=tuning)
    plan.execute()
    solo = _solo(boys, xs, nm, pr)
    torch.cuda.synchronize()
    for k, (o, s) in enumerate(zip(plan.outs, solo)):
        assert same_bits(o.cpu().numpy(), s.cpu().numpy()).all(), (tuning, k)
    plan.close()


def test_autotune_picks_a_candidate(tmp_path, monkeypatch):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    from paper_2504_07637_amd import tuning
    xs, hs, nm, pr = _batch(torch, 200, 60)
    cands = [{"schedule": 0, "tile": 256, "block": 256, "grid_per_cu": 2, "order": 0},
             {"schedule": 0, "tile": 256, "block": 256, "grid_per_cu": 4, "order": 1},
             {"schedule": 1, "tile": 512, "block": 128, "grid_per_cu": 1, "order": 2}]
    best, times = boys.autotune(xs, nm, pr, cands, warmup=1, reps=2)
    assert best in cands and all(t > 0 for t in times)
    assert times[cands.index(best)] == min(times)
    monkeypatch.setenv("BOYS_TUNING_FILE", str(tmp_path / "tuning.json"))
    t1, info1 = tuning.tuned(xs, nm, pr, candidates=cands, warmup=1, reps=2)
    t2, info2 = tuning.tuned(xs, nm, pr, candidates=cands)
    assert not info1["cached"] and info2["cached"] and t1 == t2 and t1 in cands


def test_empty_arrays_and_empty_batches():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = torch.from_numpy(inputs.integral_args(5000, seed=90)).to("cuda")
    xs = [x[:0], x[:1000], x[1000:1000], x[1000:5000]]
    nm, pr = [3, 7, 0, 20], ["fp64", "fp32x", "fp64", "fp64plus"]
    outs = boys.boys_eval_batched(xs, nm, pr)
    torch.cuda.synchronize()
    for xi, o, m, p in zip(xs, outs, nm, pr):
        assert o.shape == (m + 1, xi.numel())
        if xi.numel():
            assert torch.equal(o, boys.boys_eval(xi, m, p))
    # a batch of only empty arrays, and no arrays at all
    outs = boys.boys_eval_batched([x[:0], x[:0]], [2, 5], ["fp64", "fp32"])
    assert [o.shape for o in outs] == [(3, 0), (6, 0)]
    plan = boys.Plan([x[:0]], [4], ["fp64"])
    plan.execute()
    plan.close()
    from paper_2504_07637_amd import _lib
    assert _lib.lib().boys_eval_batched(None, 0, None) == _lib.OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("counts", [[1], [3, 1], [300, 5, 256, 257, 1, 70000]])
def test_persistent_schedule_small_batches(counts):
    # the persistent waves with fewer tiles than work queues (8), a single argument, and
    # arrays whose lengths straddle the 256-argument tile; every class
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    names = ["fp64", "fp32", "fp64plus", "fp32x", "fp32s"]
    x = inputs.integral_args(sum(counts), seed=77)
    xd = torch.from_numpy(x).to("cuda")
    xs, off = [], 0
    for c in counts:
        xs.append(xd[off:off + c])
        off += c
    nm = [(7 * k + 3) % 17 for k in range(len(counts))]
    pr = [names[k % 5] for k in range(len(counts))]
    _say(f"[persistent] lengths {counts}")
    for gpc in (1, 8):
        plan = boys.Plan(xs, nm, pr, tuning={"schedule": 0, "tile": 256, "block": 256,
                                             "grid_per_cu": gpc, "order": 1})
        for rep in range(2):
            for o in plan.outs:
                o.fill_(-3.0)
            plan.execute()
            solo = _solo(boys, xs, nm, pr)
            torch.cuda.synchronize()
            for k, (o, s) in enumerate(zip(plan.outs, solo)):
                assert same_bits(o.cpu().numpy(), s.cpu().numpy()).all(), (gpc, rep, k)
        plan.close()
