"""The serving loop's host policy (csrc/serve_core.h) on the CPU, with a fake executor.

Compiles tests/native/serve_core_harness.cpp with g++ and checks: the pool never
overlaps or leaks and coalesces back to one block; admission follows arrival order and
never exceeds the budget; every request completes once; batches overlap on different
slots, and requests that arrive while a batch runs are launched before it ends
(continuous batching); requests that can never fit are refused at submission; a failed
launch or a failed completion fails exactly its batch's requests, once, with no retry; a
released request keeps its memory until the reads of its result enqueued before the
release have completed.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(REPO, "tests", "native", "serve_core_harness.cpp")
CSRC = os.path.join(REPO, "paper_2504_07637_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    out = tmp_path_factory.mktemp("serve") / "libserve_core.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC,
                           "-o", str(out), SRC])
    L = ctypes.CDLL(str(out))
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_int64)
    L.sim_run.argtypes = [ctypes.c_int, dp, lp, ip, ip, ctypes.c_int64, ctypes.c_int,
                          ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp, ip, ip,
                          lp, ip, ip, ip]
    L.pool_fuzz.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
    L.sim_failures.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ip,
                               ctypes.c_int, ip, ctypes.c_int, ip, ip, ip]
    L.sim_pending_read.argtypes = [ctypes.c_int64, ctypes.c_double, dp,
                                   ctypes.POINTER(ctypes.c_uint64), ip]
    return L


def footprint(n, nmax, prec):
    a = lambda v: (v + 255) // 256 * 256
    es = 4 if prec in (1, 3, 4) else 8   # binary32 outputs for classes 1, 3 and 4
    q = 128 // es
    ld = (n + q - 1) // q * q
    return a(8 * n) + a((nmax + 1) * ld * es)


def simulate(L, t, ln, nm, pr, budget, slots=4, max_batch=256, bw=1e12, dt=2e-6):
    n = len(t)
    t = np.ascontiguousarray(t, dtype=np.float64)
    ln = np.ascontiguousarray(ln, dtype=np.int64)
    nm = np.ascontiguousarray(nm, dtype=np.int32)
    pr = np.ascontiguousarray(pr, dtype=np.int32)
    ta, tl, td = (np.full(n, -1.0) for _ in range(3))
    sl = np.full(n, -1, dtype=np.int32)
    rc = np.zeros(n, dtype=np.int32)
    mu, mi, mc, nb = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    c = lambda a, ty: a.ctypes.data_as(ctypes.POINTER(ty))
    done = L.sim_run(n, c(t, ctypes.c_double), c(ln, ctypes.c_int64), c(nm, ctypes.c_int),
                     c(pr, ctypes.c_int), budget, slots, max_batch, bw, dt,
                     c(ta, ctypes.c_double), c(tl, ctypes.c_double), c(td, ctypes.c_double),
                     c(sl, ctypes.c_int), c(rc, ctypes.c_int), ctypes.byref(mu),
                     ctypes.byref(mi), ctypes.byref(mc), ctypes.byref(nb))
    return dict(done=done, admit=ta, launch=tl, end=td, slot=sl, rc=rc, max_in_use=mu.value,
                max_inflight=mi.value, max_concurrent=mc.value, batches=nb.value)


def _poisson(seed, count, rate, lo=64, hi=262144, nmax_hi=20):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, count))
    ln = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    nm = g.integers(0, nmax_hi + 1, count).astype(np.int32)
    pr = g.integers(0, 5, count).astype(np.int32)
    return t, ln, nm, pr


def test_pool_invariants(harness):
    for seed in range(6):
        assert harness.pool_fuzz(seed, 20000, 1 << 30) == 0


def test_admission_order_budget_and_completion(harness):
    t, ln, nm, pr = _poisson(1, 3000, 20000.0)
    budget = 64 << 20  # small: forces queueing for memory
    r = simulate(harness, t, ln, nm, pr, budget, bw=3e10)
    assert r["done"] == len(t) and np.all(r["rc"] == 0)
    assert r["max_in_use"] <= budget
    # admitted in arrival order, never before arrival, launched after admission
    assert np.all(np.diff(r["admit"]) >= 0)
    assert np.all(r["admit"] >= t - 1e-12) and np.all(r["launch"] >= r["admit"])
    assert np.all(r["end"] >= r["launch"])
    # memory really was the limit at times: some requests waited for admission
    assert np.max(r["admit"] - t) > 1e-4


def test_continuous_batching_overlaps(harness):
    t, ln, nm, pr = _poisson(2, 2000, 20000.0)
    r = simulate(harness, t, ln, nm, pr, 8 << 30, slots=4, bw=5e10)
    assert r["done"] == len(t)
    assert r["max_concurrent"] >= 2          # batches ran on several slots at once
    assert r["batches"] < len(t)             # requests were coalesced into batches
    # some request that arrived after another request's launch was launched before that
    # other request finished: it joined while work was in flight
    order = np.argsort(r["launch"])
    joined = 0
    for j in range(1, len(order)):
        a, b = order[j - 1], order[j]
        if r["slot"][a] != r["slot"][b] and t[b] > r["launch"][a] and r["launch"][b] < r["end"][a]:
            joined += 1
    assert joined > 0


def test_oversized_requests_are_refused(harness):
    t = np.array([0.0, 1e-5, 2e-5])
    ln = np.array([1000, 10_000_000, 1000], dtype=np.int64)
    nm = np.array([4, 20, 4], dtype=np.int32)
    pr = np.array([0, 0, 1], dtype=np.int32)
    budget = footprint(10_000_000, 20, 0) - 1
    r = simulate(harness, t, ln, nm, pr, budget)
    assert list(r["rc"]) == [0, 3, 0]
    assert r["done"] == 2
    # an unknown precision class is an argument error (1), the others are admitted
    pr = np.array([5, 4, 2], dtype=np.int32)
    ln = np.array([1000, 1000, 1000], dtype=np.int64)
    r = simulate(harness, t, ln, nm, pr, 1 << 30)
    assert list(r["rc"]) == [1, 0, 0] and r["done"] == 2


def test_policy_core_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # the pool fuzz and a simulated stream, host code only, built with ASan and UBSan
    exe = tmp_path / "serve_core_sanitized"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", CSRC, "-o", str(exe),
           os.path.join(REPO, "tests", "native", "serve_core_sanitize.cpp"), SRC]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout


def _failures(L, nreq, n, slots, max_batch, fail_launch, fail_done):
    ip = ctypes.POINTER(ctypes.c_int)
    fl = np.ascontiguousarray(fail_launch, dtype=np.int32)
    fd = np.ascontiguousarray(fail_done, dtype=np.int32)
    st = np.zeros(nreq, dtype=np.int32)
    rp = np.zeros(nreq, dtype=np.int32)
    failed = ctypes.c_int()
    launches = L.sim_failures(nreq, n, slots, max_batch, fl.ctypes.data_as(ip), fl.size,
                              fd.ctypes.data_as(ip), fd.size, st.ctypes.data_as(ip),
                              rp.ctypes.data_as(ip), ctypes.byref(failed))
    return launches, st, rp, failed.value


DONE, FAILED = 3, 4


def test_failed_launches_and_completions_fail_their_batch_once(harness):
    # requests 1e-4 s apart, each served long before the next arrives: launch attempt k
    # carries request k alone.  Attempts 0 and 3 fail to launch; of the launched batches,
    # numbers 1 and 5 (requests 2 and 7) report a device error at completion.
    launches, st, rp, failed = _failures(harness, 40, 1000, 2, 4, [0, 3], [1, 5])
    assert launches == 40                      # no attempt was repeated
    assert np.all(rp == 1)                     # each request reported exactly once
    want = np.full(40, DONE)
    want[[0, 2, 3, 7]] = FAILED
    assert np.array_equal(st, want), np.nonzero(st != want)
    assert failed == 4


def test_failures_inside_coalesced_batches(harness):
    # long requests pile up behind each other, so launches carry several requests: a failed
    # launch or completion fails all of them, the rest complete, nothing is retried and the
    # pool empties
    launches, st, rp, failed = _failures(harness, 200, 3_000_000, 3, 8, [0, 3, 9], [1, 5, 6])
    assert launches > 0, launches
    assert launches < 200                      # requests were coalesced
    assert np.all(rp == 1)
    assert failed == int(np.sum(st == FAILED)) and failed >= 6
    assert np.all((st == DONE) | (st == FAILED))


def test_release_waits_for_pending_reads(harness):
    # A's result is being read until t = 10 ms; A is released at once.  B needs A's memory,
    # so B is admitted only after the read has completed, and A's bytes stay in use meanwhile
    n = 100000
    tb = ctypes.c_double()
    in_use = ctypes.c_uint64()
    freed = ctypes.c_int()
    rc = harness.sim_pending_read(n, 0.01, ctypes.byref(tb), ctypes.byref(in_use),
                                  ctypes.byref(freed))
    assert rc == 0, rc
    assert tb.value >= 0.01
    assert in_use.value == footprint(n, 4, 0)
    assert freed.value == 2
