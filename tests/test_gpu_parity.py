"""GPU parity: libboys.so (through its C ABI) against the CPU oracle, element by element.

Bar:
  * against the oracle's evaluation of the same approximant (same coefficients, same
    steps): identical bits in both precision classes.  The stated tolerance for binary64
    is 4 ulp; the arithmetic contract of the library (correctly rounded basic operations,
    correctly rounded exp, the same evaluation order) makes the expected difference 0,
    and that is what is asserted;
  * against the exact Boys function: the finite-precision error bounds of Table 1 (with
    one bit of margin, since our coefficients are a re-fit): F_n within 2^-(eb_n - 1),
    F_{n-1} within 2^-(eb_{n-1} - 1), lower orders within 2^-(min(eb_0, eb_{n-1}) - 1);
    for the mixed class the binary32 columns, over outputs with |F| >= FLT_MIN (smaller
    outputs within an absolute 2^-(bound) * FLT_MIN + FLT_TRUE_MIN).
Inputs are seeded draws of the workload distributions (paper_2504_07637_amd.inputs).
"""
import sys

import numpy as np
import pytest

from gpu_common import report_mismatch, require_gpu, same_bits
from oracle import oracle as orc
from paper_2504_07637_amd import inputs

pytestmark = pytest.mark.gpu

FLT_MIN = 1.1754943508222875e-38
FLT_TRUE_MIN = 1.401298464324817e-45


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _special():
    return np.array([0.0, -0.0, 5e-324, 1e-300, 1e-20, 2.0 ** -54, 1e-8, np.inf, -1.0, -np.inf,
                     np.nan, 1e300, 1.7e308, 1e18, 3e8, 745.0, 709.0, 120.0, 110.0, 78.0,
                     47.6, 74.5, 1.0, 0.5, 25.0])


def _gpu_eval(torch, x, n, prec, ld_pad=0):
    import paper_2504_07637_amd as boys
    xd = torch.from_numpy(x).to("cuda")
    dt = torch.float32 if prec in ("fp32", "fp32x", "fp32s") else torch.float64
    if ld_pad:
        buf = torch.full((n + 1, x.size + ld_pad), -7.0, dtype=dt, device="cuda")
        out = buf[:, : x.size]
        boys.boys_eval(xd, n, prec, out=out)
        torch.cuda.synchronize()
        pad = buf[:, x.size:].cpu().numpy()
        assert np.all(pad == -7.0), "wrote outside the (n_max+1) x n window"
    else:
        out = boys.boys_eval(xd, n, prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _mixed_inputs(seed):
    return np.concatenate([inputs.uniform_mix(65536, seed=seed),
                           inputs.integral_args((1 << 16) + 137, seed=seed + 100),
                           _special()])


def _oracle(x, n, prec):
    if prec == "fp64":
        return orc.approx_f64(x, n)
    if prec == "fp32":
        return orc.approx_mixed(x, n)
    if prec == "fp32x":
        return orc.approx_f32x(x, n)
    if prec == "fp32s":
        return orc.approx_single(x, n)
    # the order n+1 option: the oracle's order n+1 evaluation without its top row
    return orc.approx_f64(x, n + 1)[: n + 1]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp64plus", "fp32x", "fp32s"])
def test_identical_to_the_oracle_every_nmax(prec):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = _mixed_inputs(21)
    for n in range(boys.max_nmax(prec) + 1):
        _say(f"[parity] {prec} n_max={n} count={x.size}")
        got = _gpu_eval(torch, x, n, prec)
        want = _oracle(x, n, prec)
        msg = report_mismatch(f"{prec} n_max={n}", got, want)
        assert not msg, msg


def _exp_midpoint_args(count, seed):
    # x with exp(-x) within a few binary64 ulps of a binary32 rounding midpoint (below the
    # largest binary32 cut-off): the cases where the binary32 classes' exponential must
    # tell RN32(RN64(exp(-x))) apart from a nearby rounding
    g = np.random.default_rng(seed)
    f = np.float32(np.exp(-g.uniform(0.0, 78.0, count))).astype(np.float64)
    mid = f + np.spacing(f.astype(np.float32)).astype(np.float64) / 2
    x = -np.log(mid)
    x = np.concatenate([x, np.nextafter(x, 0.0), np.nextafter(x, np.inf)])
    return x[x >= 0.0]


@pytest.mark.parametrize("prec", ["fp32", "fp32s"])
def test_binary32_exp_rounding_near_midpoints(prec):
    torch = require_gpu()
    x = _exp_midpoint_args(1 << 16, 29)
    for n in (0, 1, 4, 16, 36):
        _say(f"[midpoint] {prec} n_max={n} count={x.size}")
        got = _gpu_eval(torch, x, n, prec)
        msg = report_mismatch(f"midpoint {prec} n_max={n}", got, _oracle(x, n, prec))
        assert not msg, msg


def _bounds(table1, cls, n):
    t = table1[n][cls]
    eb0, ebn1, ebn = t["eb0"], t["ebn1"], t["ebn"]
    if ebn1 is None:
        ebn1 = eb0
    out = [min(eb0, ebn1) - 1.0] * (n + 1)
    if n >= 1:
        out[n - 1] = ebn1 - 1.0
    out[n] = ebn - 1.0
    return out


@pytest.mark.parametrize("n", [1, 4, 16, 20, 35])
def test_order_plus_one_option_error_and_gain(n, table1):
    # F_n by one recursion step from the order n+1 approximant: every m within the
    # Table 1 finite-precision bounds of row n+1 (F_n is that row's F_{n-1} column), and
    # F_n itself not less accurate than the plain order-n evaluation
    torch = require_gpu()
    r = orc.record("fp64", n + 1)
    k = 1 << 15
    x = np.concatenate([np.arange(k) * (r["z"] / k), inputs.integral_args(1 << 15, seed=33)])
    _say(f"[plus] n_max={n} count={x.size}")
    plus = _gpu_eval(torch, x, n, "fp64plus")
    base = _gpu_eval(torch, x, n, "fp64")
    hi, lo = orc.exact(x, n)
    t = table1[n + 1]["fp64"]
    bound_n = t["ebn1"] - 1.0
    bound_low = min(t["eb0"], t["ebn1"]) - 1.0
    for m in range(n + 1):
        b = orc.bits(orc.rel_err(plus[m], hi[m], lo[m]))
        assert b >= (bound_n if m == n else bound_low), (n, m, b)
    gain = (orc.bits(orc.rel_err(plus[n], hi[n], lo[n]))
            - orc.bits(orc.rel_err(base[n], hi[n], lo[n])))
    _say(f"[plus] n_max={n} F_n gain {gain:.2f} bits")
    assert gain > (1.0 if n >= 4 else -0.5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [0, 1, 4, 16, 20, 36])
def test_error_against_exact_function_within_table1(prec, n, table1):
    torch = require_gpu()
    r = orc.record(prec, n)
    k = 1 << 15
    x = np.concatenate([np.arange(k) * (r["z"] / k), inputs.integral_args(1 << 15, seed=31)])
    _say(f"[exact] {prec} n_max={n} count={x.size}")
    got = _gpu_eval(torch, x, n, prec).astype(np.float64)
    hi, lo = orc.exact(x, n)
    bounds = _bounds(table1, prec, n)
    measured = []
    for m in range(n + 1):
        e = orc.rel_err(got[m], hi[m], lo[m])
        if prec == "fp32":
            normal = np.abs(hi[m]) >= FLT_MIN
            tiny_err = np.abs(got[m][~normal] - hi[m][~normal])
            assert np.all(tiny_err <= 2.0 ** -bounds[m] * FLT_MIN + FLT_TRUE_MIN), (n, m)
            e = e[normal]
        b = orc.bits(e)
        measured.append(b)
        assert b >= bounds[m], (prec, n, m, b, bounds[m])
    _say(f"[exact] {prec} n_max={n} -log2 max rel err per m: " +
         " ".join(f"{b:.1f}" for b in measured))


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 255, 257, 4099, 100003])
def test_ragged_lengths_and_padded_rows(n):
    torch = require_gpu()
    x = inputs.integral_args(n, seed=n)
    for prec in ("fp64", "fp32", "fp64plus", "fp32x", "fp32s"):
        _say(f"[ragged] {prec} n={n}")
        got = _gpu_eval(torch, x, 7, prec, ld_pad=37)
        assert same_bits(got, _oracle(x, 7, prec)).all()


@pytest.mark.parametrize("n", [0, 1, 4, 16, 20, 36])
def test_fp32x_within_half_a_binary32_ulp_of_the_exact_function(n):
    # binary32 outputs computed in binary64 with the ~28-bit approximant: within half a
    # binary32 ulp plus 2^-27.5 relative of the exact F_m (subnormals: of FLT_MIN)
    torch = require_gpu()
    r = orc.record("fp32x", n)
    k = 1 << 15
    x = np.concatenate([np.arange(k) * (r["z"] / k), inputs.integral_args(1 << 15, seed=35)])
    _say(f"[exact] fp32x n_max={n} count={x.size}")
    got = _gpu_eval(torch, x, n, "fp32x")
    hi, lo = orc.exact(x, n)
    rounded = 0
    for m in range(n + 1):
        F = hi[m] + lo[m]
        err = np.abs(got[m].astype(np.float64) - hi[m] - lo[m])
        half_ulp = 0.5 * np.spacing(np.abs(F).astype(np.float32)).astype(np.float64)
        tol = half_ulp + 2.0 ** -27.5 * np.maximum(np.abs(F), FLT_MIN)
        assert np.all(err <= tol), (n, m, float(np.max(err / tol)))
        rounded += int(np.sum(got[m] == F.astype(np.float32)))
    _say(f"[exact] fp32x n_max={n} correctly rounded: {rounded / (x.size * (n + 1)):.5f}")


def _cutoff_straddle():
    # every binary64 cut-off, and its neighbours, for the two-approximation option
    z = np.array([orc.record("fp64", n)["z"] for n in range(37)])
    return np.concatenate([z, np.nextafter(z, np.inf), np.nextafter(z, -np.inf)])


def test_two_approximation_option_identical_every_pair():
    # every (n_max, n_bar) pair: the oracle's definition (rows 0..n_bar of the order-n_bar
    # evaluation over rows n_bar+1..n_max of the order-n_max one), bit for bit
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = np.concatenate([inputs.uniform_mix(4096, seed=61), inputs.integral_args(4096, seed=62),
                        _special(), _cutoff_straddle()])
    xd = torch.from_numpy(x).to("cuda")
    top = boys.max_nmax("fp64")
    for n in range(1, top + 1):
        _say(f"[split] n_max={n} n_bar=0..{n - 1} count={x.size}")
        plain = orc.approx_f64(x, n)
        for nbar in range(n):
            got = boys.boys_eval_split(xd, n, nbar).cpu().numpy()
            want = np.concatenate([orc.approx_f64(x, nbar), plain[nbar + 1:]], axis=0)
            msg = report_mismatch(f"split n_max={n} n_bar={nbar}", got, want)
            assert not msg, msg


@pytest.mark.parametrize("n", [1, 65, 4099, 100003])
def test_two_approximation_option_ragged_and_padded(n):
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = inputs.integral_args(n, seed=n + 7)
    xd = torch.from_numpy(x).to("cuda")
    buf = torch.full((17, n + 29), -7.0, dtype=torch.float64, device="cuda")
    boys.boys_eval_split(xd, 16, 5, out=buf[:, :n])
    torch.cuda.synchronize()
    b = buf.cpu().numpy()
    assert np.all(b[:, n:] == -7.0)
    assert same_bits(b[:, :n], orc.approx_split(x, 16, 5)).all()


def test_empty_input_is_a_noop():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = torch.empty(0, dtype=torch.float64, device="cuda")
    out = boys.boys_eval(x, 5)
    torch.cuda.synchronize()
    assert out.shape == (6, 0)


def test_full_size_integral_workload_sampled():
    # the 2^26-argument n_max = 16 workload in the launch configuration the benchmark
    # times, every class it times; the oracle checks 2^17 sampled arguments (and the
    # first and last 4096)
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    n_args = 1 << 26
    x = inputs.integral_args(n_args, seed=2)
    g = np.random.default_rng(5)
    idx = np.unique(np.concatenate([np.arange(4096), np.arange(n_args - 4096, n_args),
                                    g.integers(0, n_args, 1 << 17)]))
    xd = torch.from_numpy(x).to("cuda")
    ti = torch.from_numpy(idx).to("cuda")
    for prec in ("fp64", "fp32", "fp32x", "fp32s", "fp64plus", "split8"):
        _say(f"[full] {prec} n_max=16 count={n_args}")
        if prec == "split8":
            out = boys.boys_eval_split(xd, 16, 8)
            want = orc.approx_split(x[idx], 16, 8)
        else:
            out = boys.boys_eval(xd, 16, prec)
            want = _oracle(x[idx], 16, prec)
        torch.cuda.synchronize()
        got = out[:, ti].cpu().numpy()
        msg = report_mismatch(f"full {prec}", got, want)
        assert not msg, msg
        del out
        torch.cuda.empty_cache()


def test_full_size_properties_of_every_output():
    # every output of the 2^26-argument n_max = 16 workload, on the device, against what
    # the function itself fixes at any size: 0 <= F_m <= 1/(2m+1) (F_m(0) = 1/(2m+1) and F_m
    # decreases in x; up to the class's approximation error, 2^-40 in binary64 and 2^-12
    # in the mixed class, whose F_16 carries about 15 bits), F_{m+1} <= F_m (t^(2m+2) <=
    # t^(2m) on [0, 1]; the ratio is at most (2m+1)/(2m+3), far from 1), and, in binary64,
    # the recursion identity (2m+1) F_m = 2x F_{m+1} + exp(-x) to a relative 2^-40
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    n_args, n = 1 << 26, 16
    xd = torch.from_numpy(inputs.integral_args(n_args, seed=2)).to("cuda")
    m = torch.arange(n + 1, device="cuda", dtype=torch.float64).unsqueeze(1)
    for prec, tol in (("fp64", 2.0 ** -40), ("fp32", 2.0 ** -12)):
        _say(f"[properties] {prec} n_max={n} count={n_args}")
        F = boys.boys_eval(xd, n, prec).double()
        assert bool(torch.all(F >= 0)), prec
        assert bool(torch.all(F <= (1.0 / (2 * m + 1)) * (1 + tol))), prec
        assert bool(torch.all(F[1:] <= F[:-1])), prec
        if prec == "fp64":
            lhs = (2 * m[:-1] + 1) * F[:-1]
            rhs = 2 * xd * F[1:] + torch.exp(-xd)
            assert bool(torch.all((lhs - rhs).abs() <= 2.0 ** -40 * lhs)), prec
        del F
        torch.cuda.empty_cache()


def test_runs_on_a_side_stream():
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    x = inputs.integral_args(300001, seed=77)
    xd = torch.from_numpy(x).to("cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = boys.boys_eval(xd, 16)
    s.synchronize()
    assert same_bits(out.cpu().numpy(), orc.approx_f64(x, 16)).all()


def test_concurrent_calls_from_host_threads():
    # the entry points are reentrant: four host threads, each on a stream of its own,
    # call boys_eval repeatedly with different sizes, orders and classes; the last results
    # of each equal the oracle bit for bit
    torch = require_gpu()
    import threading
    import paper_2504_07637_amd as boys
    jobs = [(inputs.integral_args(50_000 + 777 * k, seed=300 + k), n, p)
            for k, (n, p) in enumerate([(4, "fp64"), (16, "fp32"), (36, "fp32s"), (9, "fp64plus")])]
    results, errors = [None] * len(jobs), []

    def work(k):
        try:
            x, n, p = jobs[k]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                xd = torch.from_numpy(x).to("cuda")
                outs = [boys.boys_eval(xd, n, p) for _ in range(8)]
            s.synchronize()
            results[k] = [o.cpu().numpy() for o in outs[-2:]]
        except Exception as e:  # reported below, in the test's own thread
            errors.append(e)

    _say("[threads] 4 host threads x 8 calls")
    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for (x, n, p), got in zip(jobs, results):
        want = _oracle(x, n, p)
        for g in got:
            msg = report_mismatch(f"thread {p} n_max={n}", g, want)
            assert not msg, msg


def test_arrays_longer_than_one_grid():
    # more than 2^31 arguments: the host splits the launch into grids of at most
    # INT32_MAX / block workgroups' worth; check the arguments around every split point
    # and a random sample (x drawn on the device from a seeded generator, n_max = 0)
    torch = require_gpu()
    import paper_2504_07637_amd as boys
    n = (1 << 31) + 1000
    g = torch.Generator(device="cuda")
    g.manual_seed(2024)
    xd = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 60.0
    edges = []
    for block in (128, 512):
        chunk = (2**31 - 1) // block * block
        edges += list(range(chunk - 300, min(n, chunk + 300)))
    idx = np.unique(np.concatenate([np.arange(300), np.arange(n - 300, n), edges,
                                    np.random.default_rng(3).integers(0, n, 1 << 14)]))
    ti = torch.from_numpy(idx).to("cuda")
    xs = xd[ti].cpu().numpy()
    for prec in ("fp64", "fp32"):
        _say(f"[huge] {prec} n={n} n_max=0")
        out = boys.boys_eval(xd, 0, prec)
        torch.cuda.synchronize()
        got = out[:, ti].cpu().numpy()
        want = orc.approx_f64(xs, 0) if prec == "fp64" else orc.approx_mixed(xs, 0)
        msg = report_mismatch(f"huge {prec}", got, want)
        assert not msg, msg
        del out
        torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [1, 127, 128 * 9 + 5, 128 * 17 + 3, 128 * 64 * 3 + 77])
def test_xcd_block_order_lengths(n):
    # binary64 outputs of 25+ rows take the XCD-contiguous block order: grids below 8
    # blocks, grids that are not a multiple of 8 and a few hundred blocks, every row checked
    torch = require_gpu()
    x = np.concatenate([inputs.integral_args(n, seed=n + 3)[: max(0, n - 3)], [0.0, 80.0, 1e4]])[:n]
    for prec, nm in (("fp64", 24), ("fp64", 36), ("fp64plus", 30)):
        _say(f"[xcd] {prec} n_max={nm} n={n}")
        got = _gpu_eval(torch, x, nm, prec, ld_pad=19)
        msg = report_mismatch(f"xcd {prec} n_max={nm} n={n}", got, _oracle(x, nm, prec))
        assert not msg, msg
    import paper_2504_07637_amd as boys
    xd = torch.from_numpy(x).to("cuda")
    got = boys.boys_eval_split(xd, 30, 12).cpu().numpy()
    assert same_bits(got, orc.approx_split(x, 30, 12)).all()
