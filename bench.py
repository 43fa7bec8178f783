"""Benchmark: Boys-function values per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one boys_eval call over the 2^26-argument integral workload (x = rho |PQ|^2,
1% exact zeros) at n_max = 16: F_0..F_16 for every argument, binary64 (the headline) and
the mixed binary32 class (reported beside it, with its speed-up).  Inputs are resident in
HBM before the timed region.  Rank 0 prints one JSON line.

Besides the headline the line carries:
  roofline      HBM roofline of the dominant kernel (the binary64 n_max=16 kernel):
                algorithmic bytes per launch (8 B read + 17 x 8 B written per argument)
                over its average launch time from HIP events on the launch stream;
                traffic from the committed rocprofv3 counter summary when it matches
                the current kernel source, else null;
  store_reduced a diagnostic, not the headline: the same arguments and n_max = 16
                arithmetic through boys_eval_rows storing only F_0 and F_16 (24 B per
                argument), which shows the arithmetic against the VALU roofline;
  cpu_baseline  the CPU oracle's binary64 evaluation of the same approximant (built
                -O3 -march=native for this host) on a bounded prefix of the same
                workload, on this host's cores;
  accuracy      -log2 of the largest relative error per class against the exact
                oracle on 2^13 sampled arguments (every m);
  latency       p50/p99 of single calls on the small 65,536-argument workload
                (n_max = 4, binary64);
  batched       the 8,192-array workload: the autotuned plan and the persistent
                one-launch plan, each labelled with its launch structure, against a
                roofline combined from every array's bytes and VALU work;
  serving       p50/p99 request latency and sustained values/s of the serving loop
                under Poisson arrivals at 20,000 requests/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

N_ARGS = 1 << 26
N_MAX = 16
SR_ROWS = [0, N_MAX]   # the store-reduced diagnostic keeps F_0 and F_16
SPLIT_NBAR = 8   # the two-approximation option: rows 0..8 from the order-8 approximant
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6   # MI355X binary64 vector peak (an fma counts 2)
# VALU issue capacity: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at
# 2.4 GHz (the same figure as the 78.6 TFLOP/s binary64 peak: 1024 x 16 lanes x 2 x 2.4e9)
VALU_WAVE_INSTR_PER_S = 1024 * 2.4e9 / 4
VALU_TABLE_FILE = os.path.join(REPO, "profiles", "valu_per_order_integral.json")
TRAFFIC_FILE = os.path.join(REPO, "profiles", "traffic_boys_f64_n16.json")
_CSRC = os.path.join(REPO, "paper_2504_07637_amd", "csrc")
# the sources each kernel family is built from: counters taken on one family stay valid
# while these files' code is unchanged
KERNEL_SOURCES = {
    "plain": ("boys_device.h", "boys_kernels.h", "plain_inst.hip", "boys_tables.inc"),
    "eri": ("boys_device.h", "boys_kernels.h", "boys_eri.h", "eri_inst.hip", "boys_tables.inc"),
    "batched": ("boys_device.h", "boys_kernels.h", "boys_batched.h", "batched_inst.hip",
                "boys_tables.inc"),
}


def kernel_hash(family: str = "plain") -> str:
    """Hash of the code of a kernel family's sources: // comments and blank lines do not
    count."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(_CSRC, f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target length of the CPU-baseline sample")
    ap.add_argument("--skip-extras", action="store_true",
                    help="only the headline (for profiling runs)")
    ap.add_argument("--workload", choices=("boys", "eri", "eri-sides", "valu-table", "batched"),
                    default="boys",
                    help="boys: the headline bulk evaluation (default); eri: the consumer "
                         "kernel on its own (contracted (ss|ss)^(m) integrals); valu-table: "
                         "one plain launch per (class, n_max), binary64 and mixed, n_max "
                         "0..16, on 2^22 integral arguments (for per-order VALU counters); "
                         "batched: the 8,192-array batch with two fixed plans, one workgroup "
                         "per 1024-argument tile and the persistent schedule (for traces "
                         "and counters of the batched kernels); eri-sides: the consumer on "
                         "the benchmark's lists moved so that every quartet lies below the "
                         "cut-off, then past it (for per-side VALU counters)")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first run one elementwise kernel over 1 GiB (1 GiB read, 1 GiB "
                         "written), a dispatch of known traffic for scaling rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE")
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3


def cpu_model():
    """The host CPU as lscpu reports it (model name, sockets, cores), else /proc/cpuinfo."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        info = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
        keys = ("Model name", "Vendor ID", "CPU family", "Model", "Socket(s)",
                "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
        got = {k: info[k] for k in keys if k in info}
        if got:
            return got
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return {"Model name": line.split(":", 1)[1].strip()}
    except OSError:
        pass
    return None


def cpu_baseline(x, target_s):
    from oracle import oracle as orc
    os.environ.setdefault("OMP_NUM_THREADS", str(len(os.sched_getaffinity(0))))
    threads = int(os.environ["OMP_NUM_THREADS"])  # what the oracle's OpenMP loops use
    orc.use_native_build()   # the same C source at -O3 -march=native for this host
    n = 1 << 18
    while True:
        t0 = time.perf_counter()
        orc.approx_f64(x[:n], N_MAX)
        dt = time.perf_counter() - t0
        if dt * 4 > target_s or n * 4 > x.size:
            break
        n *= 4
    # the oracle's exp(-x) is binary128 expq, rounded once, taken for the arguments at or
    # below the cut-off (past it the long-range limit needs none): its share of the time
    xs = x[:n]
    below = np.ascontiguousarray(xs[~(xs > orc.record("fp64", N_MAX)["z"])])
    t0 = time.perf_counter()
    orc.exp_neg(below)
    dtx = time.perf_counter() - t0
    ne = 1 << 14
    t0 = time.perf_counter()
    orc.exact(x[:ne], N_MAX)
    dte = time.perf_counter() - t0
    return {"value": (N_MAX + 1) * n / dt, "unit": "values/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "build": "gcc -O3 -march=native -fopenmp -ffp-contract=off (schedule static)",
            "sample": f"first {n} arguments of the same 2^26 workload, n_max=16, binary64 "
                      f"approximant oracle (plain C, OpenMP, {dt:.2f} s)",
            "expq_seconds": round(dtx, 3), "expq_share": round(dtx / dt, 3),
            "expq_arguments": int(below.size),
            "expq_note": "the oracle takes exp(-x) as binary128 expq rounded to binary64 "
                         "(correct rounding by construction) for every argument at or below "
                         "the cut-off; those exponentials alone are expq_share of its time, so "
                         "this is no tuned CPU code",
            "exact_oracle_values_per_s": (N_MAX + 1) * ne / dte,
            "exact_oracle_sample": f"first {ne} arguments, F_0..F_16 from the definition in "
                                   f"binary128 (OpenMP, {dte:.2f} s)"}


def accuracy(torch, boys, xd, x):
    from oracle import oracle as orc
    g = np.random.default_rng(17)
    idx = np.sort(g.choice(x.size, 1 << 13, replace=False))
    ti = torch.from_numpy(idx).to(xd.device)
    out = {}
    hi, lo = orc.exact(x[idx], N_MAX)
    for prec in ("fp64", "fp32", "fp32x", "fp32s", "fp64_split8"):
        if prec == "fp64_split8":
            F = boys.boys_eval_split(xd, N_MAX, SPLIT_NBAR)[:, ti].cpu().numpy()
        else:
            F = boys.boys_eval(xd, N_MAX, prec)[:, ti].double().cpu().numpy()
        per_m = []
        for m in range(N_MAX + 1):
            ok = np.abs(hi[m]) >= 1.1754943508222875e-38
            e = orc.rel_err(F[m][ok], hi[m][ok], lo[m][ok])
            per_m.append(round(float(orc.bits(e)), 2))
        out[prec] = {"bits_per_m": per_m, "min_bits": min(per_m)}
        del F
    return out


def latency(torch, boys, inputs):
    x = torch.from_numpy(inputs.uniform_mix(65536, seed=1)).to("cuda")
    out = torch.empty((5, x.numel()), dtype=torch.float64, device="cuda")
    for _ in range(20):
        boys.boys_eval(x, 4, "fp64", out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(1000):
        t0 = time.perf_counter()
        boys.boys_eval(x, 4, "fp64", out=out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts = np.array(ts) * 1e6
    plan = boys.Plan([x], [4], ["fp64"], outs=[out])
    for _ in range(20):
        plan.execute()
    torch.cuda.synchronize()
    tg = []
    for _ in range(1000):
        t0 = time.perf_counter()
        plan.execute()
        torch.cuda.synchronize()
        tg.append(time.perf_counter() - t0)
    plan.close()
    tg = np.array(tg) * 1e6
    # the same arguments in sorted order: every wave on one side of the cut-off
    xs = torch.sort(x).values
    for _ in range(20):
        boys.boys_eval(xs, 4, "fp64", out=out)
    torch.cuda.synchronize()
    tb = []
    for _ in range(1000):
        t0 = time.perf_counter()
        boys.boys_eval(xs, 4, "fp64", out=out)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    tb = np.array(tb) * 1e6
    return {"workload": "65,536 arguments (1/4 zeros, U[0,1], logU[1,50], logU[50,1e4]), "
                        "n_max=4, binary64, call+synchronize, 1000 calls",
            "sorted_p50_us": round(float(np.percentile(tb, 50)), 2),
            "sorted_p99_us": round(float(np.percentile(tb, 99)), 2),
            "p50_us": round(float(np.percentile(ts, 50)), 2),
            "p99_us": round(float(np.percentile(ts, 99)), 2),
            "graph_p50_us": round(float(np.percentile(tg, 50)), 2),
            "graph_p99_us": round(float(np.percentile(tg, 99)), 2)}


def describe_plan(t):
    """The launch structure a tuning gives (boys_tuning in include/boys.h)."""
    if t.get("schedule") == 0:
        return (f"one persistent launch in the plan's graph (after a one-wave kernel that "
                f"zeroes its counters): {t.get('grid_per_cu')} workgroups of {t.get('block')} "
                f"threads per CU, each wave taking 256-argument tiles from one of 8 work "
                f"counters and loading the next tile's arguments before storing")
    if t.get("schedule") == 1:
        return (f"one launch in the plan's graph: one {t.get('block')}-thread workgroup per "
                f"{t.get('tile')}-argument tile")
    if t.get("split_nmax"):
        return (f"two launches in the plan's graph: the store-bound arrays (n_max >= "
                f"{t['split_nmax']} binary64, >= {t['split_nmax'] + 4} binary32) one "
                f"256-thread workgroup per 256-argument tile, then the rest one wave per "
                f"256-argument tile ({t.get('block')}-thread workgroups)")
    return (f"one launch in the plan's graph: one wave per 256-argument tile "
            f"({t.get('block')}-thread workgroups)")


def valu_table():
    """Per-(class, n_max) VALU wave instructions per argument on the integral workload,
    from the committed counter run, if the kernels have not changed since."""
    try:
        with open(VALU_TABLE_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    return d if d.get("kernel_hash") == kernel_hash() else None


def batch_roofline(plan_spec, ms):
    """Rooflines of the batch from every array's algorithmic bytes and VALU work (VALU
    wave instructions per argument of its (class, n_max) by counters):
      overlapped  max(sum bytes / 8 TB/s, sum VALU / issue capacity): arrays overlap on
                  the device, so no launch can beat this;
      per_array   sum over arrays of max(bytes / 8 TB/s, VALU / issue capacity): every
                  array at its own roofline, one after another."""
    tab = valu_table()
    if tab is None:
        return None
    per = tab["wave_instructions_per_argument"]
    tb = tv = tpa = 0.0
    for l, m, p in plan_spec:
        cls = "fp64" if p == 0 else "fp32"
        byt = l * (8 + (m + 1) * (8 if p == 0 else 4))
        wi = l * per[cls][m]
        tb += byt / (PEAK_HBM_GBS * 1e9)
        tv += wi / VALU_WAVE_INSTR_PER_S
        tpa += max(byt / (PEAK_HBM_GBS * 1e9), wi / VALU_WAVE_INSTR_PER_S)
    ov = max(tb, tv)
    return {"hbm_ms": tb * 1e3, "valu_ms": tv * 1e3, "overlapped_bound_ms": ov * 1e3,
            "per_array_bound_ms": tpa * 1e3, "frac_of_overlapped": ov * 1e3 / ms,
            "frac_of_per_array": tpa * 1e3 / ms,
            "source": "algorithmic bytes; VALU wave instructions per argument per (class, "
                      "n_max) from rocprofv3 counters (" + os.path.basename(VALU_TABLE_FILE) +
                      "), issue capacity 1024 SIMDs x 2.4 GHz / 4 cycles"}


PERSISTENT_SWEEP = [{"schedule": 0, "tile": 256, "block": b, "grid_per_cu": g, "order": 1}
                    for b, g in ((256, 2), (256, 4), (256, 6), (256, 8), (128, 8), (64, 16))]


def batched(torch, boys, inputs, steps):
    plan_spec = inputs.batch_plan(8192, seed=4)
    total = sum(l for l, _, _ in plan_spec)
    xall = torch.from_numpy(inputs.integral_args(total, seed=4)).to("cuda")
    xs, off = [], 0
    for l, _, _ in plan_spec:
        xs.append(xall[off:off + l])
        off += l
    nm = [m for _, m, _ in plan_spec]
    pr = ["fp64" if p == 0 else "fp32" for _, _, p in plan_spec]
    from paper_2504_07637_amd import tuning
    best, info = tuning.tuned(xs, nm, pr)
    plan = boys.Plan(xs, nm, pr, tuning=best)
    # a fresh plan runs slower for its first replays (the tuner warms each candidate up 12
    # times): 25 warm-up replays before the timed ones
    wall, gpu = timed(torch, plan.execute, steps, 25)
    values = sum(l * (m + 1) for l, m, _ in plan_spec)
    bytes_ = sum(l * (8 + (m + 1) * (8 if p == 0 else 4)) for l, m, p in plan_spec)
    ms = gpu / steps * 1e3
    # the persistent one-launch schedule over the same arrays and outputs, swept
    pers = {}
    for t in PERSISTENT_SWEEP:
        pp = boys.Plan(xs, nm, pr, tuning=t, outs=plan.outs)
        _, g = timed(torch, pp.execute, steps, 25)
        pers[json.dumps(t, sort_keys=True)] = round(g / steps * 1e3, 4)
        pp.close()
    pbest = min(pers, key=pers.get)
    # the same arrays as 8,192 separate boys_eval calls into the plan's outputs
    solo = lambda: [boys.boys_eval(xi, m, p, out=o) for xi, m, p, o in zip(xs, nm, pr, plan.outs)]
    solo_wall, solo_gpu = timed(torch, solo, 2, 1)
    # the same arguments grouped by (class, n_max), one plain launch per group: the plain
    # kernels' time for this work, without per-array call overhead
    groups = {}
    for xi, m, p in zip(xs, nm, pr):
        groups.setdefault((p, m), []).append(xi)
    gx = [(torch.cat(v), m, p) for (p, m), v in sorted(groups.items())]
    go = [boys.empty_out(xg.numel(), m, p) for xg, m, p in gx]
    grouped = lambda: [boys.boys_eval(xg, m, p, out=o) for (xg, m, p), o in zip(gx, go)]
    grp_wall, grp_gpu = timed(torch, grouped, steps, 3)
    del gx, go
    res = {"workload": "8,192 arrays, lengths logU[32,65536], n_max U{0..16}, "
                       "binary64/binary32 alternating",
           "plan": describe_plan(best),
           "arguments": total, "ms": round(ms, 4), "values_per_s": values / (gpu / steps),
           "hbm_GBs": bytes_ / (ms * 1e-3) / 1e9, "tuning": best,
           "roofline": batch_roofline(plan_spec, ms),
           "persistent": {"plan": describe_plan(json.loads(pbest)), "ms": pers[pbest],
                          "values_per_s": values / (pers[pbest] * 1e-3),
                          "tuning": json.loads(pbest), "sweep_ms": pers,
                          "roofline": batch_roofline(plan_spec, pers[pbest])},
           "solo_calls_ms": round(solo_gpu / 2 * 1e3, 3),
           "batching_gain": round(solo_gpu / 2 / (gpu / steps), 2),
           "grouped_plain_ms": round(grp_gpu / steps * 1e3, 4),
           "grouped_plain_launches": len(groups),
           "tuning_cached": info["cached"],
           "candidates_ms": {k: round(v, 4) for k, v in info["times_ms"].items()}}
    plan.close()
    return res


BATCH_FIXED = {"workgroup_tile": {"schedule": 1, "block": 256, "tile": 1024, "grid_per_cu": 1,
                                   "order": 1},
               "persistent": {"schedule": 0, "block": 256, "tile": 256, "grid_per_cu": 4,
                              "order": 1}}


def batched_fixed(torch, boys, inputs, steps, warmup):
    """The 8,192-array batch with fixed plans (no tuner), each timed on its own, for
    profiling runs: algorithmic bytes per replay beside the HIP-event time."""
    plan_spec = inputs.batch_plan(8192, seed=4)
    total = sum(l for l, _, _ in plan_spec)
    xall = torch.from_numpy(inputs.integral_args(total, seed=4)).to("cuda")
    xs, off = [], 0
    for l, _, _ in plan_spec:
        xs.append(xall[off:off + l])
        off += l
    nm = [m for _, m, _ in plan_spec]
    pr = ["fp64" if p == 0 else "fp32" for _, _, p in plan_spec]
    bytes_ = sum(l * (8 + (m + 1) * (8 if p == 0 else 4)) for l, m, p in plan_spec)
    res = {"workload": "8,192 arrays, lengths logU[32,65536], n_max U{0..16}, "
                       "binary64/binary32 alternating", "arguments": total,
           "alg_bytes_per_replay": bytes_}
    outs = None
    for name, t in BATCH_FIXED.items():
        plan = boys.Plan(xs, nm, pr, tuning=t, outs=outs)
        outs = plan.outs
        _, g = timed(torch, plan.execute, steps, warmup)
        res[name] = {"tuning": t, "plan": describe_plan(t), "ms": g / steps * 1e3,
                     "hbm_GBs": bytes_ / (g / steps) / 1e9}
        plan.close()
    return res


ERI_PAIRS = 2048   # contracted shell pairs on each side (9 primitive pairs each)
ERI_FLOPS_FILE = os.path.join(REPO, "profiles", "flops_eri_ssss_n16.json")


VALU_WAVE_ISSUE_PER_S = 1024 * 2.4e9 / 4  # 1024 SIMDs, one wave64 instruction per 4 cycles


def below_fraction(pairs, z):
    """The share of the primitive quartets of a pair list with itself whose argument
    T = rho |P - Q|^2 lies below the cut-off z (not T > z), formed with the kernel's
    operations in the kernel's order, so the classification is the kernel's."""
    p, px, py, pz = pairs[0], pairs[1], pairs[2], pairs[3]
    below = 0
    for a0 in range(0, p.size, 256):
        a = slice(a0, a0 + 256)
        pq = p[a, None] * p[None, :]
        spq = p[a, None] + p[None, :]
        rho = pq / spq
        dx = px[a, None] - px[None, :]
        dy = py[a, None] - py[None, :]
        dz = pz[a, None] - pz[None, :]
        T = rho * (dx * dx + dy * dy + dz * dz)
        below += int(np.count_nonzero(~(T > z)))
    return below / float(p.size) ** 2


def one_side_lists(inputs, side):
    """The benchmark's pair list with every product centre moved so that every primitive
    quartet lies on one side of the cut-off at n_max = 16 (z = 74.5): the bra pairs at the
    origin, the ket pairs 0.03 bohr away for 'below' (T = rho 9e-4 spans 5e-5 .. 41) or 1000
    bohr away for 'past' (T >= 6e4)."""
    c, e, w = inputs.s_basis()
    pairs, start = inputs.shell_pairs(c, e, w, max_pairs=ERI_PAIRS)
    bra = pairs.copy()
    bra[1:4] = 0.0
    ket = bra.copy()
    ket[1] = 0.03 if side == "below" else 1000.0
    return bra, ket, start


def eri(torch, boys, inputs, steps, warmup):
    """The consumer: contracted (ss|ss)^(m), m = 0..16, over ERI_PAIRS^2 contracted pairs."""
    c, e, w = inputs.s_basis()
    pairs, start = inputs.shell_pairs(c, e, w, max_pairs=ERI_PAIRS)
    P = torch.from_numpy(pairs).to("cuda")
    S = torch.from_numpy(start).to("cuda")
    nc = start.size - 1
    out = boys.empty_out(nc * nc, N_MAX, "fp64")
    wall, gpu = timed(torch, lambda: boys.boys_eri_ssss(P, S, P, S, N_MAX, out=out), steps,
                      warmup)
    launch_s = gpu / steps
    prim = float(pairs.shape[1]) ** 2
    res = {"workload": f"contracted (ss|ss)^(m), m = 0..{N_MAX}: {nc} x {nc} contracted pairs "
                       f"of an s basis (32 atoms, 8 shells of 3 primitives each), "
                       f"{int(prim)} primitive quartets, x = rho|PQ|^2 formed on the device",
           "launch_ms": launch_s * 1e3, "ms_per_step": wall / steps * 1e3,
           "quartets_per_s": nc * nc / launch_s,
           "boys_evaluations_per_s": prim / launch_s,
           "values_consumed_per_s": prim * (N_MAX + 1) / launch_s,
           "bytes_stored_per_launch": 8 * (N_MAX + 1) * nc * nc}
    fb = below_fraction(pairs, boys.cutoff(N_MAX, "fp64"))
    res["below_cutoff_fraction"] = fb
    prof = eri_profile(kernel_hash("eri"))
    if prof is not None:
        fl = prof["flops_per_launch"]
        res["roofline"] = {"bound": "alu", "achieved": fl / launch_s / 1e12,
                           "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                           "frac": fl / launch_s / 1e12 / PEAK_FP64_TFLOPS,
                           "flops_per_launch": fl, "kernel": f"k_eri_ssss<{N_MAX}>",
                           "source": "executed binary64 VALU operations by counters"}
        sides = prof.get("lane_instructions_per_quartet_by_side")
        if sides is not None:
            # the instructions the quartets need on their own sides of the cut-off (each
            # side's count measured on a list with every quartet on that side), against the
            # VALU issue capacity: what a divergence-free execution would issue
            useful = fb * sides["below"] + (1.0 - fb) * sides["past"]
            achieved = useful * prim / 64.0 / launch_s
            res["roofline"]["valu_issue"] = {
                "useful_lane_instructions_per_quartet": useful,
                "lane_instructions_per_quartet_by_side": sides,
                "achieved_wave_instructions_per_s": achieved,
                "peak_wave_instructions_per_s": VALU_WAVE_ISSUE_PER_S,
                "frac": achieved / VALU_WAVE_ISSUE_PER_S,
                "executed_lane_instructions_per_quartet":
                    prof.get("executed_lane_instructions_per_quartet")}
    return res


def eri_sides(torch, boys, inputs):
    """For counter runs: the consumer at n_max = 16 on the benchmark's lists with every
    quartet below the cut-off, then with every quartet past it (two launches each)."""
    out = None
    for side in ("below", "past"):
        bra, ket, start = one_side_lists(inputs, side)
        S = torch.from_numpy(start).to("cuda")
        B = torch.from_numpy(bra).to("cuda")
        K = torch.from_numpy(ket).to("cuda")
        nc = start.size - 1
        if out is None:
            out = boys.empty_out(nc * nc, N_MAX, "fp64")
        for _ in range(2):
            boys.boys_eri_ssss(B, S, K, S, N_MAX, out=out)
        torch.cuda.synchronize()
    return {"eri_sides": "below then past, two launches each",
            "quartets_per_launch": float(bra.shape[1]) ** 2}


def eri_profile(hash_now):
    """The consumer's counter figures (executed binary64 FLOPs per launch, VALU lane
    instructions per quartet), if the kernels have not changed since they were taken."""
    try:
        with open(ERI_FLOPS_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    return d if d.get("kernel_hash") == hash_now and "flops_per_launch" in d else None


def serving(torch, duration=10.0):
    from paper_2504_07637_amd import inputs
    from paper_2504_07637_amd import serving as srv_mod
    pool = srv_mod.argument_pool(1 << 24, seed=5)
    warm = inputs.serving_requests(rate=20000.0, duration=1.0, seed=50)
    reqs = inputs.serving_requests(rate=20000.0, duration=duration, seed=5)
    with srv_mod.Server(budget_bytes=8 << 30, streams=4) as srv:
        srv_mod.run_poisson(srv, warm, pool)   # 1 s warm-up, not reported
        res = srv_mod.run_poisson(srv, reqs, pool)
        st = srv.stats()
    out = srv_mod.summarize(res)
    out["max_admitted_bytes"] = st["max_bytes_in_use"]
    out["workload"] = ("Poisson 20,000 requests/s, lengths logU[64,262144], n_max U{0..20}, "
                       "binary64/binary32 50/50, integral-workload arguments, 8 GiB budget, "
                       f"{duration:.0f} s of steady state after a 1 s warm-up; latency = "
                       "completion - submission, host-to-device copies included")
    return out


TRACE_FILE = os.path.join(REPO, "profiles", "k_plain_n16_integral_2p26_kernel_trace.json")


def trace_for(hash_now, kernel):
    """The committed kernel trace's timed mean launch time of a plain kernel (ms), while
    the sources match the ones it was taken on."""
    try:
        with open(TRACE_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    k = (t.get("kernels") or {}).get(kernel)
    if t.get("kernel_hash") != hash_now or not k:
        return None
    return k["mean"]


def traffic_for(hash_now):
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != hash_now:
        return None
    return t.get("bytes_per_launch")


def valu_for(hash_now, kernel, launch_s):
    """The kernel's VALU use by counters (same profile file), while the sources match:
    issue fraction of the 4-cycle capacity, VALUBusy, and executed binary64 FLOP/s
    against the binary64 vector peak."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    v = (t.get("valu") or {}).get(kernel)
    if t.get("kernel_hash") != hash_now or not v:
        return None
    tf = v["fp64_flops"] / launch_s / 1e12
    return {"issue_fraction": v["issue_fraction_4cycle"], "valu_busy": v["valu_busy"],
            "lane_instructions_per_argument": v["valu_wave_instructions"] * 64 / N_ARGS,
            "fp64_tflops": tf, "fp64_peak_tflops": PEAK_FP64_TFLOPS,
            "fp64_frac": tf / PEAK_FP64_TFLOPS}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the path has no "
                                   "cross-GPU step (arguments are independent)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import paper_2504_07637_amd as boys
    from paper_2504_07637_amd import inputs

    if args.pmc_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del a, b
    if args.workload == "eri":
        r = eri(torch, boys, inputs, args.steps, args.warmup)
        line = {"metric": "contracted (ss|ss)^(m) integrals/s at n_max=16 (consumer)",
                "value": r["quartets_per_s"], "unit": "quartets/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f64", "data": "synthetic", "config": {"workload": r["workload"]}}
        line.update({k: v for k, v in r.items() if k not in line and k != "workload"})
        print(json.dumps(line), flush=True)
        return
    if args.workload == "eri-sides":
        print(json.dumps(eri_sides(torch, boys, inputs)), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(batched_fixed(torch, boys, inputs, args.steps, args.warmup)),
              flush=True)
        return
    if args.workload == "valu-table":
        # one plain launch per (class, n_max): the per-order VALU counters of the batch's
        # combined roofline are read per dispatch from a rocprofv3 --pmc run of this mode
        xt = torch.from_numpy(inputs.integral_args(1 << 22, seed=4)).to("cuda")
        for prec in ("fp64", "fp32"):
            for m in range(N_MAX + 1):
                boys.boys_eval(xt, m, prec)
                torch.cuda.synchronize()
        print(json.dumps({"valu_table": "fp64 then fp32, n_max 0..16, 2^22 integral "
                                        "arguments, one launch each"}), flush=True)
        return
    x = inputs.integral_args(N_ARGS, seed=2)
    xd = torch.from_numpy(x).to("cuda")
    out64 = torch.empty((N_MAX + 1, N_ARGS), dtype=torch.float64, device="cuda")
    out32 = torch.empty((N_MAX + 1, N_ARGS), dtype=torch.float32, device="cuda")

    wall64, gpu64 = timed(torch, lambda: boys.boys_eval(xd, N_MAX, "fp64", out=out64),
                          args.steps, args.warmup)
    wall32, gpu32 = timed(torch, lambda: boys.boys_eval(xd, N_MAX, "fp32", out=out32),
                          args.steps, args.warmup)
    wall32x, gpu32x = timed(torch, lambda: boys.boys_eval(xd, N_MAX, "fp32x", out=out32),
                            args.steps, args.warmup)
    wall32s, gpu32s = timed(torch, lambda: boys.boys_eval(xd, N_MAX, "fp32s", out=out32),
                            args.steps, args.warmup)
    wall_sp, gpu_sp = timed(torch, lambda: boys.boys_eval_split(xd, N_MAX, SPLIT_NBAR, out=out64),
                            args.steps, args.warmup)
    # the store-reduced diagnostic: the same evaluation, only F_0 and F_16 stored
    sr = {}
    for prec, dt, es in (("fp64", torch.float64, 8), ("fp32", torch.float32, 4)):
        o = torch.empty((len(SR_ROWS), N_ARGS), dtype=dt, device="cuda")
        _, g = timed(torch, lambda: boys.boys_eval_rows(xd, N_MAX, SR_ROWS, prec, out=o),
                     args.steps, args.warmup)
        sr[prec] = (g / args.steps, (8 + es * len(SR_ROWS)) * N_ARGS)
        del o
    values = (N_MAX + 1) * N_ARGS
    ms64 = wall64 / args.steps * 1e3
    v64 = values * args.steps / wall64
    v32 = values * args.steps / wall32
    launch_s = gpu64 / args.steps
    alg_bytes = (8 + 8 * (N_MAX + 1)) * N_ARGS
    achieved = alg_bytes / launch_s / 1e9
    khash = kernel_hash()
    res = {
        "metric": "F_m(x) values/s at n_max=16 FP64 vs FP32 (at stated err); p50/p99 latency",
        "value": v64,
        "unit": "values/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "integral-argument Boys evaluation: 2^26 x = rho|PQ|^2 "
                               "(a,b logU[0.05,5e4], PQ ~ N(0, 2.0^2 I3), 1% zeros), "
                               "F_0..F_16 binary64 SoA",
                   "n_args": N_ARGS, "n_max": N_MAX},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for(khash),
                     "valu": valu_for(khash, "k_plain<0, 16, false>", launch_s),
                     "kernel": "k_plain<FP64,16>", "launch_ms": launch_s * 1e3,
                     "alg_bytes_per_launch": alg_bytes, "kernel_hash": khash},
        "fp32": {"value": v32, "unit": "values/s", "ms_per_step": wall32 / args.steps * 1e3,
                 "class": "mixed: u/v, Q~, W and the recursion in binary32, x + W and "
                          "c_n/G^(n+1/2) in binary64; exp(-x) and the past-cut-off chain "
                          "(long-range limit) are also evaluated in binary64 and rounded to "
                          "binary32, beyond a strict reading of binary64 for the power only",
                 "speedup_vs_fp64": v32 / v64,
                 "launch_ms": gpu32 / args.steps * 1e3,
                 "hbm_GBs": (8 + 4 * (N_MAX + 1)) * N_ARGS / (gpu32 / args.steps) / 1e9},
        "fp64_split8": {"value": values * args.steps / wall_sp, "unit": "values/s",
                        "n_bar": SPLIT_NBAR, "ms_per_step": wall_sp / args.steps * 1e3,
                        "launch_ms": gpu_sp / args.steps * 1e3,
                        "hbm_GBs": alg_bytes / (gpu_sp / args.steps) / 1e9},
        "fp32x": {"value": values * args.steps / wall32x, "unit": "values/s",
                  "ms_per_step": wall32x / args.steps * 1e3,
                  "speedup_vs_fp64": wall64 / wall32x,
                  "launch_ms": gpu32x / args.steps * 1e3,
                  "hbm_GBs": (8 + 4 * (N_MAX + 1)) * N_ARGS / (gpu32x / args.steps) / 1e9},
        "fp32s": {"value": values * args.steps / wall32s, "unit": "values/s",
                  "ms_per_step": wall32s / args.steps * 1e3,
                  "speedup_vs_fp64": wall64 / wall32s,
                  "launch_ms": gpu32s / args.steps * 1e3,
                  "hbm_GBs": (8 + 4 * (N_MAX + 1)) * N_ARGS / (gpu32s / args.steps) / 1e9},
    }
    res["store_reduced"] = {
        "kind": "diagnostic, not the headline: the same 2^26 arguments and n_max = 16 "
                "arithmetic (boys_eval_rows), only F_0 and F_16 stored",
        "rows": SR_ROWS}
    for prec, (t, byt) in sr.items():
        kern = f"k_plain<{0 if prec == 'fp64' else 1}, {N_MAX}, true>"
        res["store_reduced"][prec] = {
            "launch_ms": t * 1e3, "arguments_per_s": N_ARGS / t,
            "alg_bytes_per_launch": byt, "hbm_GBs": byt / t / 1e9,
            "hbm_frac": byt / t / 1e9 / PEAK_HBM_GBS,
            "speedup_vs_full_store": (gpu64 if prec == "fp64" else gpu32) / args.steps / t,
            "kernel": kern, "valu": valu_for(khash, kern, t)}
    # measured HBM figures on this device: one write stream (fill) and a read+write copy
    wall_f, gpu_f = timed(torch, lambda: out64.fill_(1.0), 5, 2)
    fill_GBs = out64.numel() * 8 / (gpu_f / 5) / 1e9
    src = out64[:8].reshape(-1)
    dst = out32[:16].view(torch.float64).reshape(-1)
    wall_c, gpu_c = timed(torch, lambda: dst.copy_(src), 5, 2)
    copy_GBs = 2 * src.numel() * 8 / (gpu_c / 5) / 1e9
    tr = trace_for(khash, "k_plain<0, 16, false>")
    if tr is not None:
        # the same figure from the committed rocprofv3 kernel trace (timed dispatches)
        res["roofline"]["trace_launch_ms"] = tr
        res["roofline"]["trace_frac"] = alg_bytes / (tr * 1e-3) / 1e9 / PEAK_HBM_GBS
    res["roofline"]["measured_fill_GBs"] = fill_GBs
    res["roofline"]["measured_copy_GBs"] = copy_GBs
    res["roofline"]["frac_of_measured_fill"] = achieved / fill_GBs
    del out32
    torch.cuda.empty_cache()
    progress(f"headline {ms64:.3f} ms per step")
    if not args.skip_extras:
        res["accuracy"] = accuracy(torch, boys, xd, x)
        progress("accuracy done")
        del out64
        torch.cuda.empty_cache()
        res["latency"] = latency(torch, boys, inputs)
        progress("latency done")
        res["batched"] = batched(torch, boys, inputs, max(30, args.steps))
        progress("batched done")
        res["serving"] = serving(torch)
        progress("serving done")
        res["eri"] = eri(torch, boys, inputs, max(3, args.steps // 2), 2)
        progress("consumer done")
        res["cpu_baseline"] = cpu_baseline(x, args.cpu_seconds)
        progress("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
