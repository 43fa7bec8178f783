"""Host-side logic of the Python binding and the benchmark (no device calls)."""
import json
import os
import re
import subprocess
import sys
import types

import pytest

import paper_2504_07637_amd as boys
from paper_2504_07637_amd import _lib

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_precision_names():
    for names, code in ((("fp64", "float64", "double", 0), _lib.FP64),
                        (("fp32", "float32", "mixed", 1), _lib.FP32),
                        (("fp64plus", "fp64+", 2), _lib.FP64_PLUS),
                        (("fp32x", 3), _lib.FP32X),
                        (("fp32s", "single", 4), _lib.FP32S)):
        for nm in names:
            assert boys.precision_code(nm) == code
    for bad in ("fp16", 5, -1, None):
        with pytest.raises(ValueError):
            boys.precision_code(bad)


def test_padded_row_stride_is_whole_cache_lines():
    for n in (0, 1, 15, 16, 17, 31, 33, 1000, 65536):
        for prec, es in (("fp64", 8), ("fp64plus", 8), ("fp32", 4), ("fp32x", 4), ("fp32s", 4)):
            ld = boys.padded_ld(n, prec)
            assert ld >= max(n, 1) and (ld * es) % 128 == 0 and ld * es - n * es < 128 + 128


def test_device_guard_switches_only_when_needed(monkeypatch):
    calls = []

    class FakeCuda:
        cur = 0
        count = 4

        @staticmethod
        def current_device():
            return FakeCuda.cur

        @staticmethod
        def set_device(d):
            calls.append(d)
            FakeCuda.cur = d

        @staticmethod
        def device_count():
            return FakeCuda.count

    monkeypatch.setattr(boys, "_torch", lambda: types.SimpleNamespace(cuda=FakeCuda))
    monkeypatch.setattr(boys, "_SINGLE_DEVICE", None)
    with boys._on_device(types.SimpleNamespace(index=0)):
        pass
    with boys._on_device(types.SimpleNamespace(index=None)):
        pass
    assert calls == []
    with boys._on_device(types.SimpleNamespace(index=2)):
        assert FakeCuda.cur == 2
    assert FakeCuda.cur == 0 and calls == [2, 0]
    with boys._on_device(3):  # an index instead of a device
        assert FakeCuda.cur == 3
    assert FakeCuda.cur == 0 and calls == [2, 0, 3, 0]
    # with one visible device there is nothing to switch
    monkeypatch.setattr(boys, "_SINGLE_DEVICE", None)
    FakeCuda.count, FakeCuda.cur = 1, 5
    with boys._on_device(0):
        assert FakeCuda.cur == 5
    assert calls == [2, 0, 3, 0]


def test_stream_handle_with_and_without_the_raw_lookup(monkeypatch):
    # the current stream's handle comes from torch's raw lookup when it exists, else from
    # a Stream object; an explicit stream is used as given
    class FakeStream:
        def __init__(self, h):
            self.cuda_stream = h

    class FakeCuda:
        @staticmethod
        def current_stream(device):
            return FakeStream(1000 + (device if isinstance(device, int) else 7))

    raw = types.SimpleNamespace(_cuda_getCurrentRawStream=lambda idx: 2000 + idx)
    monkeypatch.setattr(boys, "_torch", lambda: types.SimpleNamespace(cuda=FakeCuda, _C=raw))
    assert boys._stream_ptr(None, 3) == 2003
    assert boys._stream_ptr(None, types.SimpleNamespace(index=1)) == 2001
    assert boys._stream_ptr(None, types.SimpleNamespace(index=None)) == 1007
    assert boys._stream_ptr(FakeStream(55), 3) == 55
    bare = types.SimpleNamespace()
    monkeypatch.setattr(boys, "_torch", lambda: types.SimpleNamespace(cuda=FakeCuda, _C=bare))
    assert boys._stream_ptr(None, 3) == 1003


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no CPU or PyTorch fallback: without libboys.so every entry point raises
    from paper_2504_07637_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libboys.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(REPO, "paper_2504_07637_amd")
    for root, _, files in os.walk(pkg):
        if os.sep + "fit" in root:
            continue  # the offline fitter is not on the evaluation path
        for f in files:
            if f.endswith(".py"):
                text = open(os.path.join(root, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), f


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    line = json.loads(out.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_kernel_hash_ignores_comments(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "k.h"
    src.write_text("int a; // one\n\nint b;\n")
    monkeypatch.setattr(bench, "_CSRC", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", {"plain": ("k.h",), "eri": ("k.h", "e.h")})
    (tmp_path / "e.h").write_text("int e;\n")
    h1 = bench.kernel_hash()
    he = bench.kernel_hash("eri")
    src.write_text("int a; // another comment\n// a comment line\nint b;\n")
    assert bench.kernel_hash() == h1
    # a change to one family's own source leaves the others' hashes alone
    (tmp_path / "e.h").write_text("int e2;\n")
    assert bench.kernel_hash() == h1 and bench.kernel_hash("eri") != he
    src.write_text("int a;\nint c;\n")
    assert bench.kernel_hash() != h1


def test_consumer_side_helpers_of_the_benchmark():
    # the share of quartets below the cut-off, against a plain loop over the quartets with
    # the kernel's operation order; and the one-side lists really put every quartet on
    # their side of the n_max = 16 cut-off
    import numpy as np
    import bench
    from paper_2504_07637_amd import inputs
    g = np.random.default_rng(3)
    n = 300
    pairs = np.stack([g.uniform(0.1, 50.0, n), g.normal(0, 2, n), g.normal(0, 2, n),
                      g.normal(0, 2, n), g.uniform(0.1, 1.0, n)])
    z = 20.0
    below = 0
    for a in range(n):
        for b in range(n):
            p, q = pairs[0, a], pairs[0, b]
            pq = p * q
            rho = pq / (p + q)
            dx, dy, dz = (pairs[1, a] - pairs[1, b], pairs[2, a] - pairs[2, b],
                          pairs[3, a] - pairs[3, b])
            T = rho * (dx * dx + dy * dy + dz * dz)
            below += not (T > z)
    assert bench.below_fraction(pairs, z) == below / n ** 2
    z16 = 74.50682535593259
    for side in ("below", "past"):
        bra, ket, start = bench.one_side_lists(inputs, side)
        p, q = bra[0][::37], ket[0][::41]
        rho = p[:, None] * q[None, :] / (p[:, None] + q[None, :])
        d2 = (bra[1][::37, None] - ket[1][None, ::41]) ** 2
        T = rho * d2
        assert (T <= z16).all() if side == "below" else (T > z16).all()
        assert start[-1] == bra.shape[1] == ket.shape[1]
