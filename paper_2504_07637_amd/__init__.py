"""Boys functions F_m(x), m = 0..n_max, on MI355X (gfx950) by Laikov's global closed form.

Every computation runs in the HIP library libboys.so (include/boys.h); this module only
allocates tensors with PyTorch, takes the current HIP stream and marshals arguments.

    import torch, paper_2504_07637_amd as boys
    x = torch.rand(1 << 20, dtype=torch.float64, device="cuda") * 40
    F = boys.boys_eval(x, 16)                  # (17, 2^20) float64, F[m, i] = F_m(x[i])
    G = boys.boys_eval(x, 16, precision="fp32")  # mixed class, float32 output
    H = boys.boys_eval(x, 16, precision="fp32x")  # float32 output at full single accuracy
    S = boys.boys_eval(x, 16, precision="fp32s")  # all-binary32 arithmetic
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import FP32, FP32S, FP32X, FP64, FP64_PLUS, BoysArray, BoysError, BoysTuning

__all__ = ["boys_eval", "boys_eval_rows", "boys_eval_split", "boys_eri_ssss", "boys_eval_batched", "boys_eval_batched_noalloc", "Plan", "autotune", "max_nmax", "cutoff",
           "precision_code", "padded_ld", "empty_out", "BoysError", "FP64", "FP32", "FP64_PLUS",
           "FP32X", "FP32S"]


_CODES = {}
for _code, _names in ((FP64, ("fp64", "float64", "double")), (FP32, ("fp32", "float32", "mixed")),
                      (FP64_PLUS, ("fp64plus", "fp64+")), (FP32X, ("fp32x",)),
                      (FP32S, ("fp32s", "single"))):
    _CODES[_code] = _code
    for _name in _names:
        _CODES[_name] = _code


def precision_code(precision) -> int:
    try:
        return _CODES[precision]
    except (KeyError, TypeError):
        raise ValueError(f"unknown precision {precision!r}") from None


_TORCH = None


def _torch():
    global _TORCH
    if _TORCH is None:
        import torch
        _TORCH = torch
    return _TORCH


def _out_dtype(code):
    torch = _torch()
    return torch.float32 if code in (FP32, FP32X, FP32S) else torch.float64


def _stream_ptr(stream, device):
    torch = _torch()
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        idx = device if isinstance(device, int) else device.index
        if raw is not None and idx is not None:
            return raw(idx)  # the current stream's handle, without building a Stream object
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream


_SINGLE_DEVICE = None


def _single_device():
    global _SINGLE_DEVICE
    if _SINGLE_DEVICE is None:
        _SINGLE_DEVICE = _torch().cuda.device_count() == 1
    return _SINGLE_DEVICE


class _on_device:
    """Make `device` (a torch.device or an index) current for the duration of a call (a
    no-op when it already is, and when only one device is visible)."""

    __slots__ = ("dev", "prev")

    def __init__(self, device):
        self.dev = device if isinstance(device, int) else device.index  # None: current
        self.prev = None

    def __enter__(self):
        if self.dev is None or _single_device():
            return self
        torch = _torch()
        cur = torch.cuda.current_device()
        if cur != self.dev:
            self.prev = cur
            torch.cuda.set_device(self.dev)
        return self

    def __exit__(self, *exc):
        if self.prev is not None:
            _torch().cuda.set_device(self.prev)
        return False


def padded_ld(n: int, precision) -> int:
    """Row stride (elements) that starts every output row on a 128-byte boundary.

    Rows that straddle cache lines are written as partial lines, which costs up to a
    third of the store bandwidth (measured); outputs allocated here use this stride."""
    q = 32 if precision_code(precision) in (FP32, FP32X, FP32S) else 16
    return max(q, (n + q - 1) // q * q)


def empty_out(n: int, n_max: int, precision="fp64", device="cuda"):
    """An uninitialised (n_max+1, n) output view with a padded row stride."""
    torch = _torch()
    code = precision_code(precision)
    buf = torch.empty((n_max + 1, padded_ld(n, code)), dtype=_out_dtype(code), device=device)
    return buf[:, :n]


def _check_x(x):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError("x must be a float64 tensor on a HIP device")
    if x.dim() != 1 or not x.is_contiguous():
        raise ValueError("x must be 1-D and contiguous")


def boys_eval(x, n_max: int, precision="fp64", out=None, stream=None):
    """F_m(x) for m = 0..n_max as a (n_max+1, len(x)) tensor.

    The row stride is out.stride(0); when out is not given it is padded so that every
    row starts on a 128-byte boundary (see padded_ld)."""
    _check_x(x)
    code = precision_code(precision)
    n = x.numel()
    dev = x.get_device()
    if out is None:
        out = empty_out(n, n_max, code, x.device)
    else:
        if out.dtype != _out_dtype(code) or out.get_device() != dev or out.dim() != 2:
            raise TypeError("out has the wrong dtype, device or rank")
        if out.shape[0] != n_max + 1 or out.shape[1] != n or out.stride(1) != 1:
            raise ValueError("out must be (n_max+1, n) with unit column stride")
    ld = out.stride(0) if n > 0 else max(n, 1)
    fn = _lib.lib().boys_eval
    if _single_device():  # nothing to switch: skip the guard (this call is latency-bound)
        st = fn(x.data_ptr(), n, n_max, out.data_ptr(), ld, code, _stream_ptr(stream, dev))
    else:
        with _on_device(dev):
            st = fn(x.data_ptr(), n, n_max, out.data_ptr(), ld, code, _stream_ptr(stream, dev))
    if st:
        _lib.check(st, "boys_eval")
    return out


def boys_eval_rows(x, n_max: int, rows, precision="fp64", out=None, stream=None):
    """The orders listed in `rows` (each 0..n_max) of the order-n_max evaluation, as a
    (len(rows), len(x)) tensor in increasing order of m; every order is still computed
    (each stored row equals that row of boys_eval bit for bit)."""
    _check_x(x)
    code = precision_code(precision)
    sel = sorted(set(int(m) for m in rows))
    if not sel or sel[0] < 0 or sel[-1] > n_max:
        raise ValueError("rows must name orders 0..n_max")
    mask = 0
    for m in sel:
        mask |= 1 << m
    n = x.numel()
    if out is None:
        out = empty_out(n, len(sel) - 1, code, x.device)
    elif (out.dtype != _out_dtype(code) or out.device != x.device or out.dim() != 2
          or out.shape[0] != len(sel) or out.shape[1] != n or out.stride(1) != 1):
        raise ValueError("out must be (len(rows), n) of the class's dtype, unit column stride")
    ld = out.stride(0) if n > 0 else 1
    with _on_device(x.device):
        st = _lib.lib().boys_eval_rows(x.data_ptr(), n, n_max, mask, out.data_ptr(), ld, code,
                                       _stream_ptr(stream, x.device))
    _lib.check(st, "boys_eval_rows")
    return out


def boys_eval_split(x, n_max: int, n_bar: int, out=None, stream=None):
    """The two-approximation option (binary64): rows 0..n_bar from the order-n_bar
    approximant and its recursion, rows n_bar+1..n_max from the order-n_max one."""
    torch = _torch()
    _check_x(x)
    n = x.numel()
    if out is None:
        out = empty_out(n, n_max, FP64, x.device)
    elif (out.dtype != torch.float64 or out.device != x.device or out.dim() != 2
          or out.shape[0] != n_max + 1 or out.shape[1] != n or out.stride(1) != 1):
        raise ValueError("out must be a float64 (n_max+1, n) tensor with unit column stride")
    ld = out.stride(0) if n > 0 else 1
    with _on_device(x.device):
        st = _lib.lib().boys_eval_split(ctypes.c_void_p(x.data_ptr()), n, n_bar, n_max,
                                        ctypes.c_void_p(out.data_ptr()), ld,
                                        _stream_ptr(stream, x.device))
    _lib.check(st, "boys_eval_split")
    return out


def _pair_list(pairs, start):
    """pairs: float64 (5, n) device tensor of (p, Px, Py, Pz, w) rows with unit stride
    along n; start: int32 (count+1,) device tensor."""
    torch = _torch()
    if (not isinstance(pairs, torch.Tensor) or pairs.dtype != torch.float64 or not pairs.is_cuda
            or pairs.dim() != 2 or pairs.shape[0] != 5
            or (pairs.shape[1] > 1 and pairs.stride(1) != 1)):
        raise TypeError("pairs must be a float64 (5, n) device tensor with unit column stride")
    if (not isinstance(start, torch.Tensor) or start.dtype != torch.int32 or not start.is_cuda
            or start.dim() != 1 or not start.is_contiguous() or start.numel() < 1):
        raise TypeError("start must be a contiguous int32 device tensor of count+1 entries")
    rows = [ctypes.c_void_p(pairs[k].data_ptr()) for k in range(5)]
    return _lib.BoysPairList(*rows, ctypes.c_void_p(start.data_ptr()), start.numel() - 1)


def boys_eri_ssss(bra_pairs, bra_start, ket_pairs, ket_start, n_max: int, out=None,
                  stream=None):
    """Contracted (ss|ss)^(m), m = 0..n_max, for every (bra, ket) contracted pair: a
    (n_max+1, n_bra * n_ket) float64 tensor (column i * n_ket + j).  The F_m are formed and
    consumed on the device; see include/boys.h for the arithmetic."""
    torch = _torch()
    bra = _pair_list(bra_pairs, bra_start)
    ket = _pair_list(ket_pairs, ket_start)
    total = bra.count * ket.count
    dev = bra_pairs.device
    if out is None:
        out = empty_out(total, n_max, FP64, dev)
    elif (out.dtype != torch.float64 or out.dim() != 2 or out.shape[0] != n_max + 1
          or out.shape[1] != total or out.stride(1) != 1):
        raise ValueError("out must be a float64 (n_max+1, n_bra*n_ket) tensor")
    ld = out.stride(0) if total > 0 else 1
    with _on_device(dev):
        st = _lib.lib().boys_eri_ssss(ctypes.byref(bra), ctypes.byref(ket), n_max,
                                      ctypes.c_void_p(out.data_ptr()), ld,
                                      _stream_ptr(stream, dev))
    _lib.check(st, "boys_eri_ssss")
    return out


def _arrays(xs, n_maxs, precisions, outs):
    torch = _torch()
    if not (len(xs) == len(n_maxs) == len(precisions)):
        raise ValueError("xs, n_maxs and precisions differ in length")
    if outs is None:
        outs = [empty_out(x.numel(), m, p, x.device) for x, m, p in zip(xs, n_maxs, precisions)]
    arr = (BoysArray * max(1, len(xs)))()
    for k, (x, m, p, o) in enumerate(zip(xs, n_maxs, precisions, outs)):
        _check_x(x)
        code = precision_code(p)
        if o.dtype != _out_dtype(code) or o.shape[0] != m + 1 or o.shape[1] != x.numel():
            raise ValueError(f"out[{k}] does not match its array")
        arr[k].x = x.data_ptr()
        arr[k].out = o.data_ptr()
        arr[k].n = x.numel()
        arr[k].ld_out = o.stride(0) if x.numel() > 0 else 1
        arr[k].n_max = m
        arr[k].precision = code
    return arr, outs


def boys_eval_batched(xs, n_maxs, precisions, outs=None, stream=None):
    """Evaluate several arrays in one batched launch (the default schedule: one wave per
    256-argument tile); returns the list of outputs."""
    torch = _torch()
    arr, outs = _arrays(xs, n_maxs, precisions, outs)
    dev = xs[0].device if xs else torch.device("cuda")
    with _on_device(dev):
        st = _lib.lib().boys_eval_batched(arr, len(xs), _stream_ptr(stream, dev))
    _lib.check(st, "boys_eval_batched")
    return outs


def boys_eval_batched_noalloc(xs, n_maxs, precisions, outs=None, stream=None):
    """boys_eval_batched without device allocations inside the library (its tables go to
    a fixed device array); the call returns after the batch has finished.  Outputs the
    caller does not pass are allocated here, by torch, before the call."""
    torch = _torch()
    arr, outs = _arrays(xs, n_maxs, precisions, outs)
    dev = xs[0].device if xs else torch.device("cuda")
    with _on_device(dev):
        st = _lib.lib().boys_eval_batched_noalloc(arr, len(xs), _stream_ptr(stream, dev))
    _lib.check(st, "boys_eval_batched_noalloc")
    return outs


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, BoysTuning):
        return t
    return BoysTuning(int(t.get("tile", 0)), int(t.get("block", 0)),
                      int(t.get("grid_per_cu", 0)), int(t.get("schedule", 1)),
                      int(t.get("order", 1)), int(t.get("split_nmax", 0)))


class Plan:
    """A batched schedule captured in a HIP graph; execute() replays it.

    tuning: None for the library defaults (one wave per 256-argument tile, one launch), or a
    dict of boys_tuning fields (tile, block, grid_per_cu, schedule, order, split_nmax)."""

    def __init__(self, xs, n_maxs, precisions, outs=None, tuning=None):
        torch = _torch()
        self._arr, self.outs = _arrays(xs, n_maxs, precisions, outs)
        self._keep = (list(xs), list(self.outs))
        self.device = xs[0].device if xs else torch.device("cuda")
        self._p = ctypes.c_void_p()
        t = _tuning(tuning)
        with _on_device(self.device):
            st = _lib.lib().boys_plan_create(ctypes.byref(self._p), self._arr, len(xs),
                                             ctypes.byref(t) if t is not None else None)
        _lib.check(st, "boys_plan_create")

    def execute(self, stream=None):
        fn = _lib.lib().boys_plan_execute
        if _single_device():
            st = fn(self._p, _stream_ptr(stream, self.device))
        else:
            with _on_device(self.device):
                st = fn(self._p, _stream_ptr(stream, self.device))
        if st:
            _lib.check(st, "boys_plan_execute")
        return self.outs

    def update(self, xs, outs):
        arr, outs = _arrays(xs, [a.n_max for a in self._arr[:len(xs)]],
                            [a.precision for a in self._arr[:len(xs)]], outs)
        st = _lib.lib().boys_plan_update(self._p, arr, len(xs))
        _lib.check(st, "boys_plan_update")
        self._arr, self.outs = arr, outs
        self._keep = (list(xs), list(outs))

    def close(self):
        if self._p:
            _lib.lib().boys_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(xs, n_maxs, precisions, candidates, warmup=2, reps=5, stream=None):
    """Time each candidate tuning (dicts of boys_tuning fields) on this batch.

    Returns (the fastest candidate, as given, [ms per candidate])."""
    torch = _torch()
    arr, outs = _arrays(xs, n_maxs, precisions, None)
    cand = (BoysTuning * len(candidates))(*[_tuning(c) for c in candidates])
    best = BoysTuning()
    times = (ctypes.c_float * len(candidates))()
    dev = xs[0].device
    with _on_device(dev):
        st = _lib.lib().boys_autotune(arr, len(xs), cand, len(candidates), warmup, reps,
                                      _stream_ptr(stream, dev), ctypes.byref(best), times)
    _lib.check(st, "boys_autotune")
    # the caller's own candidate (as given) that the library picked
    fields = [f for f, _ in BoysTuning._fields_]
    key = [getattr(best, f) for f in fields]
    for c, t in zip(candidates, cand):
        if [getattr(t, f) for f in fields] == key:
            return c, list(times)
    return dict(zip(fields, key)), list(times)


def max_nmax(precision="fp64") -> int:
    return int(_lib.lib().boys_max_nmax(precision_code(precision)))


def cutoff(n: int, precision="fp64") -> float:
    return float(_lib.lib().boys_cutoff(n, precision_code(precision)))
