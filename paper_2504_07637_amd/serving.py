"""Serving loop: Python face of boys_server_* (include/boys.h) and a Poisson load driver.

The scheduling, admission by device-memory budget, continuous batching and completion
tracking run in the library (C++ scheduler thread + HIP streams); this module marshals
arguments, keeps submitted host buffers alive until completion, and measures.

    srv = Server(budget_bytes=8 << 30)
    rid = srv.submit(x_pinned, n_max=12, precision="fp64")
    ...
    for rid in srv.poll():
        out = srv.fetch(rid)          # (n_max+1, n) tensor on the device (a copy)
        srv.release(rid)              # safe at once: the server keeps the memory until
                                      # the copy enqueued by fetch has completed

A request whose batch failed on the device is reported by poll too; fetch and times then
raise BoysError with status BOYS_ERR_DEVICE (release it like any other).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import _lib
from ._lib import BoysServerConfig, BoysServerStats


def _pc(p):
    from . import precision_code
    return precision_code(p)


class Server:
    def __init__(self, budget_bytes: int = 8 << 30, streams: int = 4, max_batch: int = 256,
                 tile: int = 256, max_tiles: int = 65536, device=None):
        import torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        cfg = BoysServerConfig(int(budget_bytes), streams, max_batch, tile, max_tiles)
        self._s = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _lib.lib().boys_server_create(ctypes.byref(self._s), ctypes.byref(cfg))
        _lib.check(st, "boys_server_create")
        self._live = {}   # id -> (host tensor kept alive, n, n_max, precision code)

    def submit(self, x_host, n_max: int, precision="fp64") -> int:
        """x_host: a contiguous float64 CPU tensor (pinned for asynchronous copies)."""
        import torch
        if not isinstance(x_host, torch.Tensor) or x_host.is_cuda or x_host.dtype != torch.float64:
            raise TypeError("x_host must be a float64 CPU tensor")
        if not x_host.is_contiguous():
            raise ValueError("x_host must be contiguous")
        code = _pc(precision)
        rid = ctypes.c_uint64()
        st = _lib.lib().boys_server_submit(self._s, ctypes.c_void_p(x_host.data_ptr()),
                                           x_host.numel(), n_max, code, ctypes.byref(rid))
        _lib.check(st, "boys_server_submit")
        self._live[rid.value] = (x_host, x_host.numel(), n_max, code)
        return rid.value

    def poll(self, max_ids: int = 4096):
        buf = (ctypes.c_uint64 * max_ids)()
        k = _lib.lib().boys_server_poll(self._s, buf, max_ids)
        return [buf[i] for i in range(k)]

    def times(self, rid: int):
        """(t_submit, t_done) in seconds on the server clock."""
        ts, td = ctypes.c_double(), ctypes.c_double()
        st = _lib.lib().boys_server_result(self._s, rid, None, None, ctypes.byref(ts),
                                           ctypes.byref(td))
        _lib.check(st, "boys_server_result")
        return ts.value, td.value

    def fetch(self, rid: int, stream=None):
        """A device copy of a completed request's output, shape (n_max+1, n), enqueued on
        `stream` (default: the current stream).  The request may be released right away."""
        import torch
        _, n, n_max, code = self._live[rid]
        dt = torch.float32 if code in (_lib.FP32, _lib.FP32X, _lib.FP32S) else torch.float64
        out = torch.empty((n_max + 1, n), dtype=dt, device=self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        st = _lib.lib().boys_server_copy_result(self._s, rid, ctypes.c_void_p(out.data_ptr()),
                                                n, ctypes.c_void_p(stream.cuda_stream))
        _lib.check(st, "boys_server_copy_result")
        return out

    def release(self, rid: int):
        st = _lib.lib().boys_server_release(self._s, rid)
        _lib.check(st, "boys_server_release")
        self._live.pop(rid, None)

    def stats(self) -> dict:
        s = BoysServerStats()
        _lib.check(_lib.lib().boys_server_get_stats(self._s, ctypes.byref(s)), "boys_server_get_stats")
        return {k: int(getattr(s, k)) for k, _ in BoysServerStats._fields_}

    def drain(self, timeout_s: float = 60.0):
        """Wait until no admitted request is pending or running (queued ones may remain)."""
        st = _lib.lib().boys_server_drain(self._s, timeout_s)
        if st != _lib.OK:
            raise _lib.BoysError(st, f"boys_server_drain (stats {self.stats()})")

    def close(self):
        if self._s:
            _lib.lib().boys_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def argument_pool(size: int = 1 << 24, seed: int = 5):
    """A pinned host pool of integral-workload arguments; requests take windows of it."""
    import torch

    from . import inputs
    x = inputs.integral_args(size, seed=seed)
    t = torch.empty(size, dtype=torch.float64, pin_memory=True)
    t.copy_(torch.from_numpy(x))
    return t


def run_poisson(server: Server, requests, pool, keep=None, on_done=None):
    """Submit requests [(t_arrival, length, n_max, precision class)] at their arrival times.

    Each request's arguments are a window of `pool` (starting at a request-specific
    offset).  Completed requests are released at once, except those whose index is in
    `keep` (returned so the caller can check them; release them afterwards).
    Returns a dict of latencies (seconds), values, lags and server statistics.
    """
    keep = set(keep or ())
    P = pool.numel()
    lat = {}
    lag = []
    values = 0
    id2idx = {}
    kept = {}
    t0 = time.perf_counter()
    first_submit = None

    def collect():
        for rid in server.poll():
            ts, td = server.times(rid)
            i = id2idx.pop(rid)
            lat[i] = td - ts
            if i in keep:
                kept[i] = rid
            else:
                if on_done is not None:
                    on_done(i, rid)
                server.release(rid)

    for i, (ta, ln, nm, pr) in enumerate(requests):
        while time.perf_counter() - t0 < ta:
            collect()
        off = (i * 1000003) % (P - ln)
        now = time.perf_counter() - t0
        lag.append(now - ta)
        rid = server.submit(pool[off:off + ln], nm, pr)
        if first_submit is None:
            first_submit = now
        id2idx[rid] = i
        values += ln * (nm + 1)
    # keep collecting (and releasing) until every request has completed: queued requests
    # may be waiting for the memory that completed ones still hold
    deadline = time.perf_counter() + 120.0
    while len(lat) < len(requests):
        server.drain(120.0)
        collect()
        if time.perf_counter() > deadline:
            raise RuntimeError(f"serving stalled: {server.stats()}")
    t_end = time.perf_counter() - t0
    lats = np.array([lat[i] for i in sorted(lat)])
    return {"latencies": lats, "lag": np.array(lag), "values": values,
            "wall": t_end - (first_submit or 0.0), "kept": kept, "stats": server.stats(),
            "n_requests": len(requests)}


def summarize(res) -> dict:
    lat = res["latencies"] * 1e3
    return {"requests": res["n_requests"],
            "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4),
            "values_per_s": res["values"] / res["wall"],
            "submit_lag_p99_ms": round(float(np.percentile(res["lag"], 99)) * 1e3, 4),
            "batches": res["stats"]["batches"],
            "max_inflight_requests": res["stats"]["max_inflight"],
            "max_queued": res["stats"]["max_queued"],
            "max_bytes_in_use": res["stats"]["max_bytes_in_use"]}
