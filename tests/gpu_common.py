"""Helpers shared by the GPU tests (comparison utilities only; no Boys arithmetic)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a HIP device")
    import paper_2504_07637_amd as boys  # noqa: F401  (fails loudly if libboys.so is missing)
    boys._lib.lib()
    return torch


def same_bits(a, b):
    """Elementwise identical values (NaN matches NaN)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return (a == b) | (np.isnan(a) & np.isnan(b))


def ulp_distance(a, b):
    """|a - b| in units in the last place, by ordered integer representation."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.dtype == np.float64:
        ia = a.view(np.int64).astype(np.int64)
        ib = b.view(np.int64).astype(np.int64)
        big = np.int64(0x7FFFFFFFFFFFFFFF)
    else:
        ia = a.view(np.int32).astype(np.int64)
        ib = b.view(np.int32).astype(np.int64)
        big = np.int64(0x7FFFFFFF)
    ia = np.where(ia < 0, -(ia & big), ia)
    ib = np.where(ib < 0, -(ib & big), ib)
    d = np.abs(ia - ib)
    d = np.where(np.isnan(a) & np.isnan(b), 0, d)
    return d


def report_mismatch(name, got, want):
    bad = ~same_bits(got, want)
    if not bad.any():
        return ""
    idx = np.argwhere(bad)[:5]
    rows = [f"{name}: {int(bad.sum())} of {bad.size} differ; max ulp {int(ulp_distance(got, want).max())}"]
    for i in idx:
        t = tuple(int(v) for v in i)
        rows.append(f"  at {t}: got {got[t]!r} want {want[t]!r}")
    return "\n".join(rows)
