"""Helpers shared by the GPU parity tests (comparison only, no arithmetic of
the method)."""

from __future__ import annotations

import numpy as np


def fp64_entry_ok(got, ref, absref, rel=1e-12):
    """Per-entry FP64 bound: |got - ref| <= rel * max(|ref|, sum |a||b|)."""
    got = np.asarray(got, dtype=np.float64)
    bound = rel * np.maximum(np.abs(ref), absref)
    err = np.abs(got - ref)
    bad = err > bound
    return (not bad.any()), (float(err.max()) if err.size else 0.0), int(bad.sum())


def fp32_normwise(got, ref):
    """||got - ref||_F / ||ref||_F with ref from the FP64 oracle."""
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    den = np.linalg.norm(ref)
    if den == 0:
        return float(np.linalg.norm(got))
    return float(np.linalg.norm(got - ref) / den)


def assert_values(got, ref, absref, dtype_is_fp64: bool):
    if dtype_is_fp64:
        ok, err, nbad = fp64_entry_ok(got, ref, absref)
        assert ok, f"{nbad} FP64 entries beyond 1e-12 relative (max abs err {err:g})"
    else:
        r = fp32_normwise(got, ref)
        assert r <= 1e-5, f"FP32 normwise error {r:g} > 1e-5"


def columns_of(colptr, rowidx, vals, cols):
    """Concatenated (colptr, rows, vals) of the chosen columns."""
    colptr = np.asarray(colptr)
    parts_r, parts_v, ptr = [], [], [0]
    for j in cols:
        lo, hi = int(colptr[j]), int(colptr[j + 1])
        parts_r.append(np.asarray(rowidx[lo:hi]))
        if vals is not None:
            parts_v.append(np.asarray(vals[lo:hi]))
        ptr.append(ptr[-1] + hi - lo)
    r = np.concatenate(parts_r) if parts_r else np.zeros(0, np.int32)
    v = np.concatenate(parts_v) if parts_v else np.zeros(0)
    return np.array(ptr, dtype=np.int64), r, v
