"""Dense output columns of a tall A (m above 2^18 rows): the symbolic count
and the numeric values of such columns are computed in bands of 2^18 rows,
each reaching exactly its products through the split table.  Parity with
the oracle on every stage, at m = 2^20 (four whole bands) and at a ragged
m (a short last band), in FP64 and FP32, with small value windows (windows
that split row blocks inside a band) and the dense-first bin."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")

BAND = 1 << 18


def tall_pair(m, seed, k=4096, n=192, per_col=32, dense_cols=48):
    """A: m x k, about per_col rows per column, half uniform over [0, m) and
    half packed around the band borders (so dense output columns straddle
    them); B: k x n, its first dense_cols columns with 400-1500 entries (far
    beyond the hash bins once multiplied by A), the rest with 1-8."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    borders = np.arange(BAND, m, BAND)
    for c in range(k):
        u = rng.integers(0, m, per_col)
        if borders.size:
            near = rng.choice(borders, per_col) + rng.integers(-3000, 3000, per_col)
        else:
            near = rng.integers(0, m, per_col)
        r = np.unique(np.clip(np.concatenate([u[: per_col // 2], near[: per_col // 2]]), 0, m - 1))
        rows.append(r)
        cols.append(np.full(r.size, c))
    r, c = np.concatenate(rows), np.concatenate(cols)
    A = synth.from_triplets(m, k, r, c, rng.uniform(-1, 1, r.size))
    rows, cols = [], []
    for j in range(n):
        cnt = int(rng.integers(400, 1500)) if j < dense_cols else int(rng.integers(1, 9))
        cnt = min(cnt, k)
        rr = rng.choice(k, cnt, replace=False)
        rows.append(rr)
        cols.append(np.full(rr.size, j))
    r, c = np.concatenate(rows), np.concatenate(cols)
    B = synth.from_triplets(k, n, r, c, rng.uniform(-1, 1, r.size))
    return A, B


def run_and_check(A, B, dtype, tun=None):
    Ad = spg.DeviceCsc.from_host(A, dtype=dtype)
    Bd = spg.DeviceCsc.from_host(B, dtype=dtype)
    if dtype == torch.float32:
        A, B = synth.as_fp32(A), synth.as_fp32(B)
    ref = oracle.spgemm(A, B)
    with spg.Plan(Ad, Bd, None, 64, tuning=tun) as p:
        colptr = p.symbolic()
        st = p.stats()
        assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
        for rep in range(2):  # the second run reuses the split table
            rows, vals = p.numeric()
            assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
            assert_values(vals.cpu().numpy(), ref.vals, ref.absvals, dtype == torch.float64)
    return st


@pytest.mark.parametrize("m", [1 << 20, (1 << 20) + 12345])
def test_tall_dense_columns_fp64(m):
    A, B = tall_pair(m, seed=41 + (m & 7))
    print("tall m", m, "nnzA", A.nnz, "nnzB", B.nnz, flush=True)
    st = run_and_check(A, B, torch.float64)
    assert st["sym_bins"][6] > 0 and st["num_bins"][6] + st["num_bins"][7] > 0


def test_tall_dense_columns_small_windows_and_first_bin():
    A, B = tall_pair((1 << 20) + 12345, seed=43)
    tun = spg.tuning(dense_window=256, dense_first_flop=30000)
    st = run_and_check(A, B, torch.float64, tun)
    assert st["num_bins"][7] > 0 and st["num_bins"][6] > 0


def test_tall_dense_columns_fp32():
    A, B = tall_pair(1 << 20, seed=44)
    run_and_check(A, B, torch.float32)


def test_tall_noalloc_needs_the_split_table_first():
    """spgemm_symbolic_noalloc cannot take the split table a tall plan with
    dense columns needs: it refuses (SPGEMM_ENOMEM) until one
    spgemm_symbolic run has built it, then gives the same counts."""
    A, B = tall_pair(1 << 20, seed=45, k=1024, n=64, dense_cols=8)
    ref = oracle.spgemm(A, B)
    lib = spg.load()
    with spg.Plan(spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B), None, 64) as p:
        colptr = torch.empty(B.ncols + 1, dtype=torch.int64, device="cuda")
        nnz = ctypes.c_int64(-1)
        vp = ctypes.c_void_p(colptr.data_ptr())
        assert lib.spgemm_symbolic_noalloc(p.handle, vp, ctypes.byref(nnz)) == -2
        assert b"split table" in lib.spgemm_last_error()
        assert lib.spgemm_symbolic(p.handle, vp, ctypes.byref(nnz)) == 0
        assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
        colptr.zero_()
        assert lib.spgemm_symbolic_noalloc(p.handle, vp, ctypes.byref(nnz)) == 0
        assert nnz.value == ref.colptr[-1]
        assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
        rows = torch.empty(nnz.value, dtype=torch.int32, device="cuda")
        vals = torch.empty(nnz.value, dtype=torch.float64, device="cuda")
        assert lib.spgemm_numeric(p.handle, None, None, ctypes.c_void_p(rows.data_ptr()),
                                  ctypes.c_void_p(vals.data_ptr())) == 0
        assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
        assert_values(vals.cpu().numpy(), ref.vals, ref.absvals, True)
