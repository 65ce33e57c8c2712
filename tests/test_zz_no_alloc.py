"""The no-allocation symbolic phase, spgemm_symbolic_noalloc, called through
the C ABI and checked against spgemm_symbolic on the same inputs: two calls
in a row, the second with a smaller input, each followed by the numeric
phase (column pointers and row ids bit for bit, FP64 values within 1e-12 of
the oracle per entry); then the takeover of the scratch array by the second
call (the first plan's numeric is refused) and the size limit."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _symbolic(lib, plan, ncols, noalloc):
    colptr = torch.empty(ncols + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64(-1)
    fn = lib.spgemm_symbolic_noalloc if noalloc else lib.spgemm_symbolic
    rc = fn(plan.handle, _vp(colptr), ctypes.byref(nnz))
    return rc, colptr, nnz.value


def _numeric(lib, plan, nnz):
    rows = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    vals = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda")
    rc = lib.spgemm_numeric(plan.handle, None, None, _vp(rows), _vp(vals))
    return rc, rows[:nnz], vals[:nnz]


def _both_ways(lib, A):
    """(plan run with spgemm_symbolic_noalloc, its product) after checking it
    against spgemm_symbolic and the oracle."""
    Ad = spg.DeviceCsc.from_host(A)
    ref = oracle.spgemm(A, A)
    out = []
    plans = []
    for noalloc in (False, True):
        p = spg.Plan(Ad, Ad, None, 64)
        rc, colptr, nnz = _symbolic(lib, p, A.ncols, noalloc)
        assert rc == 0, lib.spgemm_last_error()
        rc, rows, vals = _numeric(lib, p, nnz)
        assert rc == 0, lib.spgemm_last_error()
        torch.cuda.synchronize()
        out.append((colptr.cpu().numpy(), rows.cpu().numpy(), vals.cpu().numpy()))
        plans.append(p)
    st = plans[1].stats()
    (c0, r0, v0), (c1, r1, v1) = out
    assert np.array_equal(c1, c0) and np.array_equal(c1, ref.colptr)
    assert np.array_equal(r1, r0) and np.array_equal(r1, ref.rowidx)
    assert_values(v1, ref.vals, ref.absvals, True)
    assert_values(v0, ref.vals, ref.absvals, True)
    plans[0].close()
    return plans[1], st


def test_noalloc_symbolic_twice_then_takeover_and_limit():
    lib = spg.load()
    big = synth.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
    small = synth.rmat(10, 16, 0.57, 0.19, 0.19, 0.05, seed=5)
    p1, st1 = _both_ways(lib, big)
    # the kept data of both kinds went to the scratch array
    assert st1["sym_bins"][1] > 0 and st1["sym_bins"][6] > 0
    p2, st2 = _both_ways(lib, small)
    assert small.nnz < big.nnz
    # the second call took the array over: the first plan's numeric is refused
    rc, _, _ = _numeric(lib, p1, st1["nnz_C"])
    assert rc == -5
    assert b"taken over" in lib.spgemm_last_error()
    # a symbolic phase again makes the first plan usable
    rc, colptr, nnz = _symbolic(lib, p1, big.ncols, True)
    assert rc == 0 and nnz == st1["nnz_C"]
    rc, rows, _ = _numeric(lib, p1, nnz)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(rows.cpu().numpy(), oracle.spgemm(big, big).rowidx)
    p1.close()
    p2.close()
    # above the array's size: every column in the dense bin of a 65536-row
    # product needs 8 KiB, far more than 64 MiB in all
    huge = synth.rmat(16, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
    Hd = spg.DeviceCsc.from_host(huge)
    tun = spg.tuning(tiny_max_flop=0, hash_max_flop=0)
    p3 = spg.Plan(Hd, Hd, None, 64, tuning=tun)
    rc, _, _ = _symbolic(lib, p3, huge.ncols, True)
    assert rc == -2
    assert b"bytes of scratch" in lib.spgemm_last_error()
    rc, _, _ = _numeric(lib, p3, 1)
    assert rc == -5  # no symbolic phase completed
    rc, _, nnz = _symbolic(lib, p3, huge.ncols, False)  # the allocating phase still works
    assert rc == 0 and nnz > 0
    p3.close()
