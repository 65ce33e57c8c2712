"""C ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and rejects malformed requests on the host before
touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(spgemm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2408_14558_amd import _lib
    return _lib.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("spgemm_plan", "spgemm_symbolic", "spgemm_numeric", "spgemm_batched",
                     "spgemm_backward", "spgemm_plan_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2408_14558_amd import _lib
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_default_tuning_and_version(lib):
    from paper_2408_14558_amd import _lib
    t = _lib.Tuning()
    assert lib.spgemm_default_tuning(ctypes.byref(t)) == 0
    assert t.tiny_max_flop == 256 and t.hash_max_flop == 4096 and t.hash_max_nnz == 2048
    assert t.batch_streams == 0 and t.batch_form == 0 and t.reserved == 0
    assert ctypes.sizeof(_lib.Tuning) == 56
    assert lib.spgemm_default_tuning(None) == _lib.EINVAL
    assert b"gfx950" in lib.spgemm_version()


def test_default_tuning_environment_overrides(lib, monkeypatch):
    from paper_2408_14558_amd import _lib
    monkeypatch.setenv("SPGEMM_TINY_MAX_FLOP", "128")
    monkeypatch.setenv("SPGEMM_MEDIUM_KERNEL", "2")
    monkeypatch.setenv("SPGEMM_WORKSPACE_LIMIT", "123456789012")
    monkeypatch.setenv("SPGEMM_HASH_MAX_NNZ", "not-a-number")
    t = _lib.Tuning()
    assert lib.spgemm_default_tuning(ctypes.byref(t)) == 0
    assert t.tiny_max_flop == 128 and t.medium_kernel == 2
    assert t.workspace_limit == 123456789012
    assert t.hash_max_nnz == 2048  # ignored


def _csc(nrows, ncols, nnz, colptr=1, rowidx=1):
    from paper_2408_14558_amd import _lib
    return _lib.Csc(nrows, ncols, nnz, colptr, rowidx, None)


def _plan(lib, A, B, offs, P, b, tun=None, dtype=1):
    h = ctypes.c_void_p()
    o = np.asarray(offs, dtype=np.int64)
    rc = lib.spgemm_plan(ctypes.byref(A) if A is not None else None,
                         ctypes.byref(B) if B is not None else None, dtype,
                         o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if o.size else None,
                         P, b, ctypes.byref(tun) if tun is not None else None, None,
                         ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["nullA", "dims", "P0", "b0", "offs_start", "offs_end",
                                  "offs_decrease", "dtype", "neg", "big", "rows_missing",
                                  "tiny_tuning", "hash_tuning", "nnz_no_rows",
                                  "reserved_tuning", "streams_tuning"])
def test_host_side_rejections(lib, case):
    from paper_2408_14558_amd import _lib
    A = _csc(10, 8, 5)
    B = _csc(8, 4, 3)
    offs, P, b, tun, dtype = [0, 4, 8], 2, 2, None, 1
    if case == "nullA":
        A = None
    elif case == "dims":
        B = _csc(9, 4, 3)
    elif case == "P0":
        P = 0
    elif case == "b0":
        b = 0
    elif case == "offs_start":
        offs = [1, 4, 8]
    elif case == "offs_end":
        offs = [0, 4, 7]
    elif case == "offs_decrease":
        offs, P = [0, 5, 3, 8], 3
    elif case == "dtype":
        dtype = 7
    elif case == "neg":
        A = _csc(-1, 8, 5)
    elif case == "big":
        A = _csc(1 << 31, 8, 5)
    elif case == "rows_missing":
        A = _csc(10, 8, 5, rowidx=None)
    elif case == "nnz_no_rows":
        A = _csc(0, 8, 5)
    elif case.endswith("_tuning"):
        tun = _lib.Tuning()
        lib.spgemm_default_tuning(ctypes.byref(tun))
        if case == "tiny_tuning":
            tun.tiny_max_flop = 513
        elif case == "hash_tuning":
            tun.hash_max_nnz = 4096
        elif case == "reserved_tuning":
            tun.reserved = 1
        else:
            tun.batch_streams = 9
    rc, h = _plan(lib, A, B, offs, P, b, tun, dtype)
    want = _lib.EUNSUPPORTED if case == "dtype" else _lib.EINVAL
    assert rc == want
    assert not h.value
    assert len(lib.spgemm_last_error()) > 0


def test_state_and_null_handle_errors(lib):
    from paper_2408_14558_amd import _lib
    n = ctypes.c_int64()
    assert lib.spgemm_symbolic(None, None, ctypes.byref(n)) == _lib.EINVAL
    assert lib.spgemm_numeric(None, None, None, None, None) == _lib.EINVAL
    assert lib.spgemm_backward(None, None, None, None, None, None, None, None) == _lib.EINVAL
    assert lib.spgemm_plan_destroy(None) == _lib.OK
    assert lib.spgemm_batch_destroy(None) == _lib.OK
    assert lib.spgemm_plan_stats(None, None) == _lib.EINVAL


def test_c_struct_rejects_arrays_the_library_cannot_read():
    # the library reads a matrix through raw device pointers: host tensors,
    # wrong dtypes and wrong lengths are refused before any call
    import torch
    spg = pytest.importorskip("paper_2408_14558_amd")
    M = spg.DeviceCsc(5, 3, torch.tensor([0, 1, 2, 2], dtype=torch.int64),
                      torch.tensor([0, 4], dtype=torch.int32),
                      torch.tensor([1.0, 2.0], dtype=torch.float64))
    with pytest.raises(ValueError, match="on the GPU"):
        M.c_struct()


@pytest.mark.gpu
def test_c_struct_follows_the_arrays():
    # the binding keeps a matrix's C struct while its arrays stay the same
    # and builds a new one when an array, the shape or nnz changes
    import torch
    spg = pytest.importorskip("paper_2408_14558_amd")
    d = dict(device="cuda")
    M = spg.DeviceCsc(5, 3, torch.tensor([0, 1, 2, 2], dtype=torch.int64, **d),
                      torch.tensor([0, 4], dtype=torch.int32, **d),
                      torch.tensor([1.0, 2.0], dtype=torch.float64, **d))
    s1 = M.c_struct()
    assert M.c_struct() is s1
    assert (s1.nrows, s1.ncols, s1.nnz) == (5, 3, 2)
    assert s1.colptr == M.colptr.data_ptr() and s1.vals == M.vals.data_ptr()
    M.vals = torch.tensor([3.0, 4.0], dtype=torch.float64, **d)
    s2 = M.c_struct()
    assert s2 is not s1 and s2.vals == M.vals.data_ptr()
    M.rowidx = torch.tensor([1], dtype=torch.int32, **d)
    M.vals = torch.tensor([5.0], dtype=torch.float64, **d)
    M.colptr = torch.tensor([0, 1, 1, 1], dtype=torch.int64, **d)
    s3 = M.c_struct()
    assert s3.nnz == 1 and s3.rowidx == M.rowidx.data_ptr() and s3.colptr == M.colptr.data_ptr()
    E = spg.DeviceCsc(4, 2, torch.zeros(3, dtype=torch.int64, **d),
                      torch.zeros(0, dtype=torch.int32, **d), None)
    se = E.c_struct()
    assert se.nnz == 0 and not se.rowidx and not se.vals
    with pytest.raises(ValueError, match="elements"):  # colptr of the wrong length
        spg.DeviceCsc(4, 3, torch.zeros(3, dtype=torch.int64, **d),
                      torch.zeros(0, dtype=torch.int32, **d), None).c_struct()
    with pytest.raises(ValueError, match="int32"):
        spg.DeviceCsc(4, 2, torch.zeros(3, dtype=torch.int64, **d),
                      torch.zeros(0, dtype=torch.int64, **d), None).c_struct()
