"""CPU oracle for the local product of the sparsity-aware 1D SpGEMM.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct reference written
from the paper (Hong & Buluc, sparsity-aware 1D SpGEMM).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the HIP library and never imports it.

The arithmetic lives in ``oracle.c`` (FP64, built with gcc
``-O2 -ffp-contract=off -fopenmp``; the two product passes hand output
columns to OpenMP threads, each column computed by one thread in the same
order whatever the thread count); this module only marshals numpy arrays
through ctypes.  :func:`set_threads` fixes the thread count.  Matrices are accepted duck-typed: any object with
``nrows, ncols, colptr, rowidx, vals`` attributes (CSC, int64 column
pointers, int32 row ids ascending per column).

Functions and the passage each follows:

* :func:`rows_of_b`      - H_i, the nonzero rows of B_i (notation table; Alg. 1)
* :func:`block_select`   - Alg. 2 applied to every column partition of A
* :func:`gather`         - the compacted A~ of Alg. 1
* :func:`column_flops`   - sparse flops per output column (Sec. III-B)
* :func:`spgemm`         - C = A*B, Gustavson column-by-column (Sec. III-A)
* :func:`backward`       - (dC*B^T) o pattern(A) and (A^T*dC) o pattern(B)
* :func:`local_product`  - the whole local step of Alg. 1 for one partition
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)


# flags of every build of oracle.c (the sanitizer test adds its own)
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-Wall", "-Werror"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_rows_of_b.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _u8p]
    lib.oracle_block_select.argtypes = [ctypes.c_int64, _i64p, _u8p, ctypes.c_int32, _i64p,
                                        ctypes.c_int64, ctypes.c_int32, _u8p, _i32p, _i64p,
                                        _i64p, ctypes.c_int64, _i64p, _i64p]
    lib.oracle_gather.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _i32p, _i64p, _i32p, _f64p]
    lib.oracle_column_flops.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, _i64p, _i32p, _i64p]
    lib.oracle_spgemm_count.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p,
                                        ctypes.c_int64, _i64p, _i32p, ctypes.c_int64,
                                        _i64p, _i64p]
    lib.oracle_spgemm_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p,
                                       ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int64,
                                       _i64p, _i64p, _i32p, _f64p, _f64p]
    lib.oracle_backward.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p,
                                    ctypes.c_int64, _i64p, _i32p, _f64p, _i64p, _i32p,
                                    _f64p, _f64p, _f64p]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    for name in ("oracle_rows_of_b", "oracle_block_select", "oracle_gather",
                 "oracle_column_flops", "oracle_spgemm_count", "oracle_spgemm_fill",
                 "oracle_backward"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    """Threads of the product passes (n <= 0: OpenMP's default)."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    """Threads the next product pass will use."""
    return int(_load().oracle_threads())


def _p(a: Optional[np.ndarray], ptype):
    if a is None:
        return ctypes.cast(None, ptype)
    return a.ctypes.data_as(ptype)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


class Mat(NamedTuple):
    nrows: int
    ncols: int
    colptr: np.ndarray
    rowidx: np.ndarray
    vals: np.ndarray


def _arrays(M):
    colptr = np.ascontiguousarray(M.colptr, dtype=np.int64)
    rowidx = np.ascontiguousarray(M.rowidx, dtype=np.int32)
    vals = np.ascontiguousarray(M.vals, dtype=np.float64)
    return int(M.nrows), int(M.ncols), colptr, rowidx, vals


def rows_of_b(k: int, B) -> np.ndarray:
    _, _, _, Br, _ = _arrays(B)
    H = np.zeros(k, dtype=np.uint8)
    _check(_load().oracle_rows_of_b(k, Br.size, _p(Br, _i32p), _p(H, _u8p)), "rows_of_b")
    return H


class Selection(NamedTuple):
    sel: np.ndarray  # uint8[k]
    map: np.ndarray  # int32[k]
    kt: int
    blocks: np.ndarray  # int64[M, 2] (first, last) column ids
    K: int


def block_select(A, H: np.ndarray, offsets, b: int, own_whole: int = -1) -> Selection:
    _, k, Ac, _, _ = _arrays(A)
    H = np.ascontiguousarray(H, dtype=np.uint8)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    P = offs.size - 1
    sel = np.zeros(k, dtype=np.uint8)
    mp = np.zeros(k, dtype=np.int32)
    kt = ctypes.c_int64(0)
    M = ctypes.c_int64(0)
    K = ctypes.c_int64(0)
    cap = k + P
    blocks = np.zeros((max(cap, 1), 2), dtype=np.int64)
    _check(_load().oracle_block_select(k, _p(Ac, _i64p), _p(H, _u8p), P, _p(offs, _i64p), b,
                                       int(own_whole), _p(sel, _u8p), _p(mp, _i32p), ctypes.byref(kt),
                                       _p(blocks, _i64p), cap, ctypes.byref(M),
                                       ctypes.byref(K)), "block_select")
    return Selection(sel, mp, kt.value, blocks[:M.value].copy(), K.value)


def gather(A, mp: np.ndarray, kt: int) -> Mat:
    m, k, Ac, Ar, Av = _arrays(A)
    mp = np.ascontiguousarray(mp, dtype=np.int32)
    colptr = np.zeros(kt + 1, dtype=np.int64)
    lib = _load()
    _check(lib.oracle_gather(k, _p(Ac, _i64p), _p(Ar, _i32p), _p(Av, _f64p), _p(mp, _i32p),
                             _p(colptr, _i64p), _p(None, _i32p), _p(None, _f64p)), "gather")
    nnz = int(colptr[kt])
    rows = np.zeros(nnz, dtype=np.int32)
    vals = np.zeros(nnz, dtype=np.float64)
    _check(lib.oracle_gather(k, _p(Ac, _i64p), _p(Ar, _i32p), _p(Av, _f64p), _p(mp, _i32p),
                             _p(colptr, _i64p), _p(rows, _i32p), _p(vals, _f64p)), "gather")
    return Mat(m, kt, colptr, rows, vals)


def column_flops(A, B) -> np.ndarray:
    _, k, Ac, _, _ = _arrays(A)
    _, n, Bc, Br, _ = _arrays(B)
    flop = np.zeros(n, dtype=np.int64)
    _check(_load().oracle_column_flops(k, _p(Ac, _i64p), n, _p(Bc, _i64p), _p(Br, _i32p),
                                       _p(flop, _i64p)), "column_flops")
    return flop


class Product(NamedTuple):
    nrows: int
    ncols: int
    colptr: np.ndarray
    rowidx: np.ndarray
    vals: np.ndarray
    absvals: np.ndarray  # sum of |a|*|b| per stored entry


def spgemm(A, B, cols=None) -> Product:
    """C = A*B (or only the columns ``cols`` of B, in the given order)."""
    m, k, Ac, Ar, Av = _arrays(A)
    kb, n, Bc, Br, Bv = _arrays(B)
    if kb != k:
        raise ValueError("inner dimensions differ")
    lib = _load()
    if cols is None:
        ncols, cp = n, None
    else:
        cp = np.ascontiguousarray(cols, dtype=np.int64)
        ncols = cp.size
    counts = np.zeros(ncols, dtype=np.int64)
    _check(lib.oracle_spgemm_count(m, k, _p(Ac, _i64p), _p(Ar, _i32p), n, _p(Bc, _i64p),
                                   _p(Br, _i32p), ncols, _p(cp, _i64p), _p(counts, _i64p)),
           "spgemm_count")
    colptr = np.zeros(ncols + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    nnz = int(colptr[-1])
    rows = np.zeros(nnz, dtype=np.int32)
    vals = np.zeros(nnz, dtype=np.float64)
    absv = np.zeros(nnz, dtype=np.float64)
    _check(lib.oracle_spgemm_fill(m, k, _p(Ac, _i64p), _p(Ar, _i32p), _p(Av, _f64p), n,
                                  _p(Bc, _i64p), _p(Br, _i32p), _p(Bv, _f64p), ncols,
                                  _p(cp, _i64p), _p(colptr, _i64p), _p(rows, _i32p),
                                  _p(vals, _f64p), _p(absv, _f64p)), "spgemm_fill")
    return Product(m, ncols, colptr, rows, vals, absv)


def spgemm_counts(A, B, cols=None) -> np.ndarray:
    """Only the number of stored entries of each (requested) column of A*B."""
    m, k, Ac, Ar, _ = _arrays(A)
    _, n, Bc, Br, _ = _arrays(B)
    if cols is None:
        ncols, cp = n, None
    else:
        cp = np.ascontiguousarray(cols, dtype=np.int64)
        ncols = cp.size
    counts = np.zeros(ncols, dtype=np.int64)
    _check(_load().oracle_spgemm_count(m, k, _p(Ac, _i64p), _p(Ar, _i32p), n, _p(Bc, _i64p),
                                       _p(Br, _i32p), ncols, _p(cp, _i64p),
                                       _p(counts, _i64p)), "spgemm_count")
    return counts


def backward(A, B, Ccolptr, Crowidx, dCvals):
    """(dA, dB): gradients of <dC, A*B> on the stored entries of A and B."""
    m, k, Ac, Ar, Av = _arrays(A)
    _, n, Bc, Br, Bv = _arrays(B)
    Cc = np.ascontiguousarray(Ccolptr, dtype=np.int64)
    Cr = np.ascontiguousarray(Crowidx, dtype=np.int32)
    dC = np.ascontiguousarray(dCvals, dtype=np.float64)
    dA = np.zeros(Ar.size, dtype=np.float64)
    dB = np.zeros(Br.size, dtype=np.float64)
    _check(_load().oracle_backward(m, k, _p(Ac, _i64p), _p(Ar, _i32p), _p(Av, _f64p), n,
                                   _p(Bc, _i64p), _p(Br, _i32p), _p(Bv, _f64p), _p(Cc, _i64p),
                                   _p(Cr, _i32p), _p(dC, _f64p), _p(dA, _f64p), _p(dB, _f64p)),
           "backward")
    return dA, dB


class Local(NamedTuple):
    H: np.ndarray
    selection: Selection
    At: Mat
    flop: np.ndarray
    C: Product


def local_product(A, Bi, offsets, b: int, cols=None, own_whole: int = -1) -> Local:
    """One partition's step of Alg. 1: H_i, block selection, A~, flops and
    C_i.  C_i is computed from the original A, not from A~, so agreement with
    a path that multiplies A~ also shows the gather lost nothing."""
    H = rows_of_b(int(A.ncols), Bi)
    s = block_select(A, H, offsets, b, own_whole)
    At = gather(A, s.map, s.kt)
    flop = column_flops(A, Bi)
    C = spgemm(A, Bi, cols)
    return Local(H, s, At, flop, C)
