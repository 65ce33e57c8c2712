"""Python binding of the local SpGEMM: argument marshalling over the C ABI.

Every step runs inside libspgemm.so; this module only allocates the
caller-owned buffers with torch (device memory) and passes raw pointers and
the current HIP stream.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _check_tensor(t, what, dtype, n, exact=False, device=None):
    """O(1) checks before a tensor's address goes to the library: on a GPU
    (the given device, if any), contiguous, of the dtype, and holding n
    elements (at least n unless exact)."""
    if not t.is_cuda or (device is not None and t.device != device):
        raise ValueError(f"{what} must be a tensor on the GPU{'' if device is None else f' {device}'}")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous {dtype} tensor")
    if (t.numel() != n) if exact else (t.numel() < n):
        raise ValueError(f"{what} holds {t.numel()} elements, needs {n}")


def _stream(stream=None):
    if stream is None:
        if _raw_stream is not None:  # the current stream's handle without a Stream object
            return ctypes.c_void_p(_raw_stream(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class DeviceCsc:
    """A CSC matrix whose arrays live on the GPU."""
    nrows: int
    ncols: int
    colptr: torch.Tensor  # int64[ncols+1]
    rowidx: torch.Tensor  # int32[nnz]
    vals: Optional[torch.Tensor]  # float32/float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    @classmethod
    def from_host(cls, M, dtype=torch.float64, device="cuda") -> "DeviceCsc":
        """From any object with nrows, ncols, colptr, rowidx, vals (numpy)."""
        colptr = torch.as_tensor(np.ascontiguousarray(M.colptr, dtype=np.int64)).to(device)
        rowidx = torch.as_tensor(np.ascontiguousarray(M.rowidx, dtype=np.int32)).to(device)
        vals = None
        if M.vals is not None:
            vals = torch.as_tensor(np.ascontiguousarray(M.vals)).to(device=device, dtype=dtype)
        return cls(int(M.nrows), int(M.ncols), colptr, rowidx, vals)

    def c_struct(self) -> _lib.Csc:
        # kept while the shape and the arrays' addresses stay the same (a
        # plan per step marshals the same matrices again)
        nnz = self.rowidx.numel()
        key = (self.nrows, self.ncols, nnz, self.colptr.data_ptr(), self.rowidx.data_ptr(),
               None if self.vals is None else self.vals.data_ptr())
        kept = self.__dict__.get("_c_struct")
        if kept is not None and kept[0] == key:
            return kept[1]
        # the library reads these arrays through raw device pointers
        _check_tensor(self.colptr, "colptr", torch.int64, self.ncols + 1, exact=True)
        _check_tensor(self.rowidx, "rowidx", torch.int32, nnz, exact=True,
                      device=self.colptr.device)
        if self.vals is not None:
            if self.vals.dtype not in (torch.float32, torch.float64):
                raise ValueError("vals must be float32 or float64")
            _check_tensor(self.vals, "vals", self.vals.dtype, nnz, exact=True,
                          device=self.colptr.device)
        s = _lib.Csc(self.nrows, self.ncols, nnz, key[3], key[4] if nnz else None,
                     key[5] if nnz else None)
        self.__dict__["_c_struct"] = (key, s)
        return s

    def to_host(self):
        v = None if self.vals is None else self.vals.cpu().numpy()
        return HostCsc(self.nrows, self.ncols, self.colptr.cpu().numpy(),
                       self.rowidx.cpu().numpy(), v)


@dataclass
class HostCsc:
    nrows: int
    ncols: int
    colptr: np.ndarray
    rowidx: np.ndarray
    vals: Optional[np.ndarray]


def default_tuning() -> _lib.Tuning:
    t = _lib.Tuning()
    check(_lib.load().spgemm_default_tuning(ctypes.byref(t)), "spgemm_default_tuning")
    return t


def tuning(**kw) -> _lib.Tuning:
    """The defaults with the named fields of spgemm_tuning replaced."""
    t = default_tuning()
    names = {f[0] for f in _lib.Tuning._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"spgemm_tuning has no field {k!r}")
        setattr(t, k, v)
    return t


BIN_NAMES = ["empty", "tiny", "hash0", "hash1", "hash2", "hash3", "dense", "dense-first"]


class Plan:
    """One partition's local product C_i = A * B_i (plan, symbolic, numeric,
    backward).  Keeps A and B_i alive while it exists."""

    def __init__(self, A: DeviceCsc, Bi: DeviceCsc, offsets=None, block_size: int = 256,
                 tuning: Optional[_lib.Tuning] = None, stream=None):
        self.lib = _lib.load()
        if A.vals is not None and Bi.vals is not None and A.vals.dtype != Bi.vals.dtype:
            raise ValueError("A and B_i must share one value dtype")
        dt = (A.vals if A.vals is not None else Bi.vals)
        self.torch_dtype = torch.float64 if dt is None else dt.dtype
        if self.torch_dtype not in (torch.float32, torch.float64):
            raise ValueError("values must be float32 or float64")
        self.dtype = _lib.F64 if self.torch_dtype == torch.float64 else _lib.F32
        self.A, self.Bi = A, Bi
        self.device = A.colptr.device
        if offsets is None:
            offsets = [0, A.ncols]
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.offsets = offs
        self.P = offs.size - 1
        self.block_size = int(block_size)
        self._stream = stream
        handle = ctypes.c_void_p()
        a, b = A.c_struct(), Bi.c_struct()
        tun = ctypes.byref(tuning) if tuning is not None else None
        check(self.lib.spgemm_plan(ctypes.byref(a), ctypes.byref(b), self.dtype,
                                   offs.ctypes.data, self.P,
                                   self.block_size, tun, _stream(stream), ctypes.byref(handle)),
              "spgemm_plan")
        self.handle = handle
        self.C_colptr: Optional[torch.Tensor] = None
        self.nnzC: Optional[int] = None

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.spgemm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream):
        self._stream = stream
        check(self.lib.spgemm_plan_set_stream(self.handle, _stream(stream)), "set_stream")

    # -- queries ------------------------------------------------------------
    def stats(self) -> dict:
        s = _lib.Stats()
        check(self.lib.spgemm_plan_stats(self.handle, ctypes.byref(s)), "spgemm_plan_stats")
        out = {f: getattr(s, f) for f, _ in _lib.Stats._fields_ if f not in ("sym_bins", "num_bins")}
        out["sym_bins"] = list(s.sym_bins)
        out["num_bins"] = list(s.num_bins)
        return out

    def export(self) -> dict:
        st = self.stats()
        dev = self.device
        k, kt, nt, M = st["k"], st["kt"], st["nnz_At"], st["M"]
        H = torch.empty(k, dtype=torch.uint8, device=dev)
        mp = torch.empty(k, dtype=torch.int32, device=dev)
        atc = torch.empty(kt + 1, dtype=torch.int64, device=dev)
        atr = torch.empty(nt, dtype=torch.int32, device=dev)
        atv = torch.empty(nt, dtype=self.torch_dtype, device=dev)
        blocks = torch.empty((M, 2), dtype=torch.int64, device=dev)
        check(self.lib.spgemm_plan_export(self.handle, _ptr(H), _ptr(mp), _ptr(atc), _ptr(atr),
                                          _ptr(atv), _ptr(blocks)), "spgemm_plan_export")
        return {"H": H, "map": mp, "At_colptr": atc, "At_rowidx": atr, "At_vals": atv,
                "blocks": blocks, "stats": st}

    def export_bins(self):
        n = self.Bi.ncols
        flop = torch.empty(n, dtype=torch.int64, device=self.device)
        sb = torch.empty(n, dtype=torch.int32, device=self.device)
        nb = torch.empty(n, dtype=torch.int32, device=self.device)
        check(self.lib.spgemm_plan_export_bins(self.handle, _ptr(flop), _ptr(sb), _ptr(nb)),
              "spgemm_plan_export_bins")
        return flop, sb, nb

    # -- the phases -----------------------------------------------------------
    def symbolic(self) -> torch.Tensor:
        colptr = torch.empty(self.Bi.ncols + 1, dtype=torch.int64, device=self.device)
        nnz = ctypes.c_int64(0)
        check(self.lib.spgemm_symbolic(self.handle, _ptr(colptr), ctypes.byref(nnz)),
              "spgemm_symbolic")
        self.C_colptr = colptr
        self.nnzC = int(nnz.value)
        return colptr

    def numeric(self, A_vals: Optional[torch.Tensor] = None, B_vals: Optional[torch.Tensor] = None,
                out: Optional[tuple] = None):
        if self.nnzC is None:
            raise RuntimeError("numeric() needs symbolic() first")
        checks = []
        if A_vals is not None:
            checks.append((A_vals, "A_vals", self.torch_dtype, self.A.nnz))
        if B_vals is not None:
            checks.append((B_vals, "B_vals", self.torch_dtype, self.Bi.nnz))
        if out is None:
            # allocated here with the right device, dtype and length: nothing
            # to check (this runs between nnz(C_i) and the numeric launch, so
            # its host time is device idle time)
            rows = torch.empty(self.nnzC, dtype=torch.int32, device=self.device)
            vals = torch.empty(self.nnzC, dtype=self.torch_dtype, device=self.device)
        else:
            rows, vals = out
            checks.append((rows, "C_rowidx", torch.int32, self.nnzC))
            checks.append((vals, "C_vals", self.torch_dtype, self.nnzC))
        # the library reads and writes these through raw device pointers
        for t, what, dt, n in checks:
            if t.device != self.device or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{what} must be a contiguous {dt} tensor on {self.device}")
            if t.numel() < n:
                raise ValueError(f"{what} holds {t.numel()} elements, needs {n}")
        # addresses as plain ints (the argument types are void pointers)
        rc = self.lib.spgemm_numeric(self.handle,
                                     None if A_vals is None else A_vals.data_ptr(),
                                     None if B_vals is None else B_vals.data_ptr(),
                                     rows.data_ptr(), vals.data_ptr())
        if rc:
            check(rc, "spgemm_numeric")
        return rows, vals

    def backward(self, C_rowidx: torch.Tensor, dC: torch.Tensor,
                 A_vals: Optional[torch.Tensor] = None, B_vals: Optional[torch.Tensor] = None,
                 need_dA: bool = True, need_dB: bool = True):
        dA = torch.empty(self.A.nnz, dtype=self.torch_dtype, device=self.device) if need_dA else None
        dB = torch.empty(self.Bi.nnz, dtype=self.torch_dtype, device=self.device) if need_dB else None
        dC = dC.contiguous()
        check(self.lib.spgemm_backward(self.handle, _ptr(self.C_colptr), _ptr(C_rowidx),
                                       _ptr(A_vals), _ptr(B_vals), _ptr(dC), _ptr(dA), _ptr(dB)),
              "spgemm_backward")
        return dA, dB

    def run(self):
        """symbolic + numeric with the plan's values; returns C_i on the device."""
        colptr = self.symbolic()
        rows, vals = self.numeric()
        return DeviceCsc(self.A.nrows, self.Bi.ncols, colptr, rows, vals)


def spgemm(A: DeviceCsc, Bi: DeviceCsc, offsets=None, block_size: int = 256,
           tuning: Optional[_lib.Tuning] = None) -> DeviceCsc:
    """C_i = A * B_i in one call (plan, symbolic, numeric)."""
    with Plan(A, Bi, offsets, block_size, tuning) as p:
        return p.run()


class SpGEMM(torch.autograd.Function):
    """C_vals = values of A * B_i on the plan's fixed patterns, differentiable
    in A's and B_i's values.  Usage: ``SpGEMM.apply(A_vals, B_vals, plan)``
    after ``plan.symbolic()``; returns C's values (rows in plan.C_rowidx)."""

    @staticmethod
    def forward(ctx, A_vals, B_vals, plan: Plan):
        rows, vals = plan.numeric(A_vals.detach().contiguous(), B_vals.detach().contiguous())
        plan.C_rowidx = rows
        ctx.plan = plan
        ctx.save_for_backward(A_vals, B_vals)
        ctx.mark_non_differentiable(rows)
        return vals

    @staticmethod
    def backward(ctx, dC):
        A_vals, B_vals = ctx.saved_tensors
        plan: Plan = ctx.plan
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dA, dB = plan.backward(plan.C_rowidx, dC.contiguous(), A_vals.detach().contiguous(),
                               B_vals.detach().contiguous(), need_a, need_b)
        return dA, dB, None


def _io_table(io, plans):
    if len(io) != len(plans):
        raise ValueError("one io entry per plan")
    for p, d in zip(plans, io):
        nc = p.nnzC or 0  # a plan without symbolic() is refused by the library (ESTATE)
        for key, dt, n in (("A_vals", p.torch_dtype, p.A.nnz), ("B_vals", p.torch_dtype, p.Bi.nnz),
                           ("C_rowidx", torch.int32, nc), ("C_vals", p.torch_dtype, nc)):
            if d.get(key) is not None:
                _check_tensor(d[key], key, dt, n, device=p.device)
    arr = (_lib.BatchIO * len(io))()
    for t, d in enumerate(io):
        arr[t].A_vals = _ptr(d.get("A_vals"))
        arr[t].B_vals = _ptr(d.get("B_vals"))
        arr[t].C_rowidx = _ptr(d["C_rowidx"])
        arr[t].C_vals = _ptr(d["C_vals"])
        arr[t].dep_A = int(d.get("dep_A", -1))
        arr[t].dep_B = int(d.get("dep_B", -1))
    return arr


def batched(plans, io, mode: int = 0, stream=None):
    """spgemm_batched(count, plans, io, mode, stream): the numeric phase of
    the planned products as one launch DAG (mode 0), captured into a hipGraph
    and launched (1), or that graph relaunched (2).  ``io`` as for
    :class:`Batch`; the caller keeps its tensors alive while the library
    keeps the batch (until one of the plans is closed)."""
    lib = _lib.load()
    plans = list(plans)
    handles = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    check(lib.spgemm_batched(len(plans), handles, _io_table(io, plans), mode, _stream(stream)),
          "spgemm_batched")


class Batch:
    """Numeric phase of many planned products as one dependency DAG of the
    per-bin kernels, optionally captured into a hipGraph and replayed
    (spgemm_batch_create / spgemm_batch_run).

    ``io`` has one dict per plan with keys ``C_rowidx``, ``C_vals`` (output
    tensors), optional ``A_vals``/``B_vals`` (None = the plan's values) and
    optional ``dep_A``/``dep_B`` (index of an earlier product whose C is this
    product's A or B, else -1).  Tensors are kept alive by the batch.
    """

    def __init__(self, plans, io, tuning: Optional[_lib.Tuning] = None):
        self.lib = _lib.load()
        self.plans = list(plans)
        self.io = [dict(x) for x in io]
        n = len(self.plans)
        arr = _io_table(self.io, self.plans)
        handles = (ctypes.c_void_p * n)(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        tun = ctypes.byref(tuning) if tuning is not None else None
        check(self.lib.spgemm_batch_create(n, handles, arr, tun, ctypes.byref(h)),
              "spgemm_batch_create")
        self.handle = h

    def run(self, mode: int = 0, stream=None):
        """mode 0: launch; 1: capture into a hipGraph and launch; 2: replay.
        Capture needs a stream other than the null stream."""
        check(self.lib.spgemm_batch_run(self.handle, mode, _stream(stream)), "spgemm_batch_run")

    def check(self):
        """Synchronises the device and raises if a launch failed."""
        check(self.lib.spgemm_batch_check(self.handle), "spgemm_batch_check")

    def info(self):
        """(side streams, kernels one run enqueues)."""
        ns, nl = ctypes.c_int64(), ctypes.c_int64()
        check(self.lib.spgemm_batch_info(self.handle, ctypes.byref(ns), ctypes.byref(nl)),
              "spgemm_batch_info")
        return ns.value, nl.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.spgemm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def galerkin_chain(A0: DeviceCsc, levels, block_size: int = 64,
                   tuning: Optional[_lib.Tuning] = None):
    """The AMG Galerkin products A_{l+1} = P_l^T (A_l P_l) for the given
    levels [(P_0, Pt_0), (P_1, Pt_1), ...] (device CSC prolongators and their
    transposes), run once through the plain path.  Returns (plans, io,
    outputs): the plans of the 2*len(levels) products in order, batch I/O
    with the chain's dependencies (product 2l gathers A_l's values, which
    for l > 0 are product 2l-1's output; product 2l+1 reads A_l P_l from
    product 2l), and the device results of the run (the coarse operators
    are outputs[2l+1]).  The batch writes into those same output tensors.""" 
    plans, io, outs = [], [], []
    A = A0
    for lvl, (P, Pt) in enumerate(levels):
        p1 = Plan(A, P, None, block_size, tuning)
        AP = p1.run()
        plans.append(p1)
        io.append({"A_vals": A.vals, "B_vals": None,
                   "C_rowidx": AP.rowidx, "C_vals": AP.vals,
                   "dep_A": 2 * lvl - 1 if lvl > 0 else -1, "dep_B": -1})
        outs.append(AP)
        p2 = Plan(Pt, AP, None, block_size, tuning)
        Ac = p2.run()
        plans.append(p2)
        io.append({"A_vals": None, "B_vals": AP.vals, "C_rowidx": Ac.rowidx, "C_vals": Ac.vals,
                   "dep_A": -1, "dep_B": 2 * lvl})
        outs.append(Ac)
        A = Ac
    return plans, io, outs


def _dtype_of(t: torch.Tensor) -> int:
    return _lib.F64 if t.dtype == torch.float64 else _lib.F32


def row_block(B: DeviceCsc, r0: int, r1: int, stream=None) -> DeviceCsc:
    """B(r0:r1, :) with B's global row ids (spgemm_row_block); reads the
    block's entry count back (one synchronisation)."""
    lib = _lib.load()
    dev = B.colptr.device
    cap = max(B.nnz, 1)
    colptr = torch.empty(B.ncols + 1, dtype=torch.int64, device=dev)
    rows = torch.empty(cap, dtype=torch.int32, device=dev)
    vals = torch.empty(cap, dtype=B.vals.dtype, device=dev)
    c = B.c_struct()
    check(lib.spgemm_row_block(ctypes.byref(c), _dtype_of(B.vals), int(r0), int(r1),
                               _ptr(colptr), _ptr(rows), _ptr(vals), _stream(stream)),
          "spgemm_row_block")
    nnz = int(colptr[-1])
    return DeviceCsc(B.nrows, B.ncols, colptr, rows[:nnz], vals[:nnz])


def sum_parts(parts, block_size: int = 256, tuning: Optional[_lib.Tuning] = None,
              stream=None) -> DeviceCsc:
    """Sum of partial results of one shape: the stack [C_0 ... C_{P-1}] times
    the selector [I; ...; I] (spgemm_stack_parts), through the plain path."""
    lib = _lib.load()
    P = len(parts)
    m, n = parts[0].nrows, parts[0].ncols
    dev = parts[0].colptr.device
    vdt = parts[0].vals.dtype
    total = sum(p.nnz for p in parts)
    st_colptr = torch.empty(P * n + 1, dtype=torch.int64, device=dev)
    st_rows = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
    st_vals = torch.empty(max(total, 1), dtype=vdt, device=dev)
    se_colptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    se_rows = torch.empty(max(P * n, 1), dtype=torch.int32, device=dev)
    se_vals = torch.empty(max(P * n, 1), dtype=vdt, device=dev)
    arr = (_lib.Csc * P)(*[p.c_struct() for p in parts])
    check(lib.spgemm_stack_parts(P, arr, _dtype_of(parts[0].vals), _ptr(st_colptr), _ptr(st_rows),
                                 _ptr(st_vals), _ptr(se_colptr), _ptr(se_rows), _ptr(se_vals),
                                 _stream(stream)), "spgemm_stack_parts")
    stack = DeviceCsc(m, P * n, st_colptr, st_rows[:total], st_vals[:total])
    sel = DeviceCsc(P * n, n, se_colptr, se_rows[:P * n], se_vals[:P * n])
    return spgemm(stack, sel, None, block_size, tuning)


def outer_product(A: DeviceCsc, B: DeviceCsc, offsets, block_size: int = 256,
                  tuning: Optional[_lib.Tuning] = None) -> DeviceCsc:
    """C = A * B by the outer-product 1D algorithm (Alg. 3) on one GPU: the
    inner dimension split at `offsets` (A's column partitions = B's row
    blocks), one partial product A * B(K_r, :) per block (its plan selects
    A's columns K_r by Alg. 1 and 2), then the partial results summed."""
    offs = np.asarray(offsets, dtype=np.int64)
    parts = []
    for r in range(len(offs) - 1):
        Br = row_block(B, int(offs[r]), int(offs[r + 1]))
        parts.append(spgemm(A, Br, offs, block_size, tuning))
    return sum_parts(parts, block_size, tuning)

