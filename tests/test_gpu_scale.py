"""Full-size GPU parity: the R-MAT scale-18 square (FP64 and FP32) compared
with the oracle column by column over the WHOLE product (column pointers
and row ids bit for bit, FP64 values per entry, FP32 values normwise), in
slabs of columns so the host never holds two copies of C; and the AMG
Galerkin hierarchy of the 64^3 Laplacian against its closed form."""

import time

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import fp64_entry_ok

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")

# entries of C compared per slab (oracle output + the GPU's copy on the host)
SLAB_ENTRIES = 48 << 20


@pytest.fixture(scope="module")
def rmat18():
    return synth.workload("rmat18")["A"]


def _slabs(colptr, limit):
    """Consecutive column ranges holding at most `limit` entries each (a
    single column may exceed it)."""
    n = colptr.size - 1
    c0 = 0
    while c0 < n:
        c1 = int(np.searchsorted(colptr, colptr[c0] + limit, side="right")) - 1
        c1 = min(max(c1, c0 + 1), n)
        yield c0, c1
        c0 = c1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rmat18_square_every_column(rmat18, dtype):
    A = rmat18 if dtype == torch.float64 else synth.as_fp32(rmat18)
    fp64 = dtype == torch.float64
    t0 = time.time()
    Ad = spg.DeviceCsc.from_host(A, dtype=dtype)
    with spg.Plan(Ad, Ad, None, 256) as p:
        C = p.run()
        st = p.stats()
        flop, _, _ = p.export_bins()
    torch.cuda.synchronize()
    print(f"rmat18 {dtype} flops {st['flops']} nnz_C {st['nnz_C']} sym bins {st['sym_bins']} "
          f"num bins {st['num_bins']} (GPU {time.time() - t0:.1f} s)", flush=True)
    colnnz = np.diff(A.colptr)
    rownnz = np.bincount(A.rowidx, minlength=A.nrows)
    assert st["flops"] == int(colnnz @ rownnz)  # Sec. III-B inner-product identity
    assert np.array_equal(flop.cpu().numpy(), oracle.column_flops(A, A))
    # column pointers of the whole product, bit for bit
    counts = oracle.spgemm_counts(A, A)
    ref_colptr = np.zeros(A.ncols + 1, dtype=np.int64)
    np.cumsum(counts, out=ref_colptr[1:])
    gpu_colptr = C.colptr.cpu().numpy()
    assert np.array_equal(gpu_colptr, ref_colptr)
    print(f"colptr equal ({time.time() - t0:.1f} s)", flush=True)
    # every column's row ids and values, slab by slab
    err2, ref2, worst, nslab = 0.0, 0.0, 0.0, 0
    for c0, c1 in _slabs(ref_colptr, SLAB_ENTRIES):
        ref = oracle.spgemm(A, A, np.arange(c0, c1))
        lo, hi = int(ref_colptr[c0]), int(ref_colptr[c1])
        assert np.array_equal(ref.colptr + lo, ref_colptr[c0:c1 + 1])
        rows = C.rowidx[lo:hi].cpu().numpy()
        assert np.array_equal(rows, ref.rowidx), f"row ids differ in columns [{c0}, {c1})"
        vals = C.vals[lo:hi].double().cpu().numpy()
        if fp64:
            ok, e, nbad = fp64_entry_ok(vals, ref.vals, ref.absvals)
            assert ok, f"{nbad} FP64 entries beyond 1e-12 in columns [{c0}, {c1}) (max err {e:g})"
            worst = max(worst, e)
        else:
            err2 += float(np.sum((vals - ref.vals) ** 2))
            ref2 += float(np.sum(ref.vals ** 2))
        nslab += 1
        del ref, rows, vals
    if not fp64:
        r = (err2 ** 0.5) / (ref2 ** 0.5)
        print(f"FP32 normwise error {r:.3e}", flush=True)
        assert r <= 1e-5
    print(f"all {A.ncols} columns compared in {nslab} slabs ({time.time() - t0:.1f} s), "
          f"oracle threads {oracle.threads()}, max abs err {worst:g}", flush=True)


def test_amg_galerkin_hierarchy_64():
    """A_{l+1} = P^T (A_l P) for the 64^3 7-point Laplacian with 2x2x2
    aggregation, four levels, each product through the plain path; every
    level is exact (integers): A_l P holds 4^l*{3,-1} and
    A_{l+1} = 4^(l+1) L_{64/2^(l+1)}."""
    n = 64
    A = synth.laplacian3d(n)
    Ad = spg.DeviceCsc.from_host(A)
    for level in range(4):
        P = spg.DeviceCsc.from_host(synth.aggregation3d(n))
        Pt = spg.DeviceCsc.from_host(synth.aggregation3d_t(n))
        AP = spg.spgemm(Ad, P, None, 64)
        apv = torch.unique(AP.vals).cpu().numpy()
        assert set(apv.tolist()) == {3.0 * 4 ** level, -1.0 * 4 ** level}
        Ac = spg.spgemm(Pt, AP, None, 64)
        n //= 2
        ref = synth.laplacian3d(n)
        assert Ac.nnz == 7 * n ** 3 - 6 * n ** 2
        assert np.array_equal(Ac.colptr.cpu().numpy(), ref.colptr)
        assert np.array_equal(Ac.rowidx.cpu().numpy(), ref.rowidx)
        assert np.array_equal(Ac.vals.cpu().numpy(), 4.0 ** (level + 1) * ref.vals)
        Ad = Ac
