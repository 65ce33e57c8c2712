"""Full-size GPU parity: the R-MAT scale-18 square (FP64 and FP32) on sampled
columns plus invariants over the whole product, and the AMG Galerkin
hierarchy of the 64^3 Laplacian against its closed form."""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _gather_columns(C, cols):
    """Row ids and values of the chosen columns of a device CSC, on the host."""
    cp = C.colptr.cpu().numpy()
    idx = np.concatenate([np.arange(cp[j], cp[j + 1]) for j in cols])
    it = torch.as_tensor(idx, device="cuda")
    ptr = np.concatenate([[0], np.cumsum([cp[j + 1] - cp[j] for j in cols])])
    return ptr, C.rowidx[it].cpu().numpy(), C.vals[it].double().cpu().numpy()


@pytest.fixture(scope="module")
def rmat18():
    return synth.workload("rmat18")["A"]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rmat18_square_sampled(rmat18, dtype):
    A = rmat18 if dtype == torch.float64 else synth.as_fp32(rmat18)
    Ad = spg.DeviceCsc.from_host(A, dtype=dtype)
    with spg.Plan(Ad, Ad, None, 256) as p:
        C = p.run()
        st = p.stats()
        flop, sbin, nbin = p.export_bins()
    torch.cuda.synchronize()
    print("rmat18", dtype, "flops", st["flops"], "nnz_C", st["nnz_C"], "sym bins",
          st["sym_bins"], "num bins", st["num_bins"], flush=True)
    # whole-product invariants
    colnnz = np.diff(A.colptr)
    rownnz = np.bincount(A.rowidx, minlength=A.nrows)
    assert st["flops"] == int(colnnz @ rownnz)
    fl = flop.cpu().numpy()
    counts = np.diff(C.colptr.cpu().numpy())
    assert (counts <= fl).all() and ((counts == 0) == (fl == 0)).all()
    # sampled columns: random, the heaviest, and one of every bin
    rng = np.random.default_rng(0)
    nb = nbin.cpu().numpy()
    cols = set(rng.choice(A.ncols, 150, replace=False).tolist())
    cols |= set(np.argsort(fl)[-12:].tolist())
    for b in range(7):
        idx = np.nonzero(nb == b)[0]
        if idx.size:
            cols |= set(rng.choice(idx, min(5, idx.size), replace=False).tolist())
    cols = sorted(cols)
    ref = oracle.spgemm(A, A, cols)
    ptr, rows, vals = _gather_columns(C, cols)
    assert np.array_equal(ptr, ref.colptr)
    assert np.array_equal(rows, ref.rowidx)
    assert_values(vals, ref.vals, ref.absvals, dtype == torch.float64)
    # row-sum invariant over the whole product: C*1 = A*(A*1)
    Acol = torch.as_tensor(np.repeat(np.arange(A.ncols), colnnz), device="cuda")
    Arow = Ad.rowidx.long()
    Av = Ad.vals.double()
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda").index_add_(0, Arow, Av)
    z = torch.zeros(A.nrows, dtype=torch.float64, device="cuda").index_add_(0, Arow, Av * y[Acol])
    cx = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    n = C.rowidx.numel()
    step = 1 << 27
    for s0 in range(0, n, step):
        cx.index_add_(0, C.rowidx[s0:s0 + step].long(), C.vals[s0:s0 + step].double())
    rel = (cx - z).abs().max().item() / z.abs().max().item()
    print("row-sum invariant rel err", rel, flush=True)
    assert rel <= (1e-10 if dtype == torch.float64 else 1e-5)


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
