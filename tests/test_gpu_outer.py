"""GPU parity of the outer-product form (Alg. 3) through the C ABI: row
blocks of B with global row ids, the stack of partial results with its
selector, and C = sum_r A(:, K_r) * B(K_r, :) against the oracle's plain
product (pattern bit-exact, FP64 values per entry within 1e-12)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _rand(rng, m, n, density):
    mask = rng.random((m, n)) < density
    r, c = np.nonzero(mask)
    return synth.from_triplets(m, n, r, c, rng.uniform(-1, 1, r.size))


@pytest.mark.parametrize("r0,r1", [(0, 300), (0, 0), (100, 101), (37, 211), (299, 300)])
def test_row_block_keeps_global_rows(r0, r1):
    rng = np.random.default_rng(r0 * 7 + r1)
    B = _rand(rng, 300, 120, 0.05)
    Bd = spg.DeviceCsc.from_host(B)
    Br = spg.row_block(Bd, r0, r1)
    D = B.to_dense()
    D[:r0, :] = 0
    D[r1:, :] = 0
    ref = synth.from_triplets(300, 120, *np.nonzero(D), D[np.nonzero(D)])
    assert np.array_equal(Br.colptr.cpu().numpy(), ref.colptr)
    assert np.array_equal(Br.rowidx.cpu().numpy(), ref.rowidx)
    assert np.array_equal(Br.vals.cpu().numpy(), ref.vals)


def test_row_block_rejects_bad_ranges():
    B = spg.DeviceCsc.from_host(synth.erdos_renyi(50, 20, 3, seed=1))
    with pytest.raises(spg.SpgemmError):
        spg.row_block(B, 10, 5)
    with pytest.raises(spg.SpgemmError):
        spg.row_block(B, 0, 51)


def test_stack_and_selector_sum_the_parts():
    rng = np.random.default_rng(3)
    parts = [_rand(rng, 90, 40, d) for d in (0.05, 0.0, 0.2, 0.1)]
    got = spg.sum_parts([spg.DeviceCsc.from_host(p) for p in parts], block_size=16)
    dense = sum(p.to_dense() for p in parts)
    pattern = sum((p.to_dense() != 0).astype(int) for p in parts) > 0
    r, c = np.nonzero(pattern.T)  # column-major order
    assert np.array_equal(got.colptr.cpu().numpy(),
                          np.concatenate([[0], np.cumsum(pattern.sum(axis=0))]))
    assert np.array_equal(got.rowidx.cpu().numpy(), c)
    absd = sum(np.abs(p.to_dense()) for p in parts)
    assert_values(got.vals.cpu().numpy(), dense.T[pattern.T], absd.T[pattern.T], True)


@pytest.mark.parametrize("P", [1, 3, 8])
def test_outer_product_equals_the_plain_product(P):
    A = synth.rmat(10, 8, 0.57, 0.19, 0.19, 0.05, seed=21)
    B = synth.erdos_renyi(A.ncols, 300, 6, seed=22)
    offs = synth.partition_offsets(A.ncols, P)
    C = spg.outer_product(spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B), offs, 32)
    ref = oracle.spgemm(A, B)
    assert np.array_equal(C.colptr.cpu().numpy(), ref.colptr)
    assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)
    assert_values(C.vals.cpu().numpy(), ref.vals, ref.absvals, True)


@pytest.mark.parametrize("left", [False, True])
def test_galerkin_right_product_both_forms(left):
    """The right product of a Galerkin step, X * P with X = A (this
    project's order) or X = P^T A (the paper's), by both 1D forms."""
    A = synth.laplacian3d(16)
    Pm = synth.aggregation3d(16)
    X = oracle.spgemm(synth.aggregation3d_t(16), A) if left else A
    ref = oracle.spgemm(X, Pm)
    Xd, Pd = spg.DeviceCsc.from_host(X), spg.DeviceCsc.from_host(Pm)
    offs = synth.partition_offsets(X.ncols, 4)
    C = spg.outer_product(Xd, Pd, offs, 64)
    assert np.array_equal(C.colptr.cpu().numpy(), ref.colptr)
    assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)
    assert_values(C.vals.cpu().numpy(), ref.vals, ref.absvals, True)
    # the column-wise form over the same number of blocks, stitched
    coffs = synth.partition_offsets(Pm.ncols, 4)
    cols = []
    for i in range(4):
        Bi = synth.column_slice(Pm, int(coffs[i]), int(coffs[i + 1]))
        cols.append(spg.spgemm(Xd, spg.DeviceCsc.from_host(Bi), offs, 64).to_host())
    rows = np.concatenate([c.rowidx for c in cols])
    assert np.array_equal(rows, ref.rowidx)


def test_outer_product_fp32():
    """The FP32 instances of the row-block and stacking kernels."""
    A = synth.as_fp32(synth.erdos_renyi(600, 400, 5, seed=41))
    B = synth.as_fp32(synth.erdos_renyi(400, 150, 4, seed=42))
    offs = synth.partition_offsets(400, 5)
    Ad = spg.DeviceCsc.from_host(A, dtype=torch.float32)
    Bd = spg.DeviceCsc.from_host(B, dtype=torch.float32)
    C = spg.outer_product(Ad, Bd, offs, 16)
    ref = oracle.spgemm(A, B)
    assert C.vals.dtype == torch.float32
    assert np.array_equal(C.colptr.cpu().numpy(), ref.colptr)
    assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)
    assert_values(C.vals.cpu().numpy(), ref.vals, ref.absvals, False)
