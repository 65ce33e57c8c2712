"""GPU parity of the multi-source search workload: every level's product
N = A * F (frontier of 256 sources on an unweighted R-MAT graph) through the
C ABI against the oracle.  The values are shortest-path counts (integers),
so rows and values must match exactly."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def test_every_level_of_a_256_source_search():
    A = synth.unit_values(synth.rmat(10, 16, 0.57, 0.19, 0.19, 0.05, seed=13))
    F = synth.bfs_sources(A.ncols, 256, seed=17)
    visited = np.zeros((A.nrows, F.ncols), dtype=bool)
    visited[F.rowidx, np.arange(F.ncols)] = True
    Ad = spg.DeviceCsc.from_host(A)
    levels = 0
    while F.nnz:
        ref = oracle.spgemm(A, F)
        with spg.Plan(Ad, spg.DeviceCsc.from_host(F), None, 64) as p:
            colptr = p.symbolic()
            rows, vals = p.numeric()
            print("level", levels, "nnz(F)", F.nnz, "nnz(N)", ref.colptr[-1],
                  "num bins", p.stats()["num_bins"], flush=True)
        assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
        assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
        assert np.array_equal(vals.cpu().numpy(), ref.vals)
        F = synth.next_frontier(ref, visited)
        levels += 1
    assert levels >= 4


def _search_levels(A, F, b, tun=None):
    """Runs every level of the search through the C ABI and compares it with
    the oracle; returns the numeric bin counts seen at each level."""
    visited = np.zeros((A.nrows, F.ncols), dtype=bool)
    visited[F.rowidx, np.arange(F.ncols)] = True
    Ad = spg.DeviceCsc.from_host(A)
    bins = []
    while F.nnz:
        ref = oracle.spgemm(A, F)
        with spg.Plan(Ad, spg.DeviceCsc.from_host(F), None, b, tuning=tun) as p:
            colptr = p.symbolic()
            rows, vals = p.numeric()
            st = p.stats()
        print("level", len(bins), "nnz(F)", F.nnz, "nnz(N)", int(ref.colptr[-1]),
              "num bins", st["num_bins"], flush=True)
        assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
        assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
        assert np.array_equal(vals.cpu().numpy(), ref.vals)
        bins.append(st["num_bins"])
        F = synth.next_frontier(ref, visited)
    return np.array(bins)


@pytest.mark.parametrize("dense_first", [0, 1 << 14])
def test_every_level_of_a_1024_source_search_scale13(dense_first):
    """1024 sources on R-MAT scale 13: the middle levels hold output columns
    with more than 2048 entries (the dense bin); with the dense-first bin
    lowered to 2^14 products, that bin is used as well."""
    A = synth.unit_values(synth.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, seed=13))
    F = synth.bfs_sources(A.ncols, 1024, seed=17)
    tun = spg.tuning(dense_first_flop=dense_first) if dense_first else None
    bins = _search_levels(A, F, 64, tun)
    assert len(bins) >= 5
    assert bins[:, 6].max() > 0
    if dense_first:
        assert bins[:, 7].max() > 0


def test_every_level_of_the_4096_source_search_scale16():
    """The search workload itself (R-MAT scale 16, 4096 sources): every level
    equals the oracle, including the levels whose output columns fill the
    dense and dense-first bins (at least 2^18 products per column)."""
    w = synth.workload("bfs_rmat16_4096")
    bins = _search_levels(w["A"], w["B"], w["b"])
    assert bins[:, 6].max() > 0 and bins[:, 7].max() > 0
