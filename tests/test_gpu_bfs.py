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
