"""Multi-source breadth-first search (the forward search of batched
betweenness centrality, Sec. II-C and Sec. IV-C): every level is one product
N = A * F of the graph with the frontier, and the next frontier keeps the
vertices a source has not reached.  On the CPU the levels from the oracle's
product are pinned against shortest-path distances and a brute-force count
of shortest paths."""

import numpy as np
from scipy.sparse import csc_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth


def _levels(A, F, product):
    visited = np.zeros((A.nrows, F.ncols), dtype=bool)
    visited[F.rowidx, np.repeat(np.arange(F.ncols), np.diff(F.colptr))] = True
    out = [F]
    while F.nnz:
        F = synth.next_frontier(product(A, F), visited)
        out.append(F)
    return out


def test_frontiers_are_distance_levels_with_path_counts():
    A = synth.unit_values(synth.rmat(7, 8, 0.57, 0.19, 0.19, 0.05, seed=11))
    n = A.nrows
    F0 = synth.bfs_sources(n, 16, seed=3)
    src = F0.rowidx.copy()
    levels = _levels(A, F0, oracle.spgemm)
    # edge j -> i for every stored A(i, j)
    G = csc_matrix((np.ones(A.nnz), A.rowidx, A.colptr), shape=(n, n)).T.tocsr()
    dist = shortest_path(G, unweighted=True, indices=src)
    for s in range(F0.ncols):
        # brute-force shortest-path counts by increasing distance
        sigma = np.zeros(n)
        sigma[src[s]] = 1
        order = np.argsort(dist[s])
        for v in order:
            if not np.isfinite(dist[s, v]) or v == src[s]:
                continue
            preds = [u for u in G[:, [v]].nonzero()[0] if dist[s, u] == dist[s, v] - 1]
            sigma[v] = sum(sigma[u] for u in preds)
        for lvl, F in enumerate(levels):
            lo, hi = F.colptr[s], F.colptr[s + 1]
            rows = F.rowidx[lo:hi]
            expect = np.nonzero(dist[s] == lvl)[0]
            assert np.array_equal(rows, expect), (s, lvl)
            assert np.array_equal(F.vals[lo:hi], sigma[rows]), (s, lvl)
    assert levels[-1].nnz == 0 and len(levels) >= 3


def test_sources_are_distinct_unit_columns():
    F = synth.bfs_sources(1000, 64, seed=5)
    assert F.ncols == 64 and np.all(np.diff(F.colptr) == 1)
    assert len(np.unique(F.rowidx)) == 64 and np.all(F.vals == 1)
