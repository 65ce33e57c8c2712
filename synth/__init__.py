"""Seeded synthetic inputs for the local SpGEMM path.

This module only *draws* matrices: it holds none of the product's arithmetic.
Both the CPU oracle (through the tests) and the HIP path (through the tests and
the benchmark) consume what it produces; neither imports the other.

Every matrix is returned as a :class:`CSC` with

* ``colptr`` int64[ncols+1], ``rowidx`` int32[nnz] (ascending and unique inside
  each column), ``vals`` float64[nnz] (FP32 runs round them with
  :func:`as_fp32`).

The recipes (the paper's data sets are not available; these stand in for
them):

* ``laplacian2d(n)``: 5-point stencil on an n x n grid, 4 on the diagonal and
  -1 per grid neighbour, index ``x + n*y``.
* ``laplacian3d(n)``: 7-point stencil on an n^3 grid, 6 on the diagonal and -1
  per face neighbour (Dirichlet rows are not modified), index
  ``x + n*y + n*n*z``.
* ``aggregation3d(n)``: piecewise-constant prolongator on 2x2x2 aggregates,
  ``P(i, J(i)) = 1`` with ``J = x//2 + (n/2)*(y//2) + (n/2)^2*(z//2)``; one
  stored entry per row (the property the paper's restriction operators have,
  Table 3).  ``aggregation3d_t(n)`` is its transpose, drawn directly.
* ``erdos_renyi(m, n, d, seed)``: exactly ``d`` distinct rows per column,
  uniform over the d-subsets, values U(lo, hi) drawn in CSC order.
* ``rmat(scale, edge_factor, a, b, c, d, seed)``: ``edge_factor * 2^scale``
  edges; at each of ``scale`` levels (most significant bit first) one uniform
  draw u picks the quadrant (row bit, col bit): u < a -> (0,0), u < a+b ->
  (0,1), u < a+b+c -> (1,0), else (1,1).  No noise, no vertex permutation,
  self loops kept, not symmetrised; duplicate edges merged, then one U(0,1)
  value per unique entry in CSC order.
* ``sign_sketch(k, n, per_row, seed)``: every row holds ``per_row`` distinct
  columns, each value +1/2 or -1/2 with equal probability.
* ``er_batch(count, seed)``: ``count`` independent square ER pairs (A_t, B_t)
  with ``n_t = round(exp U(ln 1e3, ln 5e4))`` and
  ``d_t = round(exp U(ln 4, ln 32))``, values U(-1, 1).
* ``uniform_values(count, seed)``: U(-1, 1) values, e.g. an upstream gradient
  laid on a given sparsity pattern.
* ``partition_offsets(k, P)``: the 1D column partition ``o_r = floor(r*k/P)``.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSC",
    "as_fp32",
    "laplacian2d",
    "laplacian3d",
    "aggregation3d",
    "aggregation3d_t",
    "erdos_renyi",
    "rmat",
    "sign_sketch",
    "er_batch",
    "uniform_values",
    "partition_offsets",
    "column_slice",
    "transpose",
    "permute_symmetric",
    "from_triplets",
    "workload",
]


@dataclasses.dataclass
class CSC:
    nrows: int
    ncols: int
    colptr: np.ndarray  # int64[ncols+1]
    rowidx: np.ndarray  # int32[nnz]
    vals: np.ndarray  # float64[nnz] (or float32 after as_fp32)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.nrows, self.ncols), dtype=np.float64)
        for j in range(self.ncols):
            lo, hi = int(self.colptr[j]), int(self.colptr[j + 1])
            out[self.rowidx[lo:hi], j] = self.vals[lo:hi]
        return out


def from_triplets(nrows: int, ncols: int, rows, cols, vals) -> CSC:
    """CSC from (row, col, value) triplets without duplicates."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in triplets")
    colptr = np.zeros(ncols + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr).astype(np.int64)
    return CSC(nrows, ncols, colptr, rows.astype(np.int32), vals)


def as_fp32(M: CSC) -> CSC:
    """Same pattern, values rounded to float32."""
    return CSC(M.nrows, M.ncols, M.colptr, M.rowidx, M.vals.astype(np.float32))


def column_slice(M: CSC, lo: int, hi: int) -> CSC:
    """Columns [lo, hi) of M as a CSC of its own (the 1D slice B_i)."""
    a, b = int(M.colptr[lo]), int(M.colptr[hi])
    return CSC(M.nrows, hi - lo, (M.colptr[lo:hi + 1] - a).astype(np.int64),
               M.rowidx[a:b].copy(), M.vals[a:b].copy())


def column_subset(M: CSC, cols) -> CSC:
    """The chosen columns of M, in the given order."""
    cols = np.asarray(cols, dtype=np.int64)
    lens = M.colptr[cols + 1] - M.colptr[cols]
    colptr = np.zeros(cols.size + 1, dtype=np.int64)
    np.cumsum(lens, out=colptr[1:])
    idx = np.concatenate([np.arange(M.colptr[c], M.colptr[c + 1]) for c in cols]) \
        if cols.size else np.zeros(0, np.int64)
    return CSC(M.nrows, cols.size, colptr, M.rowidx[idx].copy(), M.vals[idx].copy())


def transpose(M: CSC) -> CSC:
    """M^T in CSC (a stable counting sort of the entries by row)."""
    cols = np.repeat(np.arange(M.ncols, dtype=np.int64), np.diff(M.colptr))
    order = np.argsort(M.rowidx, kind="stable")
    colptr = np.zeros(M.nrows + 1, dtype=np.int64)
    colptr[1:] = np.cumsum(np.bincount(M.rowidx, minlength=M.nrows))
    return CSC(M.ncols, M.nrows, colptr, cols[order].astype(np.int32), M.vals[order].copy())


def permute_symmetric(M: CSC, seed: int) -> CSC:
    """Q M Q^T for a seeded uniformly random permutation Q (square M): entry
    (i, j) moves to (q[i], q[j])."""
    if M.nrows != M.ncols:
        raise ValueError("a symmetric permutation needs a square matrix")
    q = np.random.default_rng(seed).permutation(M.nrows).astype(np.int64)
    cols = np.repeat(np.arange(M.ncols, dtype=np.int64), np.diff(M.colptr))
    return from_triplets(M.nrows, M.ncols, q[M.rowidx.astype(np.int64)], q[cols], M.vals)


def partition_offsets(k: int, P: int) -> np.ndarray:
    return np.array([(r * k) // P for r in range(P + 1)], dtype=np.int64)


# --------------------------------------------------------------------------
# structured matrices
# --------------------------------------------------------------------------

def laplacian2d(n: int) -> CSC:
    x, y = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    x = x.ravel()
    y = y.ravel()
    idx = x + n * y
    rows, cols, vals = [idx], [idx], [np.full(idx.size, 4.0)]
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        ok = (x + dx >= 0) & (x + dx < n) & (y + dy >= 0) & (y + dy < n)
        rows.append((x + dx + n * (y + dy))[ok])
        cols.append(idx[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    return from_triplets(n * n, n * n, np.concatenate(rows), np.concatenate(cols),
                         np.concatenate(vals))


def _grid3(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def laplacian3d(n: int) -> CSC:
    x, y, z = _grid3(n)
    idx = x + n * y + n * n * z
    rows, cols, vals = [idx], [idx], [np.full(idx.size, 6.0)]
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        ok = ((x + dx >= 0) & (x + dx < n) & (y + dy >= 0) & (y + dy < n)
              & (z + dz >= 0) & (z + dz < n))
        rows.append((x + dx + n * (y + dy) + n * n * (z + dz))[ok])
        cols.append(idx[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    return from_triplets(n ** 3, n ** 3, np.concatenate(rows), np.concatenate(cols),
                         np.concatenate(vals))


def _aggregate_ids(n: int):
    if n % 2:
        raise ValueError("aggregation needs an even grid size")
    x, y, z = _grid3(n)
    h = n // 2
    return x + n * y + n * n * z, x // 2 + h * (y // 2) + h * h * (z // 2)


def aggregation3d(n: int) -> CSC:
    """n^3 x (n/2)^3 prolongator P, one entry (1.0) per row."""
    i, J = _aggregate_ids(n)
    return from_triplets(n ** 3, (n // 2) ** 3, i, J, np.ones(i.size))


def aggregation3d_t(n: int) -> CSC:
    """(n/2)^3 x n^3 restriction P^T, one entry (1.0) per column."""
    i, J = _aggregate_ids(n)
    return from_triplets((n // 2) ** 3, n ** 3, J, i, np.ones(i.size))


# --------------------------------------------------------------------------
# random matrices
# --------------------------------------------------------------------------

def _distinct_per_line(rng, lines: int, per: int, universe: int) -> np.ndarray:
    """lines x per array of sorted, distinct draws from range(universe).

    Whole lines that contain a repeat are redrawn, so every line is uniform
    over the per-subsets of the universe.
    """
    if per > universe:
        raise ValueError("more distinct draws than the universe holds")
    out = np.sort(rng.integers(0, universe, size=(lines, per)), axis=1)
    while True:
        bad = np.nonzero((out[:, 1:] == out[:, :-1]).any(axis=1))[0] if per > 1 else np.zeros(0, int)
        if bad.size == 0:
            return out
        out[bad] = np.sort(rng.integers(0, universe, size=(bad.size, per)), axis=1)


def erdos_renyi(m: int, n: int, d: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> CSC:
    rng = np.random.default_rng(seed)
    rows = _distinct_per_line(rng, n, d, m)
    colptr = np.arange(n + 1, dtype=np.int64) * d
    vals = rng.uniform(lo, hi, size=n * d)
    return CSC(m, n, colptr, rows.ravel().astype(np.int32), vals)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, d: float,
         seed: int) -> CSC:
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    rng = np.random.default_rng(seed)
    n = 1 << scale
    E = edge_factor * n
    rows = np.zeros(E, dtype=np.int64)
    cols = np.zeros(E, dtype=np.int64)
    for _ in range(scale):
        u = rng.random(E)
        rbit = u >= a + b
        cbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)
        rows = (rows << 1) | rbit
        cols = (cols << 1) | cbit
    key = np.unique(cols * n + rows)
    cols = key // n
    rows = key - cols * n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr).astype(np.int64)
    vals = rng.random(key.size)
    return CSC(n, n, colptr, rows.astype(np.int32), vals)


def sign_sketch(k: int, n: int, per_row: int, seed: int) -> CSC:
    rng = np.random.default_rng(seed)
    cols = _distinct_per_line(rng, k, per_row, n).ravel()
    rows = np.repeat(np.arange(k, dtype=np.int64), per_row)
    signs = np.where(rng.random(k * per_row) < 0.5, -0.5, 0.5)
    return from_triplets(k, n, rows, cols, signs)


def uniform_values(count: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=count)


def er_batch(count: int, seed: int):
    """List of (A_t, B_t) pairs of independent square ER matrices."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n_t = int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e4)))))
        d_t = int(round(math.exp(rng.uniform(math.log(4.0), math.log(32.0)))))
        s = int(rng.integers(0, 2 ** 31 - 1))
        out.append((erdos_renyi(n_t, n_t, d_t, s), erdos_renyi(n_t, n_t, d_t, s + 1)))
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def unit_values(M: CSC) -> CSC:
    """The pattern of M with every stored value 1 (an unweighted graph)."""
    return CSC(M.nrows, M.ncols, M.colptr, M.rowidx, np.ones(M.nnz))


def bfs_sources(n: int, count: int, seed: int) -> CSC:
    """Frontier of a multi-source search at its start: column s holds a 1 at
    the s-th of `count` distinct vertices drawn uniformly from [0, n)."""
    rng = np.random.default_rng(seed)
    src = np.sort(rng.choice(n, size=count, replace=False)) if count else np.zeros(0, np.int64)
    return from_triplets(n, count, src, np.arange(count), np.ones(count))


def next_frontier(N: CSC, visited: np.ndarray):
    """One level of a multi-source breadth-first search: N = A * F holds, in
    column s, the vertices one hop from source s's frontier with their
    shortest-path counts; the next frontier keeps the entries of vertices
    that search s has not reached yet.  visited (n x count, bool) is updated
    in place.  Pure selection, no arithmetic."""
    cols = np.repeat(np.arange(N.ncols), np.diff(N.colptr))
    keep = ~visited[N.rowidx, cols]
    visited[N.rowidx[keep], cols[keep]] = True
    colptr = np.zeros(N.ncols + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols[keep], minlength=N.ncols), out=colptr[1:])
    return CSC(N.nrows, N.ncols, colptr, N.rowidx[keep].copy(), np.asarray(N.vals)[keep].copy())


def workload(name: str):
    """Named inputs used by tests and the benchmark.

    Returns a dict with the operands and the partition description.
    """
    if name == "lap2d_64_p4":
        A = laplacian2d(64)
        return {"A": A, "B": A, "P": 4, "offsets": partition_offsets(A.ncols, 4), "b": 64}
    if name == "er65536_d16_p16":
        A = erdos_renyi(65536, 65536, 16, seed=1)
        B = erdos_renyi(65536, 65536, 16, seed=2)
        return {"A": A, "B": B, "P": 16, "offsets": partition_offsets(A.ncols, 16), "b": 256}
    if name == "rmat18":
        A = rmat(18, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
        return {"A": A, "B": A, "P": 1, "offsets": partition_offsets(A.ncols, 1), "b": 256}
    if name == "sketch_er131072":
        A = erdos_renyi(131072, 131072, 8, seed=5)
        B = sign_sketch(131072, 4096, 4, seed=6)
        return {"A": A, "B": B, "P": 1, "offsets": partition_offsets(A.ncols, 1), "b": 256}
    if name == "bfs_rmat16_4096":
        # multi-source search of a batched betweenness-centrality forward
        # pass: 4096 sources on an unweighted R-MAT graph
        A = unit_values(rmat(16, 16, 0.57, 0.19, 0.19, 0.05, seed=3))
        F = bfs_sources(A.ncols, 4096, seed=7)
        return {"A": A, "B": F, "P": 1, "offsets": partition_offsets(A.ncols, 1), "b": 256}
    if name == "sketch_er512":
        A = erdos_renyi(512, 512, 8, seed=5)
        B = sign_sketch(512, 16, 4, seed=6)
        return {"A": A, "B": B, "P": 1, "offsets": partition_offsets(A.ncols, 1), "b": 64}
    raise KeyError(name)
