"""The seeded input generators produce the structures the workloads state
(checked on the CPU): exact per-column counts, value ranges, canonical CSC,
and determinism under a seed."""

import numpy as np

import synth


def _canonical(M):
    assert M.colptr[0] == 0 and M.colptr[-1] == M.rowidx.size == M.vals.size
    assert np.all(np.diff(M.colptr) >= 0)
    for j in range(M.ncols):
        r = M.rowidx[M.colptr[j]:M.colptr[j + 1]]
        assert np.all(np.diff(r) > 0), f"column {j} not strictly ascending"
    assert M.rowidx.min(initial=0) >= 0 and M.rowidx.max(initial=-1) < M.nrows


def test_erdos_renyi_has_exactly_d_distinct_rows_per_column():
    A = synth.erdos_renyi(300, 200, 7, seed=11)
    _canonical(A)
    assert np.all(np.diff(A.colptr) == 7)
    assert A.vals.min() >= -1 and A.vals.max() < 1
    B = synth.erdos_renyi(300, 200, 7, seed=11)
    assert np.array_equal(A.rowidx, B.rowidx) and np.array_equal(A.vals, B.vals)
    C = synth.erdos_renyi(300, 200, 7, seed=12)
    assert not np.array_equal(A.rowidx, C.rowidx)


def test_sign_sketch_rows():
    S = synth.sign_sketch(200, 64, 4, seed=3)
    _canonical(S)
    per_row = np.bincount(S.rowidx, minlength=S.nrows)
    assert np.all(per_row == 4)
    assert set(np.unique(S.vals).tolist()) <= {-0.5, 0.5}


def test_laplacians_and_aggregation():
    L2 = synth.laplacian2d(8)
    _canonical(L2)
    D = L2.to_dense()
    assert np.allclose(D, D.T) and np.all(np.diag(D) == 4)
    assert L2.nnz == 5 * 64 - 4 * 8
    L3 = synth.laplacian3d(6)
    _canonical(L3)
    D3 = L3.to_dense()
    assert np.all(np.diag(D3) == 6) and L3.nnz == 7 * 216 - 6 * 36
    P = synth.aggregation3d(6)
    Pt = synth.aggregation3d_t(6)
    _canonical(P)
    _canonical(Pt)
    dP = P.to_dense()
    assert np.all(dP.sum(axis=1) == 1) and np.all(dP.sum(axis=0) == 8)
    assert np.array_equal(Pt.to_dense(), dP.T)


def test_transpose_round_trip():
    A = synth.erdos_renyi(90, 70, 5, seed=2)
    T = synth.transpose(A)
    _canonical(T)
    assert np.array_equal(T.to_dense(), A.to_dense().T)
    TT = synth.transpose(T)
    assert np.array_equal(TT.colptr, A.colptr) and np.array_equal(TT.rowidx, A.rowidx)
    assert np.array_equal(TT.vals, A.vals)


def test_rmat_small_scale():
    R = synth.rmat(10, 8, 0.57, 0.19, 0.19, 0.05, seed=3)
    _canonical(R)
    assert R.nrows == R.ncols == 1024
    assert 0 < R.nnz <= 8 * 1024
    assert R.vals.min() >= 0 and R.vals.max() < 1
    # the (0,0) quadrant holds the largest share of the entries
    cols = np.repeat(np.arange(R.ncols), np.diff(R.colptr))
    q00 = np.sum((R.rowidx < 512) & (cols < 512))
    assert q00 > 0.4 * R.nnz


def test_partition_offsets_and_column_slice():
    o = synth.partition_offsets(10, 4)
    assert o.tolist() == [0, 2, 5, 7, 10]
    A = synth.erdos_renyi(20, 10, 3, seed=1)
    parts = [synth.column_slice(A, int(o[r]), int(o[r + 1])) for r in range(4)]
    stitched = np.hstack([p.to_dense() for p in parts])
    assert np.array_equal(stitched, A.to_dense())


def test_er_batch_shapes_stay_in_range():
    batch = synth.er_batch(16, seed=4)
    assert len(batch) == 16
    for A, B in batch:
        assert A.nrows == A.ncols == B.nrows == B.ncols
        assert 1000 <= A.nrows <= 50000
        d = int(A.colptr[1] - A.colptr[0])
        assert 4 <= d <= 32 and np.all(np.diff(B.colptr) == d)


def test_permute_symmetric_is_a_relabelling():
    A = synth.erdos_renyi(60, 60, 4, seed=5)
    Q = synth.permute_symmetric(A, seed=9)
    _canonical(Q)
    q = np.random.default_rng(9).permutation(60)
    D, E = A.to_dense(), Q.to_dense()
    assert np.array_equal(E[np.ix_(q, q)], D)
    assert Q.nnz == A.nnz
