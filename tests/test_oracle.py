"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check comes from the
paper's worked example, a closed form, an invariant, a special case that
reduces to a plain numpy routine, or brute force on tiny inputs.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_csc(rng, m, n, density, lo=-1.0, hi=1.0, empty_cols=()):
    mask = rng.random((m, n)) < density
    for c in empty_cols:
        mask[:, c] = False
    rows, cols = np.nonzero(mask)
    return synth.from_triplets(m, n, rows, cols, rng.uniform(lo, hi, rows.size))


def product_dense(prod):
    out = np.zeros((prod.nrows, prod.ncols))
    for j in range(prod.ncols):
        lo, hi = prod.colptr[j], prod.colptr[j + 1]
        out[prod.rowidx[lo:hi], j] = prod.vals[lo:hi]
    return out


def product_pattern(prod):
    out = np.zeros((prod.nrows, prod.ncols), dtype=bool)
    for j in range(prod.ncols):
        out[prod.rowidx[prod.colptr[j]:prod.colptr[j + 1]], j] = True
    return out


# ---------------------------------------------------------------------------
# H_i and Alg. 2
# ---------------------------------------------------------------------------

def test_paper_worked_example_block_fetch():
    """Sec. III-A example: H_0 = [1,0,1,1,0,1,0,0], 4 blocks of 2 columns;
    p_0 fetches block (1,0) (columns 4-5) although column 4 is unused."""
    g = json.load(open(os.path.join(GOLDEN, "paper_example_block_fetch.json")))
    k, P, b = g["k"], g["P"], g["columns_per_block"]
    rng = np.random.default_rng(0)
    # every column of A holds entries (the example's blocks are all non-empty)
    A = rand_csc(rng, k, k, 0.4)
    dense = A.to_dense()
    for c in range(k):
        if not dense[:, c].any():
            dense[c, c] = 1.0
    r, c = np.nonzero(dense)
    A = synth.from_triplets(k, k, r, c, dense[r, c])
    # B_0: k x 4 slice whose nonzero rows are exactly {0, 2, 3, 5}
    rows = [0, 2, 3, 5, 0, 3]
    cols = [0, 1, 2, 3, 3, 0]
    B0 = synth.from_triplets(k, 4, rows, cols, np.ones(len(rows)))
    H = oracle.rows_of_b(k, B0)
    assert H.tolist() == g["H0"]
    assert H[4:8].tolist() == [0, 1, 0, 0]
    s = oracle.block_select(A, H, synth.partition_offsets(k, P), b)
    assert s.blocks.tolist() == g["chosen_blocks_first_last"]
    assert s.K == 4 and s.blocks.shape[0] == 3
    assert np.nonzero(s.sel)[0].tolist() == g["selected_columns"]
    for c in g["remote_columns_fetched_but_unused"]:
        assert s.sel[c] == 1 and H[c] == 0
    for c in g["remote_columns_needed"]:
        assert s.sel[c] == 1 and H[c] == 1
    # the skipped remote block (1,1) is columns 6-7
    assert s.sel[6] == 0 and s.sel[7] == 0


def test_rows_of_b_marks_exactly_the_stored_rows():
    rng = np.random.default_rng(1)
    for _ in range(20):
        k = int(rng.integers(1, 40))
        B = rand_csc(rng, k, int(rng.integers(1, 10)), 0.2)
        H = oracle.rows_of_b(k, B)
        want = np.zeros(k, np.uint8)
        want[np.unique(B.rowidx)] = 1
        assert np.array_equal(H, want)
    assert oracle.rows_of_b(5, synth.from_triplets(5, 3, [], [], [])).sum() == 0


def _nonzero_cols(A):
    return np.diff(A.colptr) > 0


@pytest.mark.parametrize("seed", range(30))
def test_block_select_postconditions(seed):
    """Alg. 2 result contract: M <= K, the chosen intervals cover the required
    ids H ∩ D, each chosen interval holds a required id, intervals hold at most
    b nonzero columns and stay inside one partition; K = sum ceil(nzc_r/b)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 80))
    A = rand_csc(rng, int(rng.integers(1, 30)), k, float(rng.uniform(0.02, 0.3)))
    H = (rng.random(k) < rng.uniform(0, 0.5)).astype(np.uint8)
    P = int(rng.integers(1, min(k, 6) + 1))
    offs = np.sort(np.concatenate([[0, k], rng.choice(np.arange(1, k), P - 1, replace=False)
                                   if k > 1 and P > 1 else []])).astype(np.int64)
    P = offs.size - 1
    b = int(rng.integers(1, 9))
    s = oracle.block_select(A, H, offs, b)
    nz = _nonzero_cols(A)
    need = set(np.nonzero(nz & (H == 1))[0].tolist())
    part = np.searchsorted(offs, np.arange(k), side="right") - 1
    nzc = [int(nz[offs[r]:offs[r + 1]].sum()) for r in range(P)]
    assert s.K == sum(-(-c // b) for c in nzc)
    assert s.blocks.shape[0] <= s.K
    covered = set()
    for first, last in s.blocks:
        assert part[first] == part[last] and first <= last
        inside = [c for c in range(first, last + 1) if nz[c]]
        assert nz[first] and nz[last]
        assert 1 <= len(inside) <= b
        assert any(c in need for c in inside)
        covered.update(inside)
    assert need <= covered
    assert covered == set(np.nonzero(s.sel)[0].tolist())
    # empty columns are never selected
    assert not (s.sel.astype(bool) & ~nz).any()
    # map is the exclusive prefix of sel
    exp_map = np.where(s.sel == 1, np.cumsum(s.sel.astype(np.int64)) - 1, -1)
    assert np.array_equal(s.map, exp_map)
    assert s.kt == int(s.sel.sum())


def test_block_select_groups_are_consecutive_runs_of_b():
    """Brute force over the grouping: within a partition, the r-th nonzero
    column belongs to group floor(r/b); enumerate H over every subset of a
    small partition and compare with that grouping."""
    rng = np.random.default_rng(7)
    k = 10
    A = rand_csc(rng, 6, k, 0.5, empty_cols=(2, 7))
    nz = np.nonzero(_nonzero_cols(A))[0]
    for b in (1, 2, 3, 8, 20):
        for mask in range(1 << k):
            H = np.array([(mask >> c) & 1 for c in range(k)], dtype=np.uint8)
            s = oracle.block_select(A, H, [0, k], b)
            groups = [nz[g:g + b] for g in range(0, nz.size, b)]
            want = np.zeros(k, np.uint8)
            chosen = []
            for grp in groups:
                if H[grp].any():
                    want[grp] = 1
                    chosen.append([grp[0], grp[-1]])
            assert np.array_equal(s.sel, want)
            assert s.blocks.tolist() == chosen


def test_block_select_extremes():
    """b = 1 selects exactly H ∩ D; b >= nzc selects a whole partition as soon
    as one of its columns is required."""
    rng = np.random.default_rng(3)
    A = rand_csc(rng, 20, 64, 0.1)
    nz = _nonzero_cols(A)
    H = (rng.random(64) < 0.2).astype(np.uint8)
    offs = synth.partition_offsets(64, 4)
    s1 = oracle.block_select(A, H, offs, 1)
    assert np.array_equal(s1.sel.astype(bool), nz & (H == 1))
    sbig = oracle.block_select(A, H, offs, 10 ** 6)
    for r in range(4):
        lo, hi = offs[r], offs[r + 1]
        any_hit = (nz[lo:hi] & (H[lo:hi] == 1)).any()
        assert np.array_equal(sbig.sel[lo:hi].astype(bool), nz[lo:hi] & any_hit)


@pytest.mark.parametrize("seed", range(10))
def test_block_select_own_partition_whole(seed):
    """Naming the caller's own partition selects all of its nonzero columns
    (every one of its groups is chosen, in order), whatever H says, and
    leaves the other partitions' choice as without it."""
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(8, 70))
    A = rand_csc(rng, 15, k, 0.2, empty_cols=(0,))
    H = (rng.random(k) < 0.15).astype(np.uint8)
    offs = synth.partition_offsets(k, 3)
    b = int(rng.integers(1, 6))
    own = int(rng.integers(0, 3))
    base = oracle.block_select(A, H, offs, b)
    s = oracle.block_select(A, H, offs, b, own_whole=own)
    nz = _nonzero_cols(A)
    lo, hi = offs[own], offs[own + 1]
    want = base.sel.copy()
    want[lo:hi] = nz[lo:hi]
    assert np.array_equal(s.sel, want)
    ids = np.nonzero(nz[lo:hi])[0] + lo
    own_blocks = [[ids[g], ids[min(g + b, ids.size) - 1]] for g in range(0, ids.size, b)]
    other = [blk for blk in base.blocks.tolist() if not lo <= blk[0] < hi]
    assert sorted(s.blocks.tolist()) == sorted(other + own_blocks)
    assert s.K == base.K and s.blocks.shape[0] == len(other) + len(own_blocks)


def test_gather_copies_selected_columns_bitwise():
    rng = np.random.default_rng(4)
    A = rand_csc(rng, 30, 50, 0.15)
    H = (rng.random(50) < 0.3).astype(np.uint8)
    s = oracle.block_select(A, H, synth.partition_offsets(50, 3), 4)
    At = oracle.gather(A, s.map, s.kt)
    assert At.ncols == s.kt
    for c in range(50):
        if s.map[c] < 0:
            continue
        j = s.map[c]
        a0, a1 = A.colptr[c], A.colptr[c + 1]
        t0, t1 = At.colptr[j], At.colptr[j + 1]
        assert np.array_equal(A.rowidx[a0:a1], At.rowidx[t0:t1])
        assert np.array_equal(A.vals[a0:a1].view(np.uint64), At.vals[t0:t1].view(np.uint64))
    assert At.colptr[-1] == int(np.diff(A.colptr)[s.sel == 1].sum())


def test_laplacian2d_gather_closed_form():
    """64x64 5-point Laplacian, P = 4 (16 grid rows per partition), b = 64:
    every group is one grid row, H_i covers grid rows [16i-1, 16i+16], so
    kt = 64*|rows| and nnz(A~) = 254 per boundary grid row + 318 per other."""
    w = synth.workload("lap2d_64_p4")
    A = w["A"]
    for i in range(4):
        Bi = synth.column_slice(A, int(w["offsets"][i]), int(w["offsets"][i + 1]))
        H = oracle.rows_of_b(A.ncols, Bi)
        s = oracle.block_select(A, H, w["offsets"], 64)
        grid_rows = [y for y in range(16 * i - 1, 16 * i + 17) if 0 <= y < 64]
        assert s.kt == 64 * len(grid_rows)
        assert s.blocks.shape[0] == len(grid_rows) and s.K == 64
        At = oracle.gather(A, s.map, s.kt)
        want = sum(254 if y in (0, 63) else 318 for y in grid_rows)
        assert At.colptr[-1] == want
    assert [5342, 5724] == [sum(254 if y in (0, 63) else 318 for y in range(0, 17)),
                            18 * 318]


# ---------------------------------------------------------------------------
# sparse flops
# ---------------------------------------------------------------------------

def test_flops_inner_product_identity():
    """Total sparse flops = <nnz per column of A, nnz per row of B> (Sec. III-B)."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        m, k, n = (int(x) for x in rng.integers(1, 40, 3))
        A = rand_csc(rng, m, k, 0.2)
        B = rand_csc(rng, k, n, 0.2)
        f = oracle.column_flops(A, B)
        colnnz = np.diff(A.colptr)
        rownnz = np.bincount(B.rowidx, minlength=k)
        assert f.sum() == int(colnnz @ rownnz)
        # nnz of a column never exceeds its flops
        C = oracle.spgemm(A, B)
        assert (np.diff(C.colptr) <= f).all()


def test_flops_er_closed_form():
    A = synth.erdos_renyi(2000, 2000, 16, seed=1)
    B = synth.erdos_renyi(2000, 500, 16, seed=2)
    assert (oracle.column_flops(A, B) == 256).all()


# ---------------------------------------------------------------------------
# the product
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_spgemm_matches_dense_matmul(seed):
    rng = np.random.default_rng(100 + seed)
    m, k, n = (int(x) for x in rng.integers(1, 48, 3))
    A = rand_csc(rng, m, k, float(rng.uniform(0.0, 0.4)), empty_cols=(0,) if k > 2 else ())
    B = rand_csc(rng, k, n, float(rng.uniform(0.0, 0.4)))
    C = oracle.spgemm(A, B)
    Ad, Bd = A.to_dense(), B.to_dense()
    np.testing.assert_allclose(product_dense(C), Ad @ Bd, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(product_dense(C._replace(vals=C.absvals)),
                               np.abs(Ad) @ np.abs(Bd), rtol=1e-13, atol=1e-13)
    # pattern = structural boolean product (explicit zeros stay stored)
    assert np.array_equal(product_pattern(C), ((Ad != 0).astype(np.int64)
                                                @ (Bd != 0).astype(np.int64)) > 0)
    # rows ascending inside each column
    for j in range(n):
        r = C.rowidx[C.colptr[j]:C.colptr[j + 1]]
        assert (np.diff(r) > 0).all()


def test_spgemm_row_sum_invariant():
    """C*1 = A*(B*1), two matrix-vector products that never form C."""
    A = synth.erdos_renyi(3000, 2500, 7, seed=11)
    B = synth.erdos_renyi(2500, 1800, 5, seed=12)
    C = oracle.spgemm(A, B)
    ones = np.ones(B.ncols)
    Bx = np.zeros(B.nrows)
    np.add.at(Bx, B.rowidx, B.vals * ones[np.repeat(np.arange(B.ncols), np.diff(B.colptr))])
    ABx = np.zeros(A.nrows)
    np.add.at(ABx, A.rowidx, A.vals * Bx[np.repeat(np.arange(A.ncols), np.diff(A.colptr))])
    Cx = np.zeros(C.nrows)
    np.add.at(Cx, C.rowidx, C.vals)
    np.testing.assert_allclose(Cx, ABx, rtol=1e-11, atol=1e-11)


def test_spgemm_all_3x3_patterns():
    """Every pair of 3x3 patterns (512 x 512), packed as diagonal blocks of one
    product, against batched dense 3x3 products."""
    pats = np.array([[(p >> b) & 1 for b in range(9)] for p in range(512)], dtype=np.int64)
    pats = pats.reshape(512, 3, 3)
    ia, ib = np.meshgrid(np.arange(512), np.arange(512), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()
    N = ia.size
    rng = np.random.default_rng(9)
    Av = pats[ia] * rng.integers(1, 5, size=(N, 3, 3))
    Bv = pats[ib] * rng.integers(-4, 5, size=(N, 3, 3))  # zeros allowed in values? no:
    Bv = np.where(pats[ib] == 1, np.where(Bv == 0, 1, Bv), 0)

    def blockdiag(vals, pat):
        t, r, c = np.nonzero(pat)
        return synth.from_triplets(3 * N, 3 * N, 3 * t + r, 3 * t + c,
                                   vals[t, r, c].astype(np.float64))

    A = blockdiag(Av, pats[ia])
    B = blockdiag(Bv, pats[ib])
    C = oracle.spgemm(A, B)
    want_val = np.einsum("tij,tjk->tik", Av, Bv)
    want_pat = np.einsum("tij,tjk->tik", pats[ia], pats[ib]) > 0
    got_val = np.zeros((N, 3, 3))
    got_pat = np.zeros((N, 3, 3), dtype=bool)
    col = np.repeat(np.arange(C.ncols), np.diff(C.colptr))
    t = col // 3
    got_val[t, C.rowidx - 3 * t, col - 3 * t] = C.vals
    got_pat[t, C.rowidx - 3 * t, col - 3 * t] = True
    assert np.array_equal(got_pat, want_pat)
    assert np.array_equal(got_val, want_val)  # small integers: exact


def test_laplacian2d_square_closed_form():
    """A = 4I - Adj on a 64x64 grid: A^2 = 16I - 8 Adj + Adj^2.  Diagonal
    16 + degree (20/19/18), -8 at grid distance 1, 1 at straight distance 2,
    2 at diagonal distance 2; nnz per column in {6,8,9,11,12,13} with counts
    {4,8,240,4,240,3600}.  All values are small integers, so exact."""
    n = 64
    A = synth.laplacian2d(n)
    C = oracle.spgemm(A, A)
    counts = np.diff(C.colptr)
    vals, cnt = np.unique(counts, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == {6: 4, 8: 8, 9: 240, 11: 4, 12: 240, 13: 3600}
    assert C.colptr[-1] == 51972
    col = np.repeat(np.arange(n * n), counts)
    x0, y0 = col % n, col // n
    x1, y1 = C.rowidx % n, C.rowidx // n
    dx, dy = np.abs(x1 - x0), np.abs(y1 - y0)
    deg = (x0 > 0).astype(int) + (x0 < n - 1) + (y0 > 0) + (y0 < n - 1)
    want = np.select([(dx == 0) & (dy == 0), dx + dy == 1, (dx == 2) | (dy == 2),
                      (dx == 1) & (dy == 1)], [16.0 + deg, -8.0, 1.0, 2.0], np.nan)
    assert not np.isnan(want).any()
    assert np.array_equal(C.vals, want)


def test_galerkin_closed_form():
    """3D 7-point Laplacian with 2x2x2 aggregation: A P holds 3 inside the
    aggregate and -1 on its face neighbours; P^T (A P) = 4 * L_{n/2}, so the
    l-th level is 4^l L_{n/2^l}; nnz(L_n) = 7n^3 - 6n^2 (exact integers)."""
    n = 16
    A = synth.laplacian3d(n)
    for level in range(3):
        P = synth.aggregation3d(n)
        Pt = synth.aggregation3d_t(n)
        assert (np.diff(Pt.colptr) == 1).all()          # one entry per row of P
        AP = oracle.spgemm(A, P)
        assert set(np.unique(AP.vals).tolist()) == {3.0 * 4 ** level, -1.0 * 4 ** level}
        if level == 0:
            h = n // 2
            faces = 6 * h ** 3 - 6 * h ** 2
            assert AP.colptr[-1] == 8 * h ** 3 + 4 * faces
        Ac = oracle.spgemm(Pt, AP)
        n //= 2
        ref = synth.laplacian3d(n)
        assert Ac.colptr[-1] == 7 * n ** 3 - 6 * n ** 2
        assert np.array_equal(Ac.colptr, ref.colptr)
        assert np.array_equal(Ac.rowidx, ref.rowidx)
        assert np.array_equal(Ac.vals, 4.0 ** (level + 1) * ref.vals)
        A = synth.CSC(Ac.nrows, Ac.ncols, Ac.colptr, Ac.rowidx, Ac.vals)


def test_galerkin_coarse_nnz_at_64():
    """nnz(A_c) for the 64^3 hierarchy: 223,232 / 27,136 / 3,200 / 352."""
    assert [7 * n ** 3 - 6 * n ** 2 for n in (32, 16, 8, 4)] == [223232, 27136, 3200, 352]


def test_spgemm_column_subset_and_empty():
    rng = np.random.default_rng(21)
    A = rand_csc(rng, 25, 20, 0.2)
    B = rand_csc(rng, 20, 15, 0.2, empty_cols=(3,))
    full = oracle.spgemm(A, B)
    cols = [14, 3, 0, 7]
    sub = oracle.spgemm(A, B, cols)
    for t, j in enumerate(cols):
        assert np.array_equal(sub.rowidx[sub.colptr[t]:sub.colptr[t + 1]],
                              full.rowidx[full.colptr[j]:full.colptr[j + 1]])
    assert sub.colptr[2] - sub.colptr[1] == 0
    E = synth.from_triplets(20, 5, [], [], [])
    e = oracle.spgemm(A, E)
    assert e.colptr.tolist() == [0] * 6


def test_local_product_partition_stitch():
    """C is already in 1D layout: the P local products stacked side by side
    equal the whole product, and shrinking A to A~ loses nothing."""
    rng = np.random.default_rng(31)
    A = rand_csc(rng, 40, 36, 0.1)
    B = rand_csc(rng, 36, 24, 0.1)
    whole = product_dense(oracle.spgemm(A, B))
    offsB = synth.partition_offsets(24, 3)
    offsA = synth.partition_offsets(36, 3)
    parts = []
    for i in range(3):
        Bi = synth.column_slice(B, int(offsB[i]), int(offsB[i + 1]))
        loc = oracle.local_product(A, Bi, offsA, 2)
        parts.append(product_dense(loc.C))
        # the same product computed from A~ with B's rows renumbered by map
        keep = loc.selection.map[Bi.rowidx] >= 0
        cols = np.repeat(np.arange(Bi.ncols), np.diff(Bi.colptr))[keep]
        Bt = synth.from_triplets(loc.At.ncols, Bi.ncols, loc.selection.map[Bi.rowidx][keep],
                                 cols, Bi.vals[keep])
        np.testing.assert_array_equal(product_dense(oracle.spgemm(loc.At, Bt)), parts[-1])
    np.testing.assert_allclose(np.hstack(parts), whole, rtol=0, atol=0)


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------

def _loss(A, B, C, dC):
    prod = oracle.spgemm(A, B)
    assert np.array_equal(prod.colptr, C.colptr) and np.array_equal(prod.rowidx, C.rowidx)
    return float(np.dot(prod.vals, dC))


def test_backward_dense_masked_formula():
    rng = np.random.default_rng(41)
    A = rand_csc(rng, 12, 10, 0.3)
    B = rand_csc(rng, 10, 8, 0.3)
    C = oracle.spgemm(A, B)
    dC = rng.uniform(-1, 1, C.colptr[-1])
    dA, dB = oracle.backward(A, B, C.colptr, C.rowidx, dC)
    dCd = product_dense(C._replace(vals=dC))
    gA = dCd @ B.to_dense().T
    gB = A.to_dense().T @ dCd
    colA = np.repeat(np.arange(A.ncols), np.diff(A.colptr))
    colB = np.repeat(np.arange(B.ncols), np.diff(B.colptr))
    np.testing.assert_allclose(dA, gA[A.rowidx, colA], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(dB, gB[B.rowidx, colB], rtol=1e-13, atol=1e-13)


def test_backward_finite_differences_exact():
    """L = <dC, A B> is linear in each entry, so a central difference with any
    step equals the gradient up to rounding."""
    rng = np.random.default_rng(42)
    A = rand_csc(rng, 15, 13, 0.25)
    B = rand_csc(rng, 13, 9, 0.25)
    C = oracle.spgemm(A, B)
    dC = rng.uniform(-1, 1, C.colptr[-1])
    dA, dB = oracle.backward(A, B, C.colptr, C.rowidx, dC)
    h = 0.5
    for p in rng.choice(A.vals.size, 10, replace=False):
        Ap = synth.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, A.vals.copy())
        Am = synth.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, A.vals.copy())
        Ap.vals[p] += h
        Am.vals[p] -= h
        fd = (_loss(Ap, B, C, dC) - _loss(Am, B, C, dC)) / (2 * h)
        assert abs(fd - dA[p]) <= 1e-12 * max(1.0, abs(fd))
    for q in rng.choice(B.vals.size, 10, replace=False):
        Bp = synth.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, B.vals.copy())
        Bm = synth.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, B.vals.copy())
        Bp.vals[q] += h
        Bm.vals[q] -= h
        fd = (_loss(A, Bp, C, dC) - _loss(A, Bm, C, dC)) / (2 * h)
        assert abs(fd - dB[q]) <= 1e-12 * max(1.0, abs(fd))


def test_backward_adjoint_identities():
    """sum dA*A = <dC, C> = sum dB*B (bilinearity)."""
    w = synth.workload("sketch_er512")
    A, B = w["A"], w["B"]
    C = oracle.spgemm(A, B)
    dC = synth.uniform_values(int(C.colptr[-1]), seed=7)
    dA, dB = oracle.backward(A, B, C.colptr, C.rowidx, dC)
    ref = float(np.dot(dC, C.vals))
    assert abs(float(np.dot(dA, A.vals)) - ref) <= 1e-11 * abs(ref)
    assert abs(float(np.dot(dB, B.vals)) - ref) <= 1e-11 * abs(ref)
