"""GPU parity of the forward path (plan, symbolic, numeric) against the CPU
oracle, through the C ABI.

Bit-exact: H_i, the column map, Alg. 2's chosen blocks, A~ (row ids and
values), the sparse flops per column, C_i's column pointers and row ids.
Values: FP64 per entry within 1e-12 of max(|c|, sum |a||b|); FP32
normwise within 1e-5 of the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values, columns_of

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _dev(M, dtype):
    return spg.DeviceCsc.from_host(M, dtype=dtype)


def check_local(A, Bi, offs, b, dtype=torch.float64, tun=None, cols=None, own_whole=-1):
    """Runs the GPU path for one partition and compares every stage."""
    Ad, Bd = _dev(A, dtype), _dev(Bi, dtype)
    if dtype == torch.float32:
        A = synth.as_fp32(A)
        Bi = synth.as_fp32(Bi)
    ref = oracle.local_product(A, Bi, offs, b, own_whole=own_whole)
    with spg.Plan(Ad, Bd, offs, b, tuning=tun) as p:
        ex = p.export()
        st = ex["stats"]
        assert np.array_equal(ex["H"].cpu().numpy(), ref.H)
        assert np.array_equal(ex["map"].cpu().numpy(), ref.selection.map)
        assert st["kt"] == ref.selection.kt
        assert st["K"] == ref.selection.K
        assert st["M"] == ref.selection.blocks.shape[0]
        assert np.array_equal(ex["blocks"].cpu().numpy().reshape(-1, 2), ref.selection.blocks)
        assert st["h_count"] == int(ref.H.sum())
        assert np.array_equal(ex["At_colptr"].cpu().numpy(), ref.At.colptr)
        assert np.array_equal(ex["At_rowidx"].cpu().numpy(), ref.At.rowidx)
        atv = ex["At_vals"].cpu().numpy()
        assert np.array_equal(atv, np.asarray(ref.At.vals, dtype=atv.dtype))
        colptr = p.symbolic()
        flop, sbin, nbin = p.export_bins()
        assert np.array_equal(flop.cpu().numpy(), ref.flop)
        assert np.array_equal(colptr.cpu().numpy(), ref.C.colptr)
        st2 = p.stats()
        assert st2["flops"] == int(ref.flop.sum())
        assert st2["nnz_C"] == int(ref.C.colptr[-1])
        rows, vals = p.numeric()
        assert np.array_equal(rows.cpu().numpy(), ref.C.rowidx)
        assert_values(vals.cpu().numpy(), ref.C.vals, ref.C.absvals, dtype == torch.float64)
        return st2, sbin.cpu().numpy(), nbin.cpu().numpy()


def rand_csc(rng, m, n, density, lo=-1.0, hi=1.0, empty_cols=()):
    mask = rng.random((m, n)) < density
    for c in empty_cols:
        mask[:, c] = False
    r, c = np.nonzero(mask)
    return synth.from_triplets(m, n, r, c, rng.uniform(lo, hi, r.size))


def test_device_properties():
    props = torch.cuda.get_device_properties(0)
    print("device:", props.name, getattr(props, "gcnArchName", "?"),
          "CUs:", props.multi_processor_count, flush=True)
    assert "gfx950" in getattr(props, "gcnArchName", "gfx950")


@pytest.mark.parametrize("b", [64, 1, 256])
@pytest.mark.parametrize("i", [0, 1, 2, 3])
def test_laplacian2d_partitions(i, b):
    w = synth.workload("lap2d_64_p4")
    A = w["A"]
    Bi = synth.column_slice(A, int(w["offsets"][i]), int(w["offsets"][i + 1]))
    check_local(A, Bi, w["offsets"], b)


@pytest.mark.parametrize("seed", range(8))
def test_random_small_shapes(seed):
    rng = np.random.default_rng(1000 + seed)
    m, k, n = (int(x) for x in rng.integers(1, 300, 3))
    A = rand_csc(rng, m, k, float(rng.uniform(0.0, 0.1)), empty_cols=(0,) if k > 1 else ())
    Bi = rand_csc(rng, k, n, float(rng.uniform(0.0, 0.1)))
    P = int(rng.integers(1, min(k, 8) + 1))
    offs = synth.partition_offsets(k, P)
    b = int(rng.choice([1, 2, 3, 16, 1000]))
    check_local(A, Bi, offs, b)


@pytest.mark.parametrize("n", [8191, 8192, 8193, 20011])
def test_colptr_scan_one_workgroup_and_tiled(n):
    # up to 8192 columns of B_i one workgroup scans and bins them all; above,
    # tiles of 1024 columns with a look-back (20011: 20 tiles and a ragged one)
    rng = np.random.default_rng(n)
    A = rand_csc(rng, 3000, 500, 0.01)
    Bi = rand_csc(rng, 500, n, 0.01, empty_cols=(0, n - 1))
    st, _, nbin = check_local(A, Bi, synth.partition_offsets(500, 4), 16)
    assert int((nbin == 0).sum()) >= 2  # empty columns stay out of every list
    for b in range(1, 8):
        assert st["num_bins"][b] == int((nbin == b).sum())


def _with_long_columns(rng, k, n, base, longs):
    """B_i (k x n): `base` random entries per column, and columns j of
    `longs` = {j: length} with that many distinct random rows."""
    rows, cols = [], []
    for j in range(n):
        cnt = longs.get(j, base)
        r = rng.choice(k, size=min(cnt, k), replace=False)
        rows.append(r)
        cols.append(np.full(r.size, j))
    r, c = np.concatenate(rows), np.concatenate(cols)
    return synth.from_triplets(k, n, r, c, rng.uniform(-1.0, 1.0, r.size))


@pytest.mark.parametrize("case", ["wide_lanes", "one_lane", "chunk_edges"])
def test_long_columns_split_over_chunks(case):
    # columns longer than 16 entries per lane are walked in chunks of 8192
    # entries of B_i by several workgroups; the chunk that completes a
    # column bins it (30000 entries: five chunks; 8192: a chunk boundary
    # inside; 17 entries with one lane per column: just over the limit)
    rng = np.random.default_rng(31 if case == "wide_lanes" else 32)
    k = 40000
    A = rand_csc(rng, 300, k, 2.0 / 300)
    if case == "wide_lanes":
        Bi = _with_long_columns(rng, k, 50, 3, {7: 30000, 8: 8192, 49: 300})
    elif case == "one_lane":
        Bi = _with_long_columns(rng, k, 20000, 1, {0: 17, 5: 5000, 19999: 4000})
    else:
        # entries [0, 8192): exactly chunk 0; [8192, 16383): inside chunk 1;
        # a short column across the next edge; then a long column from
        # chunk 2 into chunk 3 by one entry, an empty and a short column
        Bi = _with_long_columns(rng, k, 6, 0, {0: 8192, 1: 8191, 2: 2, 3: 8192, 4: 0, 5: 7})
        assert list(np.diff(Bi.colptr)) == [8192, 8191, 2, 8192, 0, 7]
    check_local(A, Bi, synth.partition_offsets(k, 8), 64)


@pytest.mark.parametrize("n", [16384, 16385])
def test_tiny_symbolic_before_and_after_the_counts(n):
    # up to 16384 columns the tiny symbolic kernel is launched before the
    # host has the bin counts (count read on the device, bin list used since
    # not every column is tiny); above, after them.  Both must agree with
    # the oracle, and a second symbolic run (always after the counts) too.
    rng = np.random.default_rng(n)
    k = 2000
    A = rand_csc(rng, 4000, k, 0.004)
    Bi = _with_long_columns(rng, k, n, 2, {3: 400, 700: 900, n - 1: 1500})
    offs = synth.partition_offsets(k, 4)
    st, sbin, _ = check_local(A, Bi, offs, 32)
    assert 0 < int((sbin == 1).sum()) < n  # tiny and other bins both present
    ref = oracle.local_product(A, Bi, offs, 32)
    Ad, Bd = _dev(A, torch.float64), _dev(Bi, torch.float64)
    with spg.Plan(Ad, Bd, offs, 32) as p:
        for _ in range(2):
            colptr = p.symbolic()
            assert np.array_equal(colptr.cpu().numpy(), ref.C.colptr)
            rows, vals = p.numeric()
            assert np.array_equal(rows.cpu().numpy(), ref.C.rowidx)
            assert_values(vals.cpu().numpy(), ref.C.vals, ref.C.absvals, True)


@pytest.mark.parametrize("case", ["emptyB", "one_row", "one_col", "P_equals_k", "all_empty_A"])
def test_edge_cases(case):
    rng = np.random.default_rng(7)
    if case == "emptyB":
        A = rand_csc(rng, 50, 40, 0.1)
        Bi = synth.from_triplets(40, 10, [], [], [])
        offs = synth.partition_offsets(40, 4)
    elif case == "one_row":
        A = rand_csc(rng, 1, 30, 0.5)
        Bi = rand_csc(rng, 30, 20, 0.2)
        offs = synth.partition_offsets(30, 3)
    elif case == "one_col":
        A = rand_csc(rng, 40, 1, 1.0)
        Bi = rand_csc(rng, 1, 25, 0.7)
        offs = synth.partition_offsets(1, 1)
    elif case == "P_equals_k":
        A = rand_csc(rng, 30, 12, 0.3)
        Bi = rand_csc(rng, 12, 9, 0.3)
        offs = synth.partition_offsets(12, 12)
    else:
        A = synth.from_triplets(20, 15, [], [], [])
        Bi = rand_csc(rng, 15, 6, 0.4)
        offs = synth.partition_offsets(15, 2)
    check_local(A, Bi, offs, 2)


def _bin_tunings():
    return {
        "default": None,
        "all_dense": spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0),
        "all_dense_windows": spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0,
                                        dense_window=32),
        "no_tiny": spg.tuning(tiny_max_flop=0),
        "small_hash": spg.tuning(hash_max_flop=128, hash_max_nnz=128),
        "mid_hash": spg.tuning(hash_max_flop=512, hash_max_nnz=256),
        "force_hash": spg.tuning(tiny_max_flop=0, medium_kernel=1),
        "force_bitmap": spg.tuning(tiny_max_flop=0, medium_kernel=2),
    }


@pytest.mark.parametrize("name", ["default", "all_dense", "all_dense_windows", "no_tiny",
                                  "small_hash", "mid_hash", "force_hash", "force_bitmap"])
def test_every_bin_gives_the_same_product(name):
    """Bin thresholds move columns between kernels but never change C."""
    A = synth.rmat(11, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
    tun = _bin_tunings()[name]
    st, sbin, nbin = check_local(A, A, synth.partition_offsets(A.ncols, 1), 64, tun=tun)
    print(name, "sym bins", st["sym_bins"], "num bins", st["num_bins"], flush=True)
    if name in ("all_dense", "all_dense_windows"):
        assert set(np.unique(nbin)) <= {0, 6, 7}


@pytest.mark.parametrize("kernel", [1, 2])
def test_er_medium_bins_hash_and_bitmap(kernel):
    """ER columns with ~256 and ~1000 entries through both medium kernels."""
    A = synth.erdos_renyi(20000, 20000, 16, seed=21)
    B = synth.erdos_renyi(20000, 300, 16, seed=22)
    B2 = synth.erdos_renyi(20000, 200, 64, seed=23)
    for Bi in (B, B2):
        check_local(A, Bi, synth.partition_offsets(20000, 4), 128,
                    tun=spg.tuning(medium_kernel=kernel))


def test_dense_windows_on_big_columns():
    """Dense-bin columns split into many rank windows (window of 64 rows)."""
    A = synth.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, seed=4)
    st, _, nbin = check_local(A, A, synth.partition_offsets(A.ncols, 2), 256,
                              tun=spg.tuning(dense_window=64, hash_max_nnz=128))
    assert (nbin == 6).sum() > 0


@pytest.mark.parametrize("dense", [False, True])
def test_flat_short_list_at_its_length_limit(dense):
    """Every column of A holds exactly 64 entries (the longest a flat short
    list takes) and B_i columns hold 1024 and more entries: one staged chunk
    of 1024 entries then lists 65536 terms, the most its packed scan holds.
    m above 2^18 sends dense columns through the banded symbolic walk."""
    rng = np.random.default_rng(77)
    m, k = (1 << 18) + 1000, 3000
    rows = np.concatenate([rng.choice(m, size=64, replace=False) for _ in range(k)])
    cols = np.repeat(np.arange(k), 64)
    A = synth.from_triplets(m, k, rows, cols, rng.uniform(-1.0, 1.0, rows.size))
    Bi = _with_long_columns(rng, k, 5, 2, {0: 1024, 1: 2048, 3: 1500})
    tun = spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0) if dense else None
    st, _, nbin = check_local(A, Bi, synth.partition_offsets(k, 1), 64, tun=tun)
    if dense:
        assert set(np.unique(nbin)) <= {0, 6, 7}


@pytest.mark.parametrize("first", [1, 3000])
def test_dense_first_bin_and_self_resetting_queues(first):
    """Dense columns with at least dense_first_flop products go to numeric
    bin 7 and are handed out before the others by the same work-queue
    kernel; running symbolic and numeric twice on one plan checks that the
    dense kernels' queues put themselves back to 0 after every launch."""
    A = synth.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, seed=5)
    ref = oracle.spgemm(A, A)
    tun = spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0, dense_window=64,
                     dense_first_flop=first)
    st, _, nbin = check_local(A, A, synth.partition_offsets(A.ncols, 1), 256, tun=tun)
    print("num bins", st["num_bins"], flush=True)
    assert (nbin == 7).sum() > 0
    if first > 1:
        assert (nbin == 6).sum() > 0
    Ad = _dev(A, torch.float64)
    with spg.Plan(Ad, Ad, None, 256, tuning=tun) as p:
        for _ in range(2):
            c = p.symbolic().cpu().numpy()
            r, v = p.numeric()
            assert np.array_equal(c, ref.colptr)
            assert np.array_equal(r.cpu().numpy(), ref.rowidx)
            assert_values(v.cpu().numpy(), ref.vals, ref.absvals, True)


def test_medium_bitmap_queue_over_two_bins_and_reruns():
    """Both medium bins on the bitmap kernel: two launches share one work
    queue, which each launch puts back to 0; numeric twice on one plan."""
    A = synth.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, seed=6)
    ref = oracle.spgemm(A, A)
    tun = spg.tuning(medium_kernel=2, hash_max_nnz=2048)
    Ad = _dev(A, torch.float64)
    with spg.Plan(Ad, Ad, None, 256, tuning=tun) as p:
        c = p.symbolic().cpu().numpy()
        st = p.stats()
        print("num bins", st["num_bins"], flush=True)
        assert sum(1 for b in (2, 3, 4, 5) if st["num_bins"][b] > 0) >= 2
        for _ in range(2):
            r, v = p.numeric()
            assert np.array_equal(c, ref.colptr)
            assert np.array_equal(r.cpu().numpy(), ref.rowidx)
            assert_values(v.cpu().numpy(), ref.vals, ref.absvals, True)


def test_export_of_partial_group_before_empty_tail():
    """A partition whose last tile holds no nonzero column: its final, short
    group must still report its last column."""
    rng = np.random.default_rng(11)
    k = 3000
    A = rand_csc(rng, 40, k, 0.05, empty_cols=tuple(range(2000, 3000)))
    Bi = rand_csc(rng, k, 30, 0.01)
    check_local(A, Bi, synth.partition_offsets(k, 1), 300)
    check_local(A, Bi, synth.partition_offsets(k, 2), 7)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rmat_scale12_both_dtypes(dtype):
    A = synth.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
    check_local(A, A, synth.partition_offsets(A.ncols, 1), 256, dtype=dtype)


@pytest.mark.parametrize("b", [256, 64, 1024, 1])
def test_er65536_partition0_block_sizes(b):
    w = synth.workload("er65536_d16_p16")
    offs = w["offsets"]
    Bi = synth.column_slice(w["B"], int(offs[0]), int(offs[1]))
    st, _, _ = check_local(w["A"], Bi, offs, b)
    if b >= 64:
        assert st["kt"] == 65536 and st["nnz_At"] == w["A"].nnz  # every block is hit


@pytest.mark.parametrize("own", [0, 2])
def test_own_partition_taken_whole(own):
    """The own partition's nonzero columns all enter A~; the rest follows
    Alg. 2; C_i is unchanged."""
    A = synth.rmat(12, 8, 0.57, 0.19, 0.19, 0.05, seed=13)
    offs = synth.partition_offsets(A.ncols, 4)
    Bi = synth.column_slice(A, int(offs[own]), int(offs[own + 1]))
    tun = spg.tuning(own_partition=own, own_partition_whole=1)
    check_local(A, Bi, offs, 16, tun=tun, own_whole=own)


@pytest.mark.parametrize("i", list(range(1, 16)))
def test_er65536_other_partitions(i):
    """Every other partition of the ER 65536 workload (partition 0 is checked
    at four block sizes above), each stage bit for bit."""
    w = synth.workload("er65536_d16_p16")
    offs = w["offsets"]
    Bi = synth.column_slice(w["B"], int(offs[i]), int(offs[i + 1]))
    check_local(w["A"], Bi, offs, 256)


def test_numeric_rerun_with_new_values():
    """Same patterns, new values of A and B_i (gathered again into A~)."""
    rng = np.random.default_rng(5)
    A = synth.erdos_renyi(3000, 2000, 6, seed=11)
    B = synth.erdos_renyi(2000, 700, 5, seed=12)
    offs = synth.partition_offsets(2000, 4)
    Ad, Bd = _dev(A, torch.float64), _dev(B, torch.float64)
    with spg.Plan(Ad, Bd, offs, 16) as p:
        p.symbolic()
        p.numeric()
        A2 = synth.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, rng.uniform(-2, 2, A.nnz))
        B2 = synth.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, rng.uniform(-2, 2, B.nnz))
        rows, vals = p.numeric(torch.tensor(A2.vals, device="cuda"),
                               torch.tensor(B2.vals, device="cuda"))
        ref = oracle.spgemm(A2, B2)
        assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
        assert_values(vals.cpu().numpy(), ref.vals, ref.absvals, True)


@pytest.mark.parametrize("tiny", [256, 512])
def test_symbolic_rerun_on_one_plan(tiny):
    """A second symbolic phase on the same plan (it clears its own counters)
    gives the same pointers, bins and product; both tiny register widths."""
    A = synth.rmat(12, 8, 0.57, 0.19, 0.19, 0.05, seed=9)
    ref = oracle.spgemm(A, A)
    Ad = _dev(A, torch.float64)
    with spg.Plan(Ad, Ad, None, 64, tuning=spg.tuning(tiny_max_flop=tiny)) as p:
        c1 = p.symbolic().cpu().numpy()
        f1, s1, n1 = [t.cpu().numpy() for t in p.export_bins()]
        st1 = p.stats()
        r1, v1 = p.numeric()
        c2 = p.symbolic().cpu().numpy()
        f2, s2, n2 = [t.cpu().numpy() for t in p.export_bins()]
        st2 = p.stats()
        r2, v2 = p.numeric()
    assert np.array_equal(c1, ref.colptr) and np.array_equal(c2, ref.colptr)
    assert np.array_equal(f1, f2) and np.array_equal(s1, s2) and np.array_equal(n1, n2)
    assert st1["flops"] == st2["flops"] and st1["num_bins"] == st2["num_bins"]
    assert st1["sym_bins"] == st2["sym_bins"] and st2["nnz_C"] == ref.colptr[-1]
    for r, v in ((r1, v1), (r2, v2)):
        assert np.array_equal(r.cpu().numpy(), ref.rowidx)
        assert_values(v.cpu().numpy(), ref.vals, ref.absvals, True)


@pytest.mark.parametrize("tiny,d", [(256, 24), (512, 40)])
def test_tall_a_uses_unpacked_tiny_keys(tiny, d):
    """m above 2^22 rows: the tiny-column sort carries (row, value) pairs
    instead of packed (row, slot) keys; 8*d products per column take 4 or 8
    terms per lane."""
    A = synth.erdos_renyi(5_000_000, 1500, 8, seed=21)
    B = synth.erdos_renyi(1500, 300, d, seed=22)
    check_local(A, B, synth.partition_offsets(1500, 3), 32, tun=spg.tuning(tiny_max_flop=tiny))


def test_validation_on_device_rejects_unsorted_rows():
    A = synth.erdos_renyi(100, 50, 4, seed=1)
    bad = synth.CSC(A.nrows, A.ncols, A.colptr, A.rowidx.copy(), A.vals)
    bad.rowidx[0], bad.rowidx[1] = bad.rowidx[1], bad.rowidx[0]
    B = synth.erdos_renyi(50, 10, 3, seed=2)
    with pytest.raises(spg.SpgemmError) as e:
        spg.Plan(_dev(bad, torch.float64), _dev(B, torch.float64), None, 4,
                 tuning=spg.tuning(validate=1))
    assert e.value.code == -1
    # the valid pair passes validation
    with spg.Plan(_dev(A, torch.float64), _dev(B, torch.float64), None, 4,
                  tuning=spg.tuning(validate=1)) as p:
        p.run()


def test_numeric_before_symbolic_is_a_state_error():
    A = synth.erdos_renyi(100, 50, 4, seed=1)
    B = synth.erdos_renyi(50, 10, 3, seed=2)
    with spg.Plan(_dev(A, torch.float64), _dev(B, torch.float64)) as p:
        lib = spg.load()
        rc = lib.spgemm_numeric(p.handle, None, None, None, None)
        assert rc == -5


def test_workspace_limit_forces_enomem():
    A = synth.erdos_renyi(100, 50, 4, seed=1)
    B = synth.erdos_renyi(50, 10, 3, seed=2)
    with pytest.raises(spg.SpgemmError) as e:
        spg.Plan(_dev(A, torch.float64), _dev(B, torch.float64), None, 4,
                 tuning=spg.tuning(workspace_limit=1024))
    assert e.value.code == -2


def test_plans_reuse_pooled_workspace():
    """Many plan/destroy cycles on one stream stay correct (pooled blocks)."""
    A = synth.erdos_renyi(2000, 2000, 8, seed=1)
    ref = oracle.spgemm(A, A)
    Ad = _dev(A, torch.float64)
    for _ in range(5):
        C = spg.spgemm(Ad, Ad, None, 64)
        assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)


def test_set_stream_between_symbolic_and_numeric():
    """spgemm_plan_set_stream right after a symbolic phase whose counts are
    still in flight (one-workgroup scan, n <= 8192): the counts are read
    before the switch and the new stream's work is ordered after the old
    stream's, so numeric on the new stream gives the oracle's product."""
    A = synth.erdos_renyi(4096, 4096, 12, seed=61)
    B = synth.erdos_renyi(4096, 2000, 9, seed=62)
    ref = oracle.spgemm(A, B)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Ad, Bd = _dev(A, torch.float64), _dev(B, torch.float64)
    torch.cuda.synchronize()
    for rep in range(3):
        with spg.Plan(Ad, Bd, None, 64, stream=s1) as p:
            colptr = p.symbolic()
            p.set_stream(s2)
            with torch.cuda.stream(s2):
                rows, vals = p.numeric()
            s2.synchronize()
            assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
            assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
            assert_values(vals.cpu().numpy(), ref.vals, ref.absvals, True)
