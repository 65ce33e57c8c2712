"""GPU tests of the batched form: the numeric phase of many planned products
(the 64^3 AMG Galerkin hierarchy, four levels, chained; plus 64 independent
ER products of uneven sizes) as one dependency DAG, with the products of a
depth that have tiny and hash columns only sharing one launch per bin
(tuning.batch_form = 0) or every product launching its own kernels on side
streams (batch_form = 2), directly and as a captured hipGraph replayed
several times; and the same table as one persistent launch
(batch_form = 1)."""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _levels(n, levels):
    out = []
    for _ in range(levels):
        out.append((spg.DeviceCsc.from_host(synth.aggregation3d(n)),
                    spg.DeviceCsc.from_host(synth.aggregation3d_t(n))))
        n //= 2
    return out


@pytest.fixture(scope="module")
def workload():
    A0 = spg.DeviceCsc.from_host(synth.laplacian3d(64))
    plans, io, outs = spg.galerkin_chain(A0, _levels(64, 4))
    er = []
    for A, B in synth.er_batch(64, seed=4):
        Ad, Bd = spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B)
        p = spg.Plan(Ad, Bd, None, 64)
        C = p.run()
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
        outs.append(C)
        er.append((A, B))
    torch.cuda.synchronize()
    return A0, plans, io, outs, er


def _check_amg(outs, scale=1.0):
    n = 64
    for lvl in range(4):
        AP = outs[2 * lvl]
        vals = set(torch.unique(AP.vals).cpu().numpy().tolist())
        assert vals == {3.0 * 4 ** lvl * scale, -1.0 * 4 ** lvl * scale}
        n //= 2
        ref = synth.laplacian3d(n)
        Ac = outs[2 * lvl + 1]
        assert np.array_equal(Ac.rowidx.cpu().numpy(), ref.rowidx)
        assert np.array_equal(Ac.vals.cpu().numpy(), scale * 4.0 ** (lvl + 1) * ref.vals)


def _check_er(outs, er):
    for t, (A, B) in enumerate(er):
        C = outs[8 + t]
        ref = oracle.spgemm(A, B)
        assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)
        assert_values(C.vals.cpu().numpy(), ref.vals, ref.absvals, True)


def test_plain_chain_is_exact(workload):
    _check_amg(workload[3])


def test_batched_direct_launch(workload):
    A0, plans, io, outs, er = workload
    b = spg.Batch(plans, io)
    streams, launches = b.info()
    print("batch side streams", streams, "launches", launches, flush=True)
    # at depth 0 the ER products of at most 4096 columns share one launch
    # per non-empty bin and kernel; the larger ones and the chain run their
    # own kernels
    sep = spg.Batch(plans, io, spg.tuning(batch_form=2))
    streams2, launches2 = sep.info()
    sep.close()
    assert streams == 4 and launches < launches2
    assert streams2 == 4 and launches2 >= len(plans)
    for C in outs:
        C.vals.fill_(-7.0)
        C.rowidx.fill_(-1)
    b.run(0)
    b.check()
    _check_amg(outs)
    _check_er(outs, er)
    b.close()


def test_batched_graph_replays(workload):
    A0, plans, io, outs, er = workload
    s = torch.cuda.Stream()
    b = spg.Batch(plans, io)
    with torch.cuda.stream(s):
        b.run(1, stream=s)
    b.check()
    _check_amg(outs)
    for rep in range(3):
        with torch.cuda.stream(s):
            for C in outs:      # eager work between replays
                C.vals.zero_()
            A0.vals.mul_(2.0)   # new fine-level values propagate down the chain
            b.run(2, stream=s)
        b.check()
        _check_amg(outs, scale=2.0 ** (rep + 1))
    with torch.cuda.stream(s):
        A0.vals.mul_(2.0 ** -3)
        b.run(2, stream=s)
    b.check()
    _check_amg(outs)
    _check_er(outs, er)
    b.close()


def test_batched_stream_counts_give_the_same_results(workload):
    A0, plans, io, outs, er = workload
    for tun in (spg.tuning(batch_streams=1), spg.tuning(batch_streams=8),
                spg.tuning(batch_form=2), spg.tuning(batch_form=2, batch_streams=1)):
        b = spg.Batch(plans, io, tun)
        for C in outs:
            C.vals.fill_(3.0)
        b.run(0)
        b.check()
        _check_amg(outs)
        _check_er(outs, er)
        b.close()


def test_batched_errors(workload):
    A0, plans, io, outs, er = workload
    bad = [dict(x) for x in io[:3]]
    bad[1]["dep_A"] = 2  # forward dependency
    with pytest.raises(spg.SpgemmError) as e:
        spg.Batch(plans[:3], bad)
    assert e.value.code == -1
    with pytest.raises(spg.SpgemmError) as e:  # one plan twice
        spg.Batch([plans[8], plans[8]], [io[8], io[8]])
    assert e.value.code == -1
    with pytest.raises(spg.SpgemmError) as e:
        spg.Batch(plans[:2], io[:2], spg.tuning(batch_streams=9))
    assert e.value.code == -1
    with pytest.raises(spg.SpgemmError) as e:
        spg.Batch(plans[:2], io[:2], spg.tuning(batch_form=3))
    assert e.value.code == -1
    b = spg.Batch(plans[:2], io[:2])
    lib = spg.load()
    assert lib.spgemm_batch_run(b.handle, 2, None) == -5  # replay before capture
    assert lib.spgemm_batch_run(b.handle, 7, None) == -1
    b.close()
    A = spg.DeviceCsc.from_host(synth.erdos_renyi(100, 100, 4, seed=1))
    p = spg.Plan(A, A)
    with pytest.raises(spg.SpgemmError) as e:
        spg.Batch([p], [{"C_rowidx": A.rowidx, "C_vals": A.vals}])
    assert e.value.code == -5  # symbolic has not run


def test_graph_replays_of_dense_queue_kernels():
    """A batch whose products run the dense kernels (all dense bins, small
    windows; one product with dense-first columns): the work-queue counters
    live in each plan's device counters and put themselves back to 0 at the
    end of every launch, so every replay of the captured graph computes the
    same product."""
    tun_all = spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0, dense_window=64,
                         dense_first_flop=2000)
    mats = [synth.rmat(11, 16, 0.57, 0.19, 0.19, 0.05, seed=s) for s in (31, 32)]
    plans, io, refs = [], [], []
    for M in mats:
        Md = spg.DeviceCsc.from_host(M)
        p = spg.Plan(Md, Md, None, 64, tuning=tun_all)
        C = p.run()
        st = p.stats()
        assert st["num_bins"][6] + st["num_bins"][7] > 0
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
        refs.append(oracle.spgemm(M, M))
    s = torch.cuda.Stream()
    for p in plans:
        p.set_stream(s)
    # the persistent form takes tiny and hash columns only
    with pytest.raises(spg.SpgemmError) as e:
        spg.Batch(plans, io, spg.tuning(batch_form=1))
    assert e.value.code == -4
    b = spg.Batch(plans, io)
    try:
        b.run(1, stream=s)
        for rep in range(3):
            with torch.cuda.stream(s):  # cleared in stream order before the replay
                for d in io:
                    d["C_vals"].zero_()
            b.run(2, stream=s)
            s.synchronize()
            for d, ref in zip(io, refs):
                assert np.array_equal(d["C_rowidx"].cpu().numpy(), ref.rowidx)
                assert_values(d["C_vals"].cpu().numpy(), ref.vals, ref.absvals, True)
        b.check()
    finally:
        b.close()
        for p in plans:
            p.close()


def _device(M, dt):
    return spg.DeviceCsc(M.nrows, M.ncols, torch.as_tensor(M.colptr).cuda(),
                         torch.as_tensor(M.rowidx).cuda(),
                         torch.as_tensor(np.asarray(M.vals)).to(dt).cuda())


def test_grouped_depths_with_dense_products_and_dependencies():
    """Depth 0 holds five small ER products without dense columns (one
    grouped launch per bin and kernel) beside two R-MAT squares whose columns
    are all dense (their own kernels on side streams); depth 1 holds two grouped
    products that read depth-0 outputs: A1 * C_0 (B values are product 0's C,
    read in place) and C_1 * S (A values are product 1's C, gathered into
    A~ first, since S needs few of C_1's columns).  Unit values make every
    result an integer, so the batch is compared exactly with the oracle,
    directly, captured and replayed, in FP64 and FP32."""
    tun_dense = spg.tuning(tiny_max_flop=0, hash_max_flop=0, hash_max_nnz=0, dense_window=64)
    for dt in (torch.float64, torch.float32):
        # five products small enough to be grouped (at most 4096 columns),
        # from tiny to medium columns (d = 32: about 1000 products a column)
        host = []
        for t, (n, d) in enumerate(((500, 4), (1200, 8), (2500, 12), (3000, 20), (4000, 32))):
            host.append((synth.unit_values(synth.erdos_renyi(n, n, d, seed=50 + t)),
                         synth.unit_values(synth.erdos_renyi(n, n, d, seed=60 + t)), None))
        for sd in (41, 42):
            M = synth.unit_values(synth.rmat(10, 16, 0.57, 0.19, 0.19, 0.05, seed=sd))
            host.append((M, M, tun_dense))
        plans, io, refs = [], [], []
        for A, B, tun in host:
            p = spg.Plan(_device(A, dt), _device(B, dt), None, 64, tuning=tun)
            C = p.run()
            plans.append(p)
            io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
            refs.append(oracle.spgemm(A, B))
        C0, C1 = refs[0], refs[1]
        A1 = synth.unit_values(synth.erdos_renyi(C0.nrows, C0.nrows, 2, seed=43))
        p = spg.Plan(_device(A1, dt), _device(C0, dt), None, 64)
        C = p.run()
        plans.append(p)
        io.append({"B_vals": io[0]["C_vals"], "C_rowidx": C.rowidx, "C_vals": C.vals,
                   "dep_B": 0})
        refs.append(oracle.spgemm(A1, C0))
        S = synth.unit_values(synth.erdos_renyi(C1.ncols, 4, 1, seed=44))
        p = spg.Plan(_device(C1, dt), _device(S, dt), None, 64)
        C = p.run()
        assert p.stats()["nnz_At"] < C1.colptr[-1]  # part of C_1: a value gather
        plans.append(p)
        io.append({"A_vals": io[1]["C_vals"], "C_rowidx": C.rowidx, "C_vals": C.vals,
                   "dep_A": 1})
        refs.append(oracle.spgemm(C1, S))
        dense = [not _no_dense(q) for q in plans]
        assert dense == [False] * 5 + [True, True] + [False, False]
        s = torch.cuda.Stream()
        b = spg.Batch(plans, io)
        try:
            streams, launches = b.info()
            assert streams >= 2  # the dense products beside depth 0's grouped launches
            sep = spg.Batch(plans, io, spg.tuning(batch_form=2))
            assert launches < sep.info()[1]
            sep.close()
            for mode in (0, 1, 2, 2):
                with torch.cuda.stream(s):
                    for d in io:
                        d["C_vals"].fill_(-3.0)
                        d["C_rowidx"].fill_(-1)
                    b.run(mode, stream=s)
                s.synchronize()
                b.check()
                for d, ref in zip(io, refs):
                    assert np.array_equal(d["C_rowidx"].cpu().numpy(), ref.rowidx)
                    assert np.array_equal(d["C_vals"].cpu().double().numpy(), ref.vals)
        finally:
            b.close()
            for q in plans:
                q.close()


def test_grouped_many_small_products():
    """Two hundred independent small ER products (100-800 columns, 2-8 per
    column): the default form puts all of them in one launch per bin and
    kernel; direct run, capture and replays against the oracle."""
    rng = np.random.default_rng(7)
    plans, io, refs = [], [], []
    for t in range(200):
        n = int(rng.integers(100, 801))
        d = int(rng.integers(2, 9))
        A = synth.erdos_renyi(n, n, d, seed=1000 + 2 * t)
        B = synth.erdos_renyi(n, n, d, seed=1001 + 2 * t)
        p = spg.Plan(spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B), None, 64)
        C = p.run()
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
        refs.append(oracle.spgemm(A, B))
    s = torch.cuda.Stream()
    b = spg.Batch(plans, io)
    try:
        streams, launches = b.info()
        assert launches <= 5  # tiny, and one per medium bin present
        for mode in (0, 1, 2, 2):
            with torch.cuda.stream(s):
                for d in io:
                    d["C_vals"].fill_(-3.0)
                b.run(mode, stream=s)
            s.synchronize()
            b.check()
            for d, ref in zip(io, refs):
                assert np.array_equal(d["C_rowidx"].cpu().numpy(), ref.rowidx)
                assert_values(d["C_vals"].cpu().numpy(), ref.vals, ref.absvals, True)
    finally:
        b.close()
        for p in plans:
            p.close()


def test_grouped_medium_columns_of_tall_products():
    """Grouped products whose medium columns go to the LDS bitmap over more
    than 65536 rows (the wide bitmap launch) beside one with fewer rows, in
    FP64 and FP32, against the oracle and against the separate form."""
    shapes = ((100000, 40, 30, 71), (70000, 40, 24, 72), (30000, 40, 30, 73))
    for dt in (torch.float64, torch.float32):
        plans, io, refs = [], [], []
        for m, da, db, sd in shapes:
            A = synth.erdos_renyi(m, 2000, da, seed=sd)
            B = synth.erdos_renyi(2000, 500, db, seed=sd + 100)
            p = spg.Plan(spg.DeviceCsc.from_host(A, dtype=dt), spg.DeviceCsc.from_host(B, dtype=dt),
                         None, 64)
            C = p.run()
            st = p.stats()
            assert sum(st["num_bins"][2:6]) > 0 and st["num_bins"][6] + st["num_bins"][7] == 0
            plans.append(p)
            io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
            refs.append(oracle.spgemm(synth.as_fp32(A) if dt == torch.float32 else A,
                                      synth.as_fp32(B) if dt == torch.float32 else B))
        b = spg.Batch(plans, io)
        sep = spg.Batch(plans, io, spg.tuning(batch_form=2))
        try:
            assert b.info()[1] < sep.info()[1]
            for bb in (b, sep):
                for d in io:
                    d["C_vals"].fill_(-3.0)
                bb.run(0)
                bb.check()
                for d, ref in zip(io, refs):
                    assert np.array_equal(d["C_rowidx"].cpu().numpy(), ref.rowidx)
                    assert_values(d["C_vals"].cpu().numpy(), ref.vals, ref.absvals,
                                  dt == torch.float64)
        finally:
            b.close()
            sep.close()
            for p in plans:
                p.close()


def test_spgemm_batched_by_table(workload):
    """spgemm_batched(count, plans, io, mode, stream): mode 0 runs the table,
    mode 1 captures and launches it, mode 2 replays that capture (with new
    fine-level values propagating down the chain); a replay of a table that
    was never captured is an ordering error."""
    A0, plans, io, outs, er = workload
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for C in outs:
            C.vals.fill_(-7.0)
        spg.batched(plans, io, 0, stream=s)
    s.synchronize()
    _check_amg(outs)
    _check_er(outs, er)
    with torch.cuda.stream(s):
        for C in outs:
            C.vals.zero_()
        spg.batched(plans, io, 1, stream=s)
    s.synchronize()
    _check_amg(outs)
    for rep in range(2):
        with torch.cuda.stream(s):
            for C in outs:
                C.vals.zero_()
            A0.vals.mul_(2.0)
            spg.batched(plans, io, 2, stream=s)
        s.synchronize()
        _check_amg(outs, scale=2.0 ** (rep + 1))
    with torch.cuda.stream(s):
        A0.vals.mul_(0.25)
        spg.batched(plans, io, 2, stream=s)
    s.synchronize()
    _check_amg(outs)
    _check_er(outs, er)
    with pytest.raises(spg.SpgemmError) as e:  # this sub-table was never captured
        spg.batched(plans[:2], io[:2], 2)
    assert e.value.code == -5
    with pytest.raises(spg.SpgemmError) as e:
        spg.batched(plans[:2], io[:2], 3)
    assert e.value.code == -1


def _no_dense(p):
    st = p.stats()
    return st["num_bins"][6] + st["num_bins"][7] == 0


def test_persistent_batch_matches_plain(workload):
    """tuning.batch_form = 1: the AMG chain and the ER products without
    dense columns as ONE persistent launch (items by ticket in dependency
    order, per-item completion flags, bounded waits).  Direct runs, a
    capture and replays with new fine-level values give the plain results,
    and the batch's error word stays clear."""
    A0, plans, io, outs, er = workload
    keep = [t for t, p in enumerate(plans) if _no_dense(p)]
    assert keep[:8] == list(range(8))
    print("persistent batch of", len(keep), "products", flush=True)
    b = spg.Batch([plans[t] for t in keep], [io[t] for t in keep],
                  spg.tuning(batch_form=1))
    streams, launches = b.info()
    assert streams == 0 and launches == 1

    def check(scale=1.0):
        _check_amg(outs, scale)
        for t in keep[8:]:
            A, B = er[t - 8]
            ref = oracle.spgemm(A, B)
            C = outs[t]
            assert np.array_equal(C.rowidx.cpu().numpy(), ref.rowidx)
            assert_values(C.vals.cpu().numpy(), ref.vals, ref.absvals, True)

    s = torch.cuda.Stream()
    try:
        for rep in range(2):
            with torch.cuda.stream(s):
                for t in keep:
                    outs[t].vals.fill_(-7.0)
                    outs[t].rowidx.fill_(-1)
                b.run(0, stream=s)
            b.check()
            check()
        with torch.cuda.stream(s):
            b.run(1, stream=s)
        b.check()
        check()
        for rep in range(3):
            with torch.cuda.stream(s):
                for t in keep:
                    outs[t].vals.zero_()
                A0.vals.mul_(2.0)
                b.run(2, stream=s)
            b.check()
            check(2.0 ** (rep + 1))
        with torch.cuda.stream(s):
            A0.vals.mul_(2.0 ** -3)
            b.run(2, stream=s)
        b.check()
        check()
    finally:
        b.close()


def test_persistent_batch_fp32_with_a_dependency():
    """The persistent launch in FP32: ER products (tiny and hash columns) and
    one product whose B is another product's C (read inside the launch),
    against the oracle on FP32-rounded inputs (normwise)."""
    pairs = synth.er_batch(3, seed=12)
    plans, io, refs = [], [], []
    for A, B in pairs:
        p = spg.Plan(spg.DeviceCsc.from_host(A, dtype=torch.float32),
                     spg.DeviceCsc.from_host(B, dtype=torch.float32), None, 64)
        C = p.run()
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
        refs.append(oracle.spgemm(synth.as_fp32(A), synth.as_fp32(B)))
    # A1 * C_0 with a sparse A1: its B values are product 0's C
    C0 = refs[0]
    C0f = synth.CSC(C0.nrows, C0.ncols, C0.colptr, C0.rowidx,
                    np.asarray(C0.vals, dtype=np.float32).astype(np.float64))
    A1 = synth.erdos_renyi(C0.nrows, C0.nrows, 2, seed=13)
    Cd0 = spg.DeviceCsc(C0.nrows, C0.ncols, torch.as_tensor(C0.colptr).cuda(),
                        torch.as_tensor(C0.rowidx).cuda(),
                        torch.as_tensor(np.asarray(C0f.vals, dtype=np.float32)).cuda())
    p3 = spg.Plan(spg.DeviceCsc.from_host(A1, dtype=torch.float32), Cd0, None, 64)
    C3 = p3.run()
    plans.append(p3)
    io.append({"B_vals": io[0]["C_vals"], "C_rowidx": C3.rowidx, "C_vals": C3.vals, "dep_B": 0})
    refs.append(oracle.spgemm(synth.as_fp32(A1), C0f))
    assert all(_no_dense(p) for p in plans)
    b = spg.Batch(plans, io, spg.tuning(batch_form=1))
    try:
        for rep in range(2):
            for d in io:
                d["C_vals"].fill_(-3.0)
            b.run(0)
            b.check()
            for d, ref in zip(io, refs):
                assert np.array_equal(d["C_rowidx"].cpu().numpy(), ref.rowidx)
                assert_values(d["C_vals"].cpu().numpy(), ref.vals, ref.absvals, False)
    finally:
        b.close()
        for p in plans:
            p.close()
