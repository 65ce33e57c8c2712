#!/usr/bin/env python3
"""Benchmark of the local SpGEMM hot path on one MI355X.

A step is one pass of the whole path for one partition: spgemm_plan (H_i,
Alg. 2 block selection, column map, gather of A~), spgemm_symbolic (flops,
binning, nnz count, scan) and spgemm_numeric, with inputs resident in HBM.

Default workload (N=1): C = A * A for A the R-MAT scale-18 matrix (262,144
rows and columns, edge factor 16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
duplicates merged, U(0,1) values, FP64), one partition (the largest
single-GPU configuration).  The other configurations are reported beside it
under "workloads" (warm and with the 256 MB last-level cache flushed before
every step), with the batched and differentiable forms under "batched" and
"backward".  --workload selects another headline.

Prints ONE JSON line.  value = 2 * sparse flops / step time (GFLOP/s).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s + achieved HBM GB/s (% peak); batched/backward vs plain speedup"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the numeric phase, from two rocprofv3 counter
# passes (FETCH_SIZE, then WRITE_SIZE) summarised in
# profiles/numeric_phase_hbm_traffic.md: each of its "traffic-record:" lines
# holds a JSON object with the workload, the scaled bytes and the digest of
# the kernel sources the counters were taken on.  When the sources have
# changed since, traffic is reported as null.
TRAFFIC_SOURCES = ("numeric.hip", "numeric.hpp", "terms.hpp", "common.hpp", "internal.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "numeric_phase_hbm_traffic.md")


def kernel_sources_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2408_14558_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_desc):
    """(bytes, record) of the counter summary for this workload while the
    kernel sources are unchanged, else (None, reason)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [ln for ln in fh if ln.startswith("traffic-record:")]
    except OSError:
        return None, "no counter summary"
    digest = kernel_sources_digest()
    for ln in lines:
        rec = json.loads(ln.split(":", 1)[1])
        if rec.get("workload") == workload_desc:
            if rec.get("sources") != digest:
                return None, f"kernels changed since the counters ({rec.get('sources')} != {digest})"
            return rec["bytes"], rec
    return None, "no counter record for this workload"


def workload(name):
    import synth
    if name == "er65536":
        w = synth.workload("er65536_d16_p16")
        offs = w["offsets"]
        Bi = synth.column_slice(w["B"], int(offs[0]), int(offs[1]))
        return dict(A=w["A"], Bi=Bi, offs=offs, b=256, dtype="f64",
                    desc="er65536_d16_p16_block0_b256",
                    config={"A": "ER 65536x65536, 16/col, U(-1,1), seed 1",
                            "B": "ER 65536x65536, 16/col, U(-1,1), seed 2",
                            "partitions": 16, "partition": 0, "block_size": 256})
    if name in ("rmat18", "rmat18-f32"):
        w = synth.workload("rmat18")
        f32 = name.endswith("f32")
        return dict(A=w["A"], Bi=w["A"], offs=w["offsets"], b=256,
                    dtype="f32" if f32 else "f64",
                    desc=f"rmat18_ef16_AxA_{'f32' if f32 else 'f64'}",
                    config={"A": "R-MAT scale 18, ef 16, (0.57,0.19,0.19,0.05), U(0,1), seed 3",
                            "B": "A", "partitions": 1, "block_size": 256})
    if name == "lap2d":
        w = synth.workload("lap2d_64_p4")
        offs = w["offsets"]
        Bi = synth.column_slice(w["A"], int(offs[0]), int(offs[1]))
        return dict(A=w["A"], Bi=Bi, offs=offs, b=64, dtype="f64", desc="lap2d_64_p4_block0_b64",
                    config={"A": "5-point Laplacian 64x64 grid", "partitions": 4,
                            "partition": 0, "block_size": 64})
    if name == "sketch":
        w = synth.workload("sketch_er131072")
        return dict(A=w["A"], Bi=w["B"], offs=w["offsets"], b=256, dtype="f32",
                    desc="er131072_d8_x_sketch4096_f32",
                    config={"A": "ER 131072^2, 8/col, seed 5",
                            "B": "sign sketch 131072x4096, 4/row, seed 6", "partitions": 1})
    raise SystemExit(f"unknown workload {name}")


def phase_bytes(st, vsize):
    """Algorithmic bytes of the three phases (each input array read once,
    each output written once): plan (H_i, Alg. 2, map, A~), symbolic (counts
    and scan), numeric (values)."""
    k, n, kt = st["k"], st["n"], st["kt"]
    nb, nt, nc = st["nnz_B"], st["nnz_At"], st["nnz_C"]
    plan = 4 * nb + 8 * (k + 1) + k + 4 * k + 2 * (4 + vsize) * nt + 8 * (kt + 1)
    symbolic = 8 * (n + 1) + 4 * nb + 4 * nt + 8 * n
    numeric = (4 + vsize) * (nb + nt + nc) + 8 * (n + 1)
    return {"plan": plan, "symbolic": symbolic, "numeric": numeric}


def _host_cpu():
    model = "?"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return model, os.cpu_count()


def cpu_baseline(w, budget_s=10.0):
    """The oracle as it stands (FP64 C, output columns on OpenMP threads)
    on the host cores: the whole local step (H_i, Alg. 2, A~, flops, C_i)
    for an evenly strided sample of B_i's columns, grown until one pass takes
    between budget_s / 4 and budget_s seconds on one thread; then the same
    sample on every thread the host offers."""
    import oracle
    import synth
    A, Bi = w["A"], w["Bi"]
    if w["dtype"] == "f32":
        A, Bi = synth.as_fp32(A), synth.as_fp32(Bi)
    model, ncpu = _host_cpu()

    def run(cols, threads):
        oracle.set_threads(threads)
        blk = synth.column_subset(Bi, cols)
        t0 = time.perf_counter()
        loc = oracle.local_product(A, blk, w["offs"], w["b"])
        return time.perf_counter() - t0, int(loc.flop.sum()), oracle.threads()

    stride = max(1, Bi.ncols // 256)
    el, flops, _ = run(np.arange(0, Bi.ncols, stride), 1)
    while el < budget_s / 4 and stride > 1:
        stride = max(1, stride // 4)
        el, flops, _ = run(np.arange(0, Bi.ncols, stride), 1)
    cols = np.arange(0, Bi.ncols, stride)
    el_all, flops_all, used = run(cols, 0)
    oracle.set_threads(0)
    sample = (f"{cols.size} of {Bi.ncols} columns of B_i (every {stride}th) through the whole "
              f"local step, {flops} flops")
    return {"value": round(2.0 * flops_all / el_all / 1e9, 4), "unit": "GFLOP/s", "cores": used,
            "kind": "oracle", "sample": sample, "seconds": round(el_all, 3),
            "one_core": {"value": round(2.0 * flops / el / 1e9, 4), "cores": 1,
                         "seconds": round(el, 3)},
            "host": {"cpu_model": model, "nproc": ncpu}}


def _time_on(stream, fn, reps):
    """Average ms of fn() over reps calls, HIP events on `stream` (one
    untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(spg, reps=20):
    """The batched form on its workload: the AMG Galerkin hierarchy of the
    3D 7-point Laplacian on 64^3 (2x2x2 aggregation, 4 levels, A_c =
    P^T (A P), chained) plus 64 independent ER products (seed 4).  Plain =
    every product's spgemm_numeric in order on one stream; batched = one
    replay of the captured DAG (the products of a depth with tiny and hash
    columns only sharing one launch per bin; `separate_graph_replay_ms`:
    every product launching its own kernels).  All gather new A values where
    the chain needs them and write the same outputs."""
    import torch
    import synth
    A0 = spg.DeviceCsc.from_host(synth.laplacian3d(64))
    levels, n = [], 64
    for _ in range(4):
        levels.append((spg.DeviceCsc.from_host(synth.aggregation3d(n)),
                       spg.DeviceCsc.from_host(synth.aggregation3d_t(n))))
        n //= 2
    plans, io, outs = spg.galerkin_chain(A0, levels)
    for A, B in synth.er_batch(64, seed=4):
        p = spg.Plan(spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B), None, 64)
        C = p.run()
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
        outs.append(C)
    torch.cuda.synchronize()
    flops = sum(p.stats()["flops"] for p in plans)
    amg_flops = sum(p.stats()["flops"] for p in plans[:8])
    s = torch.cuda.Stream()
    for p in plans:
        p.set_stream(s)

    def plain():
        for p, d in zip(plans, io):
            p.numeric(d.get("A_vals"), d.get("B_vals"), out=(d["C_rowidx"], d["C_vals"]))

    def plain_amg():
        for p, d in list(zip(plans, io))[:8]:
            p.numeric(d.get("A_vals"), d.get("B_vals"), out=(d["C_rowidx"], d["C_vals"]))

    plain_ms = _time_on(s, plain, reps)
    plain_amg_ms = _time_on(s, plain_amg, reps)
    b = spg.Batch(plans, io)
    eager_ms = _time_on(s, lambda: b.run(0, stream=s), reps)
    b.run(1, stream=s)
    graph_ms = _time_on(s, lambda: b.run(2, stream=s), reps)
    sep = spg.Batch(plans, io, spg.tuning(batch_form=2))
    sep.run(1, stream=s)
    sep_graph_ms = _time_on(s, lambda: sep.run(2, stream=s), reps)
    sep.check()
    sep.close()
    b_amg = spg.Batch(plans[:8], io[:8])
    eager_amg_ms = _time_on(s, lambda: b_amg.run(0, stream=s), reps)
    b_amg.run(1, stream=s)
    graph_amg_ms = _time_on(s, lambda: b_amg.run(2, stream=s), reps)
    b.check()
    streams, launches = b.info()
    # the persistent form (one launch per run) on the AMG chain, and on every
    # product without dense columns against the stream DAG of the same table
    persistent_tun = spg.tuning(batch_form=1)
    p_amg = spg.Batch(plans[:8], io[:8], persistent_tun)
    p_amg_ms = _time_on(s, lambda: p_amg.run(0, stream=s), reps)
    p_amg.run(1, stream=s)
    p_amg_graph_ms = _time_on(s, lambda: p_amg.run(2, stream=s), reps)
    p_amg.check()
    keep = [t for t, p in enumerate(plans)
            if p.stats()["num_bins"][6] + p.stats()["num_bins"][7] == 0]
    sub_plans, sub_io = [plans[t] for t in keep], [io[t] for t in keep]
    p_all = spg.Batch(sub_plans, sub_io, persistent_tun)
    p_all_ms = _time_on(s, lambda: p_all.run(0, stream=s), reps)
    p_all.check()
    d_all = spg.Batch(sub_plans, sub_io)
    d_all.run(1, stream=s)
    d_all_graph_ms = _time_on(s, lambda: d_all.run(2, stream=s), reps)
    d_all.check()
    # many small independent products: one launch per bin and kernel for all
    # of them (the default form) against a launch per product and bin
    rng = np.random.default_rng(6)
    small_plans, small_io = [], []
    for t in range(1024):
        n_t = int(round(math.exp(rng.uniform(math.log(100), math.log(1000)))))
        d_t = int(round(math.exp(rng.uniform(math.log(2), math.log(8)))))
        sd = int(rng.integers(0, 2 ** 31 - 1))
        p = spg.Plan(spg.DeviceCsc.from_host(synth.erdos_renyi(n_t, n_t, d_t, sd)),
                     spg.DeviceCsc.from_host(synth.erdos_renyi(n_t, n_t, d_t, sd + 1)), None, 64)
        C = p.run()
        p.set_stream(s)
        small_plans.append(p)
        small_io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
    torch.cuda.synchronize()
    small_flops = sum(p.stats()["flops"] for p in small_plans)
    small = {}
    for form, key in ((0, "grouped"), (2, "separate")):
        bs = spg.Batch(small_plans, small_io, spg.tuning(batch_form=form))
        bs.run(1, stream=s)
        small[key + "_graph_replay_ms"] = round(_time_on(s, lambda: bs.run(2, stream=s), reps), 4)
        small[key + "_launches"] = bs.info()[1]
        bs.check()
        bs.close()
    for p in small_plans:
        p.close()
    out = {
        "workload": "amg7pt64_4levels_plus_64er_f64",
        "products": len(plans), "launches": launches, "side_streams": streams,
        "flops": int(flops),
        "plain_ms": round(plain_ms, 4), "dag_eager_ms": round(eager_ms, 4),
        "graph_replay_ms": round(graph_ms, 4),
        "speedup_vs_plain": round(plain_ms / graph_ms, 3),
        "separate_graph_replay_ms": round(sep_graph_ms, 4),
        "graph_GFLOPs": round(2 * flops / (graph_ms * 1e-3) / 1e9, 2),
        "amg_only": {"products": 8, "flops": int(amg_flops), "plain_ms": round(plain_amg_ms, 4),
                     "dag_eager_ms": round(eager_amg_ms, 4),
                     "graph_replay_ms": round(graph_amg_ms, 4),
                     "speedup_vs_plain": round(plain_amg_ms / graph_amg_ms, 3),
                     "eager_speedup_vs_plain": round(plain_amg_ms / eager_amg_ms, 3),
                     "persistent_ms": round(p_amg_ms, 4),
                     "persistent_graph_replay_ms": round(p_amg_graph_ms, 4),
                     "persistent_speedup_vs_plain": round(plain_amg_ms / p_amg_ms, 3)},
        "small_products": {"workload": "1024 ER products, n 100-1000, 2-8 per column (seed 6)",
                           "flops": int(small_flops), **small,
                           "grouped_speedup": round(small["separate_graph_replay_ms"] /
                                                    small["grouped_graph_replay_ms"], 3)},
        "no_dense_table": {"products": len(keep), "persistent_ms": round(p_all_ms, 4),
                           "dag_graph_replay_ms": round(d_all_graph_ms, 4)},
    }
    for x in (b, b_amg, p_amg, p_all, d_all):
        x.close()
    for p in plans:
        p.close()
    return out


def bench_backward(spg, reps=10):
    """The differentiable form on its workload (FP32): A = ER 131072^2 at 8
    per column (seed 5), B = 131072 x 4096 sign sketch (4 per row, seed 6),
    dC = U(-1,1) on pattern(C) (seed 7).  Reports the sampled backward
    (dA and dB on the patterns of A and B) against the forward numeric and
    against the plain path computing the unmasked products dC*B^T and
    A^T*dC (plan + symbolic + numeric each; the masking those would still
    need is not timed)."""
    import torch
    import synth
    w = synth.workload("sketch_er131072")
    A = spg.DeviceCsc.from_host(w["A"], dtype=torch.float32)
    B = spg.DeviceCsc.from_host(w["B"], dtype=torch.float32)
    s = torch.cuda.Stream()
    p = spg.Plan(A, B, None, 256, stream=s)
    with torch.cuda.stream(s):
        colptr = p.symbolic()
        rows, vals = p.numeric()
        s.synchronize()
        dC = torch.as_tensor(synth.uniform_values(p.nnzC, seed=7)).to(
            device="cuda", dtype=torch.float32)
        fwd_ms = _time_on(s, lambda: p.numeric(A.vals, B.vals, out=(rows, vals)), reps)
        bwd_ms = _time_on(s, lambda: p.backward(rows, dC, A.vals, B.vals), reps)
        dCm = spg.DeviceCsc(A.nrows, B.ncols, colptr, rows, dC)
        Bt = spg.DeviceCsc.from_host(synth.transpose(w["B"]), dtype=torch.float32)
        At = spg.DeviceCsc.from_host(synth.transpose(w["A"]), dtype=torch.float32)

        def unmasked():
            for L, R in ((dCm, Bt), (At, dCm)):
                q = spg.Plan(L, R, None, 256, stream=s)
                q.run()
                q.close()

        plain_ms = _time_on(s, unmasked, 2)
    st = p.stats()
    p.close()
    return {
        "workload": "er131072_d8_x_sketch4096_f32",
        "forward_flops": int(st["flops"]), "sampled_backward_flops": 2 * int(st["flops"]),
        "forward_numeric_ms": round(fwd_ms, 4), "backward_ms": round(bwd_ms, 4),
        "backward_over_forward": round(bwd_ms / fwd_ms, 3),
        "unmasked_plain_ms": round(plain_ms, 4),
        "speedup_vs_plain": round(plain_ms / bwd_ms, 2),
    }


def study_gather_volume(spg, blocks=(1, 16, 64, 256, 1024, 4096), P=16, reps=3):
    """Gather volume of the block-fetch rule (Alg. 2) against the block size b
    and the ordering of the input: R-MAT 18 (C = A*A, B_i = A's i-th column
    block of P) in its generated order and under a seeded random symmetric
    permutation, and the 2D Laplacian 64x64 (P = 4).  Per (input, order, b):
    nnz(A~)/nnz(A) averaged over the partitions (the paper's CV/memA), the
    block (message) count M summed over the partitions, and the plan time
    (H_i, Alg. 2, map and the gather of A~) averaged over the partitions."""
    import torch
    import synth
    inputs = []
    R = synth.workload("rmat18")["A"]
    inputs.append(("rmat18", "original", R, P))
    inputs.append(("rmat18", "random_symmetric_perm", synth.permute_symmetric(R, seed=11), P))
    L = synth.laplacian2d(64)
    inputs.append(("lap2d_64", "original", L, 4))
    inputs.append(("lap2d_64", "random_symmetric_perm", synth.permute_symmetric(L, seed=11), 4))
    rows = []
    s = torch.cuda.current_stream()
    for name, order, M, parts in inputs:
        Ad = spg.DeviceCsc.from_host(M)
        offs = synth.partition_offsets(M.ncols, parts)
        Bis = [spg.DeviceCsc.from_host(synth.column_slice(M, int(offs[i]), int(offs[i + 1])))
               for i in range(parts)]
        for b in blocks:
            cv, msgs, ms = [], 0, []
            for Bi in Bis:
                def plan():
                    return spg.Plan(Ad, Bi, offs, b)
                with plan() as p:
                    st = p.stats()
                cv.append(st["nnz_At"] / max(1, M.nnz))
                msgs += st["M"]
                t = _time_on(s, lambda: plan().close(), reps)
                ms.append(t)
            rows.append({"input": name, "order": order, "P": parts, "b": b,
                         "cv_memA_mean": round(sum(cv) / len(cv), 4),
                         "messages_M": int(msgs), "plan_ms_mean": round(sum(ms) / len(ms), 4)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def study_bfs(spg, levels_max=32):
    """Forward search of batched betweenness centrality: 4096 sources on an
    unweighted R-MAT scale-16 graph; every level is one product N = A * F
    (plan + symbolic + numeric, timed with events on the launch stream), the
    next frontier keeps the vertices a source has not reached (a selection
    done here with torch on the device; it is not part of the timed work)."""
    import torch

    import synth

    w = synth.workload("bfs_rmat16_4096")
    A, F = w["A"], w["B"]
    n, ns = A.nrows, F.ncols
    dev = "cuda"
    Ad = spg.DeviceCsc.from_host(A, device=dev)
    Fd = spg.DeviceCsc.from_host(F, device=dev)
    visited = torch.zeros(n * ns, dtype=torch.bool, device=dev)
    cols0 = torch.repeat_interleave(torch.arange(ns, device=dev), Fd.colptr.diff())
    visited[cols0 * n + Fd.rowidx.long()] = True
    stream = torch.cuda.current_stream()
    rows_out, total_ms, total_flops = [], 0.0, 0
    for level in range(levels_max):
        if Fd.nnz == 0:
            break
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        with spg.Plan(Ad, Fd, None, w["b"]) as p:
            N = p.run()
            st = p.stats()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        total_ms += ms
        total_flops += st["flops"]
        rows_out.append({"level": level, "nnz_F": Fd.nnz, "flops": st["flops"],
                         "nnz_N": st["nnz_C"], "ms": round(ms, 4),
                         "GFLOPs": round(2 * st["flops"] / (ms * 1e-3) / 1e9, 2),
                         "num_bins": st["num_bins"]})
        cols = torch.repeat_interleave(torch.arange(ns, device=dev), N.colptr.diff())
        key = cols * n + N.rowidx.long()
        keep = ~visited[key]
        visited[key[keep]] = True
        colptr = torch.zeros(ns + 1, dtype=torch.int64, device=dev)
        colptr[1:] = torch.cumsum(torch.bincount(cols[keep], minlength=ns), 0)
        Fd = spg.DeviceCsc(n, ns, colptr, N.rowidx[keep].contiguous(), N.vals[keep].contiguous())
    return {"workload": "bfs_rmat16_4096 (R-MAT scale 16, ef 16, unit values, seed 3; "
                        "4096 sources, seed 7)",
            "levels": rows_out, "total_ms": round(total_ms, 3),
            "total_GFLOPs": round(2 * total_flops / (total_ms * 1e-3) / 1e9, 2)}


def study_outer(spg, parts=(4, 8, 16), reps=3):
    """The right product of a Galerkin step, X * P (P the 2x2x2 aggregation
    prolongator of the 64^3 7-point Laplacian A), by the two 1D forms on one
    GPU, over the same number of blocks p: column-wise (Alg. 1: C_i = X * P_i
    for P's column blocks, uploaded beforehand) and outer-product (Alg. 3:
    row blocks P(K_r, :), partial products X(:, K_r) * P(K_r, :), their sum).
    X = A is this project's order, X = P^T A the paper's.  Times are the
    whole local work of each form (plans included), averaged over reps."""
    import torch
    import synth

    A = spg.DeviceCsc.from_host(synth.laplacian3d(64))
    Ph = synth.aggregation3d(64)
    P = spg.DeviceCsc.from_host(Ph)
    Pt = spg.DeviceCsc.from_host(synth.aggregation3d_t(64))
    X_paper = spg.spgemm(Pt, A, None, 64)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    rows = []
    for name, X in (("A*P", A), ("(P^T A)*P", X_paper)):
        for p in parts:
            offs = synth.partition_offsets(X.ncols, p)
            coffs = synth.partition_offsets(Ph.ncols, p)
            blocks = [spg.DeviceCsc.from_host(synth.column_slice(Ph, int(coffs[i]), int(coffs[i + 1])))
                      for i in range(p)]
            cw_ms, cw = timed(lambda: [spg.spgemm(X, Bi, offs, 64) for Bi in blocks])
            op_ms, C = timed(lambda: spg.outer_product(X, P, offs, 64))
            # volumes (untimed): entries of X each form's products take into
            # A~, and the partial results the outer-product form's merge moves
            cw_At = 0
            for Bi in blocks:
                with spg.Plan(X, Bi, offs, 64) as q:
                    cw_At += q.stats()["nnz_At"]
            op_At, partial = 0, 0
            for r in range(p):
                with spg.Plan(X, spg.row_block(P, int(offs[r]), int(offs[r + 1])), offs, 64) as q:
                    op_At += q.stats()["nnz_At"]
                    partial += q.run().nnz
            rows.append({"product": name, "p": p, "nnz_X": X.nnz, "nnz_C": C.nnz,
                         "column_wise_At_entries": cw_At, "outer_At_entries": op_At,
                         "partial_nnz": partial,
                         "column_wise_ms": round(cw_ms, 4), "outer_product_ms": round(op_ms, 4),
                         "outer_over_column_wise": round(op_ms / cw_ms, 3)})
    return rows


def step_timer(spg, w, tun=None):
    """Uploads a workload and returns (run_step, plan_stats): run_step(record)
    runs one whole step (plan, symbolic, numeric, release) on the current
    stream; with record=True it returns HIP events at the phase borders."""
    import torch
    tdt = torch.float64 if w["dtype"] == "f64" else torch.float32
    Ad = spg.DeviceCsc.from_host(w["A"], dtype=tdt)
    Bd = spg.DeviceCsc.from_host(w["Bi"], dtype=tdt)
    stream = torch.cuda.current_stream()

    def run_step(record=False):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            ev[0].record(stream)
        p = spg.Plan(Ad, Bd, w["offs"], w["b"], tuning=tun)
        if record:
            ev[1].record(stream)
        p.symbolic()
        if record:
            ev[2].record(stream)
        p.numeric()
        if record:
            ev[3].record(stream)
        p.close()
        return ev

    with spg.Plan(Ad, Bd, w["offs"], w["b"], tuning=tun) as p:
        p.symbolic()
        rows, vals = p.numeric()
        st = p.stats()
    return run_step, st, (Ad, Bd)


def timed_steps(run_step, steps, flush=None):
    """Wall-clock ms of `steps` single steps, each bracketed by device
    synchronisations; with `flush` (a device tensor larger than the
    last-level cache) every step starts after that tensor is rewritten."""
    import torch
    out = []
    for r in range(steps):
        if flush is not None:
            flush.fill_(float(r))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_step()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return out


def side_workloads(spg, names, steps=10):
    """Warm and cache-flushed step times of the other configurations."""
    import torch
    flush = torch.empty(512 << 20 >> 3, dtype=torch.float64, device="cuda")
    res = {}
    for name in names:
        w = workload(name)
        run_step, st, keep = step_timer(spg, w)
        vs = 8 if w["dtype"] == "f64" else 4
        for _ in range(2):
            run_step()
        warm = timed_steps(run_step, steps)
        cold = timed_steps(run_step, steps, flush)
        mw, mc = float(np.median(warm)), float(np.median(cold))
        byt = phase_bytes(st, vs)
        res[w["desc"]] = {
            "flops": st["flops"], "nnz_C": st["nnz_C"], "dtype": w["dtype"],
            "ms_per_step_warm": round(mw, 4), "ms_per_step_flushed": round(mc, 4),
            "GFLOPs_warm": round(2 * st["flops"] / (mw * 1e-3) / 1e9, 3),
            "GFLOPs_flushed": round(2 * st["flops"] / (mc * 1e-3) / 1e9, 3),
            "algorithmic_bytes_per_step": int(sum(byt.values())),
            "step_GBs_flushed": round(sum(byt.values()) / (mc * 1e-3) / 1e9, 1)}
        print(json.dumps({name: res[w["desc"]]}), file=sys.stderr, flush=True)
        del keep, run_step
        torch.cuda.synchronize()
    del flush
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat18")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and backward measurements")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the other configurations' warm/flushed step times")
    ap.add_argument("--study", choices=["gather-volume", "bfs", "outer"],
                    help="instead of the benchmark, run a study and print its table as JSON")
    ap.add_argument("--tune", action="append", default=[], metavar="FIELD=VALUE",
                    help="override a spgemm_tuning field for the main workload (repeatable)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes, 5 times "
                         "(reference for HBM byte counters), and print its bandwidth")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library computes one partition's local "
              "product on one device and has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_ref:
        src = torch.empty(args.copy_ref // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        dst.copy_(src)
        ev[0].record()
        for _ in range(5):
            dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 5
        print(json.dumps({"copy_ref_bytes": src.numel() * 8, "ms": ms,
                          "GBps_read_plus_write": 2 * src.numel() * 8 / (ms * 1e-3) / 1e9}))
        return

    import paper_2408_14558_amd as spg

    if args.study == "gather-volume":
        print(json.dumps({"study": "gather_volume_vs_block_size_and_order",
                          "rows": study_gather_volume(spg)}), flush=True)
        return
    if args.study == "outer":
        print(json.dumps({"study": "galerkin_right_product_column_wise_vs_outer_product",
                          "rows": study_outer(spg)}), flush=True)
        return
    if args.study == "bfs":
        print(json.dumps({"study": "multi_source_bfs_forward_search", **study_bfs(spg)}),
              flush=True)
        return

    w = workload(args.workload)
    vsize = 8 if w["dtype"] == "f64" else 4
    stream = torch.cuda.current_stream()
    tun = spg.tuning(**{k: int(v) for k, v in (t.split("=", 1) for t in args.tune)}) \
        if args.tune else None
    run_step, st, keep = step_timer(spg, w, tun)
    print(f"workload {w['desc']}: flops {st['flops']} nnz_C {st['nnz_C']}", file=sys.stderr,
          flush=True)

    for _ in range(args.warmup):
        run_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # phase times inside steps (extra steps, outside the timed region)
    evs = [run_step(record=True) for _ in range(min(args.steps, 5))]
    torch.cuda.synchronize()
    ph = {name: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
          for i, name in enumerate(("plan", "symbolic", "numeric"))}

    # the numeric phase alone (the step's dominant kernels): back-to-back
    # launches on one plan between two HIP events on the launch stream
    Ad, Bd = keep
    reps = 10 if st["flops"] > 10 ** 8 else 50
    with spg.Plan(Ad, Bd, w["offs"], w["b"], tuning=tun) as p:
        p.symbolic()
        rows, vals = p.numeric()
        loop_ms = _time_on(stream, lambda: p.numeric(out=(rows, vals)), reps)
    del rows, vals
    flops = st["flops"]
    value = 2.0 * flops / (ms_per_step * 1e-3) / 1e9
    byt = phase_bytes(st, vsize)
    step_bytes = sum(byt.values())
    achieved = byt["numeric"] / (loop_ms * 1e-3) / 1e9
    traffic, trec = measured_traffic(w["desc"])
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["dtype"],
        "data": "synthetic",
        "config": {"workload": w["desc"], **w["config"],
                   **({"tuning": dict(t.split("=", 1) for t in args.tune)} if args.tune else {})},
        "roofline": {
            "bound": "hbm",
            "kernel": "numeric phase (the k_num_* launches of one spgemm_numeric)",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_note": trec if traffic is None else "rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                            "profiles/numeric_phase_hbm_traffic.md",
            "algorithmic_bytes": int(byt["numeric"]),
            "avg_ms": round(loop_ms, 5),
            "avg_ms_in_step": round(ph["numeric"], 5),
        },
        "roofline_step": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "algorithmic_bytes": {k: int(v) for k, v in byt.items()},
            "achieved": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 2),
            "frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "phase_ms": {k: round(v, 4) for k, v in ph.items()},
            "phase_frac": {k: round(byt[k] / (ph[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                           for k in ph},
            "GFLOPs_symbolic_plus_numeric": round(
                2 * flops / ((ph["symbolic"] + ph["numeric"]) * 1e-3) / 1e9, 2),
            # upper reference: every product's row id (symbolic) or row id and
            # value (numeric) read once, as a Gustavson walk streams them
            "gustavson_stream_bytes": {"symbolic": 4 * flops, "numeric": (4 + vsize) * flops},
            "gustavson_stream_GBs": {
                "symbolic": round(4 * flops / (ph["symbolic"] * 1e-3) / 1e9, 2),
                "numeric": round((4 + vsize) * flops / (loop_ms * 1e-3) / 1e9, 2)},
        },
        "sizes": {"flops": flops, "nnz_C": st["nnz_C"], "nnz_At": st["nnz_At"], "kt": st["kt"],
                  "M": st["M"], "K": st["K"], "cv_memA": round(st["cv_memA"], 4),
                  "sym_bins": st["sym_bins"], "num_bins": st["num_bins"]},
    }
    del keep, run_step, Ad, Bd
    torch.cuda.synchronize()
    if not args.no_side:
        names = [n for n in ("rmat18-f32", "er65536", "lap2d", "sketch") if n != args.workload]
        out["workloads"] = side_workloads(spg, names)
    if not args.no_forms:
        out["batched"] = bench_batched(spg)
        out["backward"] = bench_backward(spg)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
