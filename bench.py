#!/usr/bin/env python3
"""Benchmark of the local SpGEMM hot path on one MI355X.

A step is one pass of the whole path for one partition: spgemm_plan (H_i,
Alg. 2 block selection, column map, gather of A~), spgemm_symbolic (flops,
binning, nnz count, scan) and spgemm_numeric, with inputs resident in HBM.

Default workload (N=1): C_0 = A * B_0 for one of 16 column blocks, A and B
independent 65536 x 65536 Erdos-Renyi matrices with 16 entries per column,
U(-1,1) FP64 values, block size b = 256.  Other workloads are selectable with
--workload for reporting, the JSON line always names the one it ran.

Prints ONE JSON line.  value = 2 * sparse flops / step time (GFLOP/s).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s + achieved HBM GB/s (% peak); batched/backward vs plain speedup"
HBM_PEAK_GBS = 8000.0


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
        return dict(A=w["A"], Bi=w["A"], offs=w["offsets"], b=256,
                    dtype="f32" if name.endswith("f32") else "f64",
                    desc=f"rmat18_ef16_AxA_{'f32' if name.endswith('f32') else 'f64'}",
                    config={"A": "R-MAT scale 18, ef 16, (0.57,0.19,0.19,0.05), seed 3",
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


def cpu_baseline(w, budget_s=12.0):
    """The oracle as it stands (single-threaded FP64 C) on the host cores:
    the whole local step (H_i, Alg. 2, A~, flops, C_i) over consecutive
    blocks of at most 4096 columns of B_i, cycling, until about budget_s
    seconds have run."""
    import oracle
    import synth
    A, Bi = w["A"], w["Bi"]
    if w["dtype"] == "f32":
        A, Bi = synth.as_fp32(A), synth.as_fp32(Bi)
    chunk = min(Bi.ncols, 4096)
    starts = list(range(0, Bi.ncols, chunk))
    flops = 0
    cols = 0
    t0 = time.perf_counter()
    i = 0
    while True:
        c0 = starts[i % len(starts)]
        blk = synth.column_slice(Bi, c0, min(Bi.ncols, c0 + chunk))
        loc = oracle.local_product(A, blk, w["offs"], w["b"])
        flops += int(loc.flop.sum())
        cols += blk.ncols
        i += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el * (i + 1) / i > 30.0:
            break
    return {"value": 2.0 * flops / el / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{i} blocks of <= {chunk} columns of B_i ({cols} columns, {flops} "
                      f"flops) through the whole local step, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="er65536")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes, 5 times "
                         "(reference for HBM byte counters), and print its bandwidth")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharded design is described in DESIGN.md); use --gpus 1", file=sys.stderr)
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

    w = workload(args.workload)
    tdt = torch.float64 if w["dtype"] == "f64" else torch.float32
    vsize = 8 if w["dtype"] == "f64" else 4
    dev = "cuda"
    Ad = spg.DeviceCsc.from_host(w["A"], dtype=tdt, device=dev)
    Bd = spg.DeviceCsc.from_host(w["Bi"], dtype=tdt, device=dev)
    stream = torch.cuda.current_stream()

    ev = []  # (numeric start, numeric end) per timed step

    def step(record):
        p = spg.Plan(Ad, Bd, w["offs"], w["b"])
        p.symbolic()
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        rows, vals = p.numeric()
        if record:
            e1.record(stream)
            ev.append((e0, e1))
        p.close()
        return rows, vals

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    num_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)

    # sizes of the workload (from the library's own statistics)
    with spg.Plan(Ad, Bd, w["offs"], w["b"]) as p:
        p.symbolic()
        p.numeric()
        st = p.stats()
    flops = st["flops"]
    value = 2.0 * flops / (ms_per_step * 1e-3) / 1e9
    num_bytes = (4 + vsize) * (st["nnz_B"] + st["nnz_At"] + st["nnz_C"]) + 8 * (st["n"] + 1)
    achieved = num_bytes / (num_ms * 1e-3) / 1e9
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
        "config": {"workload": w["desc"], **w["config"]},
        "roofline": {
            "bound": "hbm",
            "kernel": "numeric phase (spgemm_numeric)",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes": int(num_bytes),
            "avg_ms": round(num_ms, 5),
        },
        "sizes": {"flops": flops, "nnz_C": st["nnz_C"], "nnz_At": st["nnz_At"], "kt": st["kt"],
                  "M": st["M"], "K": st["K"], "cv_memA": round(st["cv_memA"], 4),
                  "num_bins": st["num_bins"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
