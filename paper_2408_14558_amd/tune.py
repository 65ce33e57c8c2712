"""Autotuner for the local SpGEMM's kernel choices (``spgemm_tuning``): the
bin thresholds that route output columns to the tiny, hash, bitmap or dense
kernels, the medium-bin kernel, and the batched form's stream count.  None
of these change the result, only which kernel computes a column.

A product is summarised by a signature: the device, the value dtype, the
row count and the symbolic phase's bin histogram (counts on a log2 scale).
The fastest tuning measured for a signature is kept in a JSON cache, so
later products with the same shape of work reuse it without measuring.
The cache lives at ``$SPGEMM_TUNING_CACHE`` or
``~/.cache/spgemm_mi355x/tuning.json``.

Measurements time symbolic + numeric of one plan with HIP events on a
private stream (the plan phase does not depend on these fields).
"""

from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

import torch

from . import _lib
from .api import Batch, DeviceCsc, Plan, default_tuning, tuning as make_tuning

# Values tried per field, in the order the coordinate search visits them.
SEARCH_SPACE: Dict[str, Tuple[int, ...]] = {
    "tiny_max_flop": (128, 256, 512),
    "hash_max_nnz": (512, 1024, 2048),
    "hash_max_flop": (1024, 2048, 4096),
    "medium_kernel": (1, 2),
    # the dense kernel's value window (0: as many slots as the LDS holds)
    # and the product count from which dense columns are handed out first
    "dense_window": (0, 8192, 4096),
    "dense_first_flop": (1 << 18, 1 << 16, 1 << 20, 0),
}

CACHE_VERSION = 1


def cache_path() -> str:
    return os.environ.get("SPGEMM_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "spgemm_mi355x", "tuning.json")


def _log2_bucket(x: int) -> int:
    return 0 if x <= 0 else int(math.log2(x)) + 1


def signature(stats: dict, dtype: torch.dtype, arch: Optional[str] = None) -> str:
    """Key of a product's shape of work, from a plan's stats after symbolic."""
    if arch is None:
        arch = _lib.load().spgemm_version().decode()
    sym = ",".join(str(_log2_bucket(c)) for c in stats["sym_bins"])
    num = ",".join(str(_log2_bucket(c)) for c in stats["num_bins"])
    dt = "f64" if dtype == torch.float64 else "f32"
    return f"{arch}|{dt}|m{_log2_bucket(stats['m'])}|sym[{sym}]|num[{num}]"


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {"version": CACHE_VERSION, "entries": {}}
    if data.get("version") != CACHE_VERSION or not isinstance(data.get("entries"), dict):
        return {"version": CACHE_VERSION, "entries": {}}
    return data


def save_cache(data: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuning_fields(t: _lib.Tuning) -> dict:
    return {name: getattr(t, name) for name in SEARCH_SPACE}


def coordinate_search(measure: Callable[[dict], float], start: dict,
                      space: Dict[str, Sequence[int]] = SEARCH_SPACE,
                      sweeps: int = 2) -> Tuple[dict, float, list]:
    """Minimises measure(fields) one field at a time (each field tries every
    value of its range with the others fixed), for up to `sweeps` passes or
    until a pass changes nothing.  Returns (best fields, best time, log)."""
    best = dict(start)
    best_t = measure(best)
    log = [(dict(best), best_t)]
    for _ in range(sweeps):
        changed = False
        for name, values in space.items():
            current = best.get(name)
            for v in values:
                if v == current:
                    continue
                cand = dict(best, **{name: v})
                t = measure(cand)
                log.append((cand, t))
                if t < best_t:
                    best, best_t, changed = cand, t, True
        if not changed:
            break
    return best, best_t, log


def measure_product(A: DeviceCsc, Bi: DeviceCsc, offsets, block_size: int, fields: dict,
                    reps: int = 3) -> float:
    """Average ms of symbolic + numeric for one tuning (one untimed run)."""
    s = torch.cuda.Stream()
    t = make_tuning(**fields)
    with torch.cuda.stream(s):
        with Plan(A, Bi, offsets, block_size, tuning=t, stream=s) as p:
            colptr = p.symbolic()
            rows, vals = p.numeric()
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                p.symbolic()
                p.numeric(out=(rows, vals))
            e1.record(s)
            s.synchronize()
            del colptr
    return e0.elapsed_time(e1) / reps


def tune(A: DeviceCsc, Bi: DeviceCsc, offsets=None, block_size: int = 256, reps: int = 3,
         space: Dict[str, Sequence[int]] = SEARCH_SPACE, sweeps: int = 2,
         cache: Optional[str] = None, use_cache: bool = True) -> Tuple[_lib.Tuning, dict]:
    """The fastest tuning for C_i = A * B_i; cached under the product's
    signature.  Returns (tuning, report)."""
    base = default_tuning()
    with Plan(A, Bi, offsets, block_size, tuning=base) as p:
        p.symbolic()
        key = signature(p.stats(), p.torch_dtype)
    data = load_cache(cache) if use_cache else {"version": CACHE_VERSION, "entries": {}}
    hit = data["entries"].get(key)
    if hit is not None:
        return make_tuning(**hit["fields"]), {"signature": key, "cached": True, **hit}
    best, best_t, log = coordinate_search(
        lambda f: measure_product(A, Bi, offsets, block_size, f, reps),
        tuning_fields(base), space, sweeps)
    default_t = log[0][1]
    entry = {"fields": best, "ms": round(best_t, 5), "default_ms": round(default_t, 5),
             "tried": len(log)}
    if use_cache:
        data["entries"][key] = entry
        save_cache(data, cache)
    return make_tuning(**best), {"signature": key, "cached": False, **entry}


def tune_batch(plans: Sequence[Plan], io: Sequence[dict],
               streams: Iterable[int] = (1, 2, 4, 8), persistent: bool = True,
               reps: int = 10) -> Tuple[dict, dict]:
    """The batched form with the fastest graph replay of a batch: the stream
    DAG with grouped launches, and with every product launched on its own,
    on each side-stream count, and (when the products allow it) one
    persistent launch.  Returns (the batch fields of spgemm_tuning, report);
    spgemm_batched takes them from the first plan's tuning."""
    s = torch.cuda.Stream()
    cands = [({"batch_streams": ns, "batch_form": f}, f"{'grouped' if f == 0 else 'separate'},"
              f" streams={ns}") for f in (0, 2) for ns in streams]
    if persistent:
        cands.append(({"batch_streams": 0, "batch_form": 1}, "persistent"))
    times = {}
    best = None
    for fields, name in cands:
        try:
            b = Batch(plans, io, make_tuning(**fields))
        except _lib.SpgemmError as e:
            if e.code != _lib.EUNSUPPORTED:
                raise
            times[name] = None  # this form does not take these products
            continue
        try:
            b.run(1, stream=s)
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                b.run(2, stream=s)
            e1.record(s)
            s.synchronize()
            b.check()
            times[name] = e0.elapsed_time(e1) / reps
        finally:
            b.close()
        if best is None or times[name] < times[best[1]]:
            best = (fields, name)
    return dict(best[0]), {"ms": times, "best": best[1]}
