"""The autotuner's host logic (CPU): signatures, the JSON cache and the
coordinate search, with a synthetic cost in place of GPU timings."""

import torch

from paper_2408_14558_amd import tune


def _stats(sym, num, m=1000):
    return {"sym_bins": sym, "num_bins": num, "m": m}


def test_signature_buckets_counts_on_a_log_scale():
    a = tune.signature(_stats([0, 100, 3, 0, 0, 0, 5, 0], [0, 90, 0, 2, 0, 0, 5, 0]),
                       torch.float64, arch="gfx950")
    b = tune.signature(_stats([0, 120, 2, 0, 0, 0, 4, 0], [0, 100, 0, 3, 0, 0, 6, 0]),
                       torch.float64, arch="gfx950")
    c = tune.signature(_stats([0, 100, 3, 0, 0, 0, 5, 0], [0, 90, 0, 2, 0, 0, 5, 0]),
                       torch.float32, arch="gfx950")
    d = tune.signature(_stats([0, 1000, 3, 0, 0, 0, 5, 0], [0, 90, 0, 2, 0, 0, 5, 0]),
                       torch.float64, arch="gfx950")
    assert a == b            # same powers of two
    assert a != c and a != d  # dtype and a tenfold bin change matter
    assert a.startswith("gfx950|f64|m10|")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    data = tune.load_cache(path)
    assert data == {"version": tune.CACHE_VERSION, "entries": {}}
    data["entries"]["k"] = {"fields": {"tiny_max_flop": 128}, "ms": 1.0}
    tune.save_cache(data, path)
    assert tune.load_cache(path)["entries"]["k"]["fields"] == {"tiny_max_flop": 128}
    with open(path, "w") as f:
        f.write("not json")
    assert tune.load_cache(path)["entries"] == {}


def test_coordinate_search_finds_the_separable_minimum():
    target = {"tiny_max_flop": 128, "hash_max_nnz": 1024, "hash_max_flop": 2048,
              "medium_kernel": 2, "dense_window": 4096, "dense_first_flop": 1 << 18}
    calls = []

    def cost(f):
        calls.append(dict(f))
        return sum((f[k] != v) * (i + 1) for i, (k, v) in enumerate(target.items()))

    start = {"tiny_max_flop": 256, "hash_max_nnz": 2048, "hash_max_flop": 4096,
             "medium_kernel": 1, "dense_window": 0, "dense_first_flop": 1 << 18}
    best, t, log = tune.coordinate_search(cost, start)
    assert best == target and t == 0
    assert len(log) == len(calls)
    # one sweep finds it; the second confirms nothing changes, then stops
    per_sweep = sum(len(v) - 1 for v in tune.SEARCH_SPACE.values())
    assert len(calls) == 1 + 2 * per_sweep
