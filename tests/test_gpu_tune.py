"""GPU test of the autotuner: it measures candidate tunings of a small
power-law product, caches the winner under the product's signature, and the
tuned product still matches the oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_values

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def test_tune_caches_and_keeps_the_product(tmp_path):
    A = synth.rmat(11, 8, 0.57, 0.19, 0.19, 0.05, seed=17)
    Ad = spg.DeviceCsc.from_host(A)
    cache = str(tmp_path / "tuning.json")
    t, rep = spg.tune.tune(Ad, Ad, None, 64, reps=1, sweeps=1, cache=cache)
    print("tuned", rep, flush=True)
    assert not rep["cached"] and rep["tried"] >= 1 and rep["ms"] <= rep["default_ms"]
    t2, rep2 = spg.tune.tune(Ad, Ad, None, 64, cache=cache)
    assert rep2["cached"] and rep2["fields"] == rep["fields"]
    ref = oracle.spgemm(A, A)
    with spg.Plan(Ad, Ad, None, 64, tuning=t2) as p:
        colptr = p.symbolic()
        rows, vals = p.numeric()
    assert np.array_equal(colptr.cpu().numpy(), ref.colptr)
    assert np.array_equal(rows.cpu().numpy(), ref.rowidx)
    assert_values(vals.cpu().numpy(), ref.vals, ref.absvals, True)


def test_tune_batch_picks_a_stream_count():
    plans, io = [], []
    for A, B in synth.er_batch(6, seed=8):
        p = spg.Plan(spg.DeviceCsc.from_host(A), spg.DeviceCsc.from_host(B), None, 64)
        C = p.run()
        plans.append(p)
        io.append({"C_rowidx": C.rowidx, "C_vals": C.vals})
    torch.cuda.synchronize()
    best, rep = spg.tune.tune_batch(plans, io, streams=(1, 4), reps=2)
    assert set(rep["ms"]) == {"grouped, streams=1", "grouped, streams=4",
                              "separate, streams=1", "separate, streams=4", "persistent"}
    assert rep["best"] in rep["ms"] and rep["ms"][rep["best"]] == min(
        t for t in rep["ms"].values() if t is not None)
    assert set(best) == {"batch_streams", "batch_form"}
    # spgemm_batched takes the batch fields from the first plan's tuning
    t = spg.tuning(**best)
    p0 = spg.Plan(plans[0].A, plans[0].Bi, None, 64, tuning=t)
    C0 = p0.run()
    tab = [{"C_rowidx": C0.rowidx, "C_vals": C0.vals}] + io[1:]
    before = [d["C_vals"].clone() for d in tab]
    for d in tab:
        d["C_vals"].zero_()
    spg.batched([p0] + plans[1:], tab, 0)
    torch.cuda.synchronize()
    for d, v in zip(tab, before):  # same products (LDS sums may round differently)
        tol = 1e-12 * max(float(v.abs().max()), 1.0) if v.numel() else 0.0
        assert torch.allclose(d["C_vals"], v, rtol=1e-12, atol=tol)
    p0.close()
    for p in plans:
        p.close()
