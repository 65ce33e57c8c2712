"""GPU parity of the sampled backward pass and the autograd Function.

dA = (dC B^T) o pattern(A) and dB = (A^T dC) o pattern(B) against the FP64
oracle; exact finite differences (the loss <dC, A B> is bilinear);
torch.autograd.gradcheck in FP64 on the 512-size instance (dA is summed
with atomics, so repeated backward passes may differ in the last bits: the
check allows 1e-12); adjoint identities at full size.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import fp32_normwise

pytestmark = pytest.mark.gpu

spg = pytest.importorskip("paper_2408_14558_amd")


def _abs(M):
    return synth.CSC(M.nrows, M.ncols, M.colptr, M.rowidx, np.abs(np.asarray(M.vals, np.float64)))


def _setup(A, B, dtype):
    Ad = spg.DeviceCsc.from_host(A, dtype=dtype)
    Bd = spg.DeviceCsc.from_host(B, dtype=dtype)
    p = spg.Plan(Ad, Bd, None, 64)
    p.symbolic()
    rows, vals = p.numeric()
    return p, Ad, Bd, rows, vals


def test_backward_512_fp64_against_oracle():
    w = synth.workload("sketch_er512")
    A, B = w["A"], w["B"]
    p, Ad, Bd, rows, vals = _setup(A, B, torch.float64)
    C = oracle.spgemm(A, B)
    assert np.array_equal(rows.cpu().numpy(), C.rowidx)
    dC = synth.uniform_values(int(C.colptr[-1]), seed=7)
    dA, dB = p.backward(rows, torch.tensor(dC, device="cuda"))
    rA, rB = oracle.backward(A, B, C.colptr, C.rowidx, dC)
    bA, bB = oracle.backward(_abs(A), _abs(B), C.colptr, C.rowidx, np.abs(dC))
    assert np.all(np.abs(dA.cpu().numpy() - rA) <= 1e-12 * np.maximum(np.abs(rA), bA))
    assert np.all(np.abs(dB.cpu().numpy() - rB) <= 1e-12 * np.maximum(np.abs(rB), bB))
    # one side only
    dA2, dB2 = p.backward(rows, torch.tensor(dC, device="cuda"), need_dA=False)
    assert dA2 is None and np.array_equal(dB2.cpu().numpy(), dB.cpu().numpy())
    p.close()


def test_backward_finite_differences_are_exact():
    w = synth.workload("sketch_er512")
    A, B = w["A"], w["B"]
    p, Ad, Bd, rows, vals = _setup(A, B, torch.float64)
    dC = torch.tensor(synth.uniform_values(rows.numel(), seed=8), device="cuda")
    dA, dB = p.backward(rows, dC)
    rng = np.random.default_rng(3)
    h = 0.25
    for idx in rng.choice(A.nnz, 6, replace=False):
        ap = Ad.vals.clone()
        am = Ad.vals.clone()
        ap[idx] += h
        am[idx] -= h
        lp = torch.dot(p.numeric(ap, Bd.vals)[1], dC).item()
        lm = torch.dot(p.numeric(am, Bd.vals)[1], dC).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dA[idx].item()) <= 1e-11 * max(1.0, abs(fd))
    for idx in rng.choice(B.nnz, 6, replace=False):
        bp = Bd.vals.clone()
        bm = Bd.vals.clone()
        bp[idx] += h
        bm[idx] -= h
        lp = torch.dot(p.numeric(Ad.vals, bp)[1], dC).item()
        lm = torch.dot(p.numeric(Ad.vals, bm)[1], dC).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dB[idx].item()) <= 1e-11 * max(1.0, abs(fd))
    p.close()


def test_autograd_gradcheck_fp64_512():
    w = synth.workload("sketch_er512")
    A, B = w["A"], w["B"]
    Ad = spg.DeviceCsc.from_host(A)
    Bd = spg.DeviceCsc.from_host(B)
    p = spg.Plan(Ad, Bd, None, 64)
    p.symbolic()
    a = Ad.vals.clone().requires_grad_(True)
    b = Bd.vals.clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x, y: spg.SpGEMM.apply(x, y, p), (a, b),
                                    eps=1e-3, atol=1e-9, rtol=1e-7, fast_mode=True,
                                    nondet_tol=1e-12)
    # a plain backward through a scalar loss
    out = spg.SpGEMM.apply(a, b, p)
    g = torch.tensor(synth.uniform_values(out.numel(), seed=9), device="cuda")
    (out * g).sum().backward()
    C = oracle.spgemm(A, B)
    rA, rB = oracle.backward(A, B, C.colptr, C.rowidx, g.cpu().numpy())
    np.testing.assert_allclose(a.grad.cpu().numpy(), rA, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b.grad.cpu().numpy(), rB, rtol=1e-12, atol=1e-12)
    p.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_backward_full_size_sketch(dtype):
    """C = A*B with A the 131072^2 ER (8/col) and B the 131072x4096 sign
    sketch; dC uniform on pattern(C).  FP64 runs are checked per entry on a
    sample of columns' worth of entries and by the adjoint identities; FP32
    runs normwise against the FP64 oracle."""
    w = synth.workload("sketch_er131072")
    A, B = w["A"], w["B"]
    if dtype == torch.float32:
        A, B = synth.as_fp32(A), synth.as_fp32(B)
    p, Ad, Bd, rows, vals = _setup(A, B, dtype)
    C = oracle.spgemm(A, B)
    assert np.array_equal(rows.cpu().numpy(), C.rowidx)
    dC = synth.uniform_values(int(C.colptr[-1]), seed=7)
    if dtype == torch.float32:
        dC = dC.astype(np.float32)
    dA, dB = p.backward(rows, torch.tensor(dC, device="cuda"))
    rA, rB = oracle.backward(A, B, C.colptr, C.rowidx, dC)
    if dtype == torch.float64:
        bA, bB = oracle.backward(_abs(A), _abs(B), C.colptr, C.rowidx, np.abs(dC))
        assert np.all(np.abs(dA.cpu().numpy() - rA) <= 1e-12 * np.maximum(np.abs(rA), bA))
        assert np.all(np.abs(dB.cpu().numpy() - rB) <= 1e-12 * np.maximum(np.abs(rB), bB))
        ref = float(np.dot(dC, C.vals))
        assert abs(float(dA.double() @ Ad.vals.double()) - ref) <= 1e-10 * abs(ref)
        assert abs(float(dB.double() @ Bd.vals.double()) - ref) <= 1e-10 * abs(ref)
    else:
        assert fp32_normwise(dA.cpu().numpy(), rA) <= 1e-5
        assert fp32_normwise(dB.cpu().numpy(), rB) <= 1e-5
        assert fp32_normwise(vals.cpu().numpy(), C.vals) <= 1e-5
    p.close()
