"""Grouped block GEMM on the FP64 matrix cores against numpy (float64)."""
import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_block_gemm_shapes_and_transposes():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    rng = np.random.default_rng(0)
    shapes = [(1, 1, 1), (3, 5, 7), (16, 16, 4), (17, 33, 15), (32, 32, 32), (33, 31, 65),
              (64, 64, 64), (65, 130, 47), (150, 7, 200), (5, 150, 1), (200, 190, 130)]
    probs, refs, keep = [], [], []
    for (M, N, K) in shapes:
        for ta in (0, 1):
            for tb in (0, 1):
                A = rng.normal(size=(K, M) if ta else (M, K))
                Bm = rng.normal(size=(N, K) if tb else (K, N))
                C0 = rng.normal(size=(M, N + 3))
                alpha, beta = rng.normal(), (0.0 if (M + N) % 2 else rng.normal())
                ref = C0.copy()
                ref[:, :N] = alpha * ((A.T if ta else A) @ (Bm.T if tb else Bm)) + beta * C0[:, :N]
                tA, tB, tC = (torch.from_numpy(x).cuda() for x in (A, Bm, C0))
                keep += [tA, tB, tC]
                probs.append({"A": tA, "B": tB, "C": tC, "M": M, "N": N, "K": K, "lda": A.shape[1],
                              "ldb": Bm.shape[1], "ldc": N + 3, "transA": ta, "transB": tb,
                              "alpha": alpha, "beta": beta})
                refs.append(ref)
    say(f"block_gemm: {len(probs)} problems")
    B.bsdmrg_block_gemm(probs)
    torch.cuda.synchronize()
    for p, ref in zip(probs, refs):
        got = p["C"].cpu().numpy()
        err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
        assert err < 1e-13, (p["M"], p["N"], p["K"], p["transA"], p["transB"], err)


def test_block_gemm_empty_and_k0():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    C = torch.ones(4, 4, dtype=torch.float64, device="cuda")
    A = torch.ones(4, 1, dtype=torch.float64, device="cuda")
    B.bsdmrg_block_gemm([{"A": A, "B": A, "C": C, "M": 4, "N": 4, "K": 0, "lda": 1, "ldb": 4, "ldc": 4,
                          "alpha": 1.0, "beta": 2.0}])
    torch.cuda.synchronize()
    assert torch.all(C == 2.0)
    B.bsdmrg_block_gemm([])
    with pytest.raises(B.BsdmrgError):
        B.bsdmrg_block_gemm([{"A": A, "B": A, "C": C, "M": 4, "N": 4, "K": 2, "lda": 1, "ldb": 4, "ldc": 4}])


@pytest.mark.parametrize("precision,nparts", [(1, 2), (2, 3)])
def test_split_bf16_gemm_error_bound(precision, nparts):
    """Element-wise bound from the split: each operand keeps 8 nparts mantissa
    bits (dropped products <= 3 u^nparts |a||b| with u = 2^-8 per part after
    the leading one), plus float32 accumulation over at most 256 values of K
    between float64 flushes (<= 2^-24 (sqrt(256) + 2) |a||b| per flush)."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    rng = np.random.default_rng(1)
    shapes = [(7, 9, 5), (64, 64, 300), (100, 37, 1000), (33, 130, 64)]
    probs, data = [], []
    for (M, N, K) in shapes:
        A = rng.normal(size=(M, K)) * np.exp(rng.normal(size=(M, K)))
        Bm = rng.normal(size=(K, N))
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(Bm).cuda()
        tC = torch.zeros(M, N, dtype=torch.float64, device="cuda")
        probs.append({"A": tA, "B": tB, "C": tC, "M": M, "N": N, "K": K, "lda": K, "ldb": N, "ldc": N})
        data.append((A, Bm, tC))
    say(f"split bf16 x{3 if nparts == 2 else 6}")
    B.bsdmrg_block_gemm(probs, precision)
    torch.cuda.synchronize()
    worst = 0.0
    for A, Bm, tC in data:
        ref = A @ Bm
        absprod = np.abs(A) @ np.abs(Bm)
        u = 2.0 ** -8
        split = 3.0 * u ** nparts * 2.0 if nparts == 2 else 6.0 * u ** 3 * 2.0
        acc = 2.0 ** -24 * (np.sqrt(256) + 2) * (A.shape[1] / 256 + 1)
        bound = (split + acc) * absprod
        err = np.abs(tC.cpu().numpy() - ref)
        assert np.all(err <= bound), float((err / bound).max())
        worst = max(worst, float(np.linalg.norm(err) / np.linalg.norm(ref)))
    say(f"  worst relative 2-norm error {worst:.2e}")
