"""The allocation-free pack (bsdmrg_pack_desc_noalloc, for callers that cannot
allocate device memory) against bsdmrg_pack_desc: byte-identical streams on two
calls in a row, the second with a smaller input (the scratch array keeps the
first call's tables), and a clear error beyond the scratch size."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _families(rng, nfam, maxb, maxdim, device):
    import torch
    fams = []
    for k in range(nfam):
        nb = int(rng.integers(1, maxb + 1))
        rows = rng.integers(0, maxdim + 1, nb).astype(np.int32)
        cols = rng.integers(1, maxdim + 1, nb).astype(np.int32)
        ld = (cols + rng.integers(0, 3, nb)).astype(np.int32)
        off = np.concatenate([[0], np.cumsum(rows.astype(np.int64) * ld)])[:-1].astype(np.int64)
        stride = int(np.sum(rows.astype(np.int64) * ld)) + 2
        stride += stride % 2
        nl = int(rng.integers(1, 4))
        data = torch.from_numpy(rng.normal(size=max(1, nl * stride))).to(device)
        fams.append({"tag": 100 + k, "dq": (int(rng.integers(-1, 2)), int(rng.integers(-1, 2))), "n_layers": nl,
                     "block_q": [[i, k] for i in range(nb)], "rows": rows, "cols": cols, "ld": ld,
                     "elem_offset": off, "layer_stride": stride, "data": data})
    return fams


def test_noalloc_pack_matches_allocating_pack():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    fn = B._lib.bsdmrg_pack_desc_noalloc
    rng = np.random.default_rng(7)
    for case, (nfam, maxb, maxdim) in enumerate(((24, 40, 70), (5, 6, 20))):
        say(f"no-alloc pack call {case}: {nfam} families")
        fams = _families(rng, nfam, maxb, maxdim, "cuda")
        n = B.bsdmrg_serialized_size_desc(fams)
        a = torch.full((n // 8 + 64,), -1.0, dtype=torch.float64, device="cuda")
        b = torch.full((n // 8 + 64,), -2.0, dtype=torch.float64, device="cuda")
        B.bsdmrg_pack_desc(fams, a, a.numel() * 8)
        arr, keep = B.make_family_descs(fams)
        rc = fn(len(fams), ctypes.cast(arr, ctypes.c_void_p), b.data_ptr(), b.numel() * 8,
                torch.cuda.current_stream().cuda_stream)
        assert rc == 0, B.bsdmrg_last_error()
        torch.cuda.synchronize()
        # bitwise: the tables hold integers whose bit patterns may be NaNs as float64
        assert torch.equal(a[: n // 8].view(torch.int64), b[: n // 8].view(torch.int64))
        assert torch.all(b[n // 8:] == -2.0)   # nothing past the stream is written
    # tables beyond the scratch size: rejected before any launch
    big = _families(rng, 1, 1, 1, "cuda")[0]
    nb = 600000
    big.update({"block_q": [[i, 0] for i in range(nb)], "rows": np.ones(nb, np.int32),
                "cols": np.ones(nb, np.int32), "ld": np.ones(nb, np.int32),
                "elem_offset": np.arange(nb, dtype=np.int64), "layer_stride": nb, "n_layers": 1,
                "data": torch.zeros(nb, dtype=torch.float64, device="cuda")})
    n = B.bsdmrg_serialized_size_desc([big])
    dst = torch.empty(n // 8 + 64, dtype=torch.float64, device="cuda")
    arr, keep = B.make_family_descs([big])
    rc = fn(1, ctypes.cast(arr, ctypes.c_void_p), dst.data_ptr(), dst.numel() * 8,
            torch.cuda.current_stream().cuda_stream)
    assert rc == B.EINVAL
    assert "scratch" in B.bsdmrg_last_error()
