"""Streamed right operators under a device budget (the one-GPU form of the
environment that exceeds the accelerator memory, Sec. III.A strategy 2 and
Sec. IV): the product copies each chunk's right operators from pinned host
memory into a device slot on a side stream while the previous chunk computes.
It must equal the resident product bit for bit, keep working after the right
block's device memory is released, and give the same Davidson run."""
import numpy as np
import pytest

from gpu_helpers import build_system, psi_for, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,na,nb,D,site,chunk_kib", [(10, 5, 5, 60, 4, 64), (10, 7, 6, 60, 4, 16), (12, 6, 6, 100, 5, 256)])
def test_streamed_product_bit_identical(L, na, nb, D, site, chunk_kib):
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    say(f"streamed product L={L} ({na},{nb}) D={D} chunks of {chunk_kib} KiB")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    # resident product with the same chunks (the chunks fix the order of the
    # float64 additions across them)
    B.bsdmrg_set_hbm_budget(ctx, 0, chunk_kib * 1024)
    B.bsdmrg_hpsi_prepare(ctx, site)
    assert not B.bsdmrg_hpsi_streamed(ctx, site)[0]
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 6), lay)).cuda()
    ref = {}
    for prec in (B.FP64, B.BF16X3, B.BF16X6):
        y = torch.empty_like(x)
        B.bsdmrg_hpsi(ctx, site, x, y, prec)
        torch.cuda.synchronize()
        ref[prec] = y
    x0 = x.clone()
    e0, it0, r0, _ = B.bsdmrg_davidson(ctx, site, x0, max_iter=12, precond=1)
    # a budget below the two blocks: the product is prepared in streamed form
    B.bsdmrg_set_hbm_budget(ctx, 1, chunk_kib * 1024)
    B.bsdmrg_hpsi_prepare(ctx, site)
    streamed, host_bytes, nchunks = B.bsdmrg_hpsi_streamed(ctx, site)
    say(f"  streamed {streamed}, {host_bytes} pinned bytes per product in {nchunks} chunks")
    assert streamed and host_bytes > 0 and nchunks >= 2
    for prec in ref:
        y = torch.empty_like(x)
        B.bsdmrg_hpsi(ctx, site, x, y, prec)
        torch.cuda.synchronize()
        assert torch.equal(y, ref[prec]), prec
    # release the right block: the streamed product does not read it
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    n = B.bsdmrg_serialized_size(ctx, B.RIGHT, site + 2)
    st = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
    pin = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
    B.bsdmrg_offload(ctx, B.RIGHT, site + 2, st, pin, n, 1, comp, side)
    B.bsdmrg_offload_wait(ctx, B.RIGHT, site + 2)
    assert B.bsdmrg_block_bytes(ctx, B.RIGHT, site + 2) == 0
    # with a forced late copy the compute stream waits; the result is the same
    B.bsdmrg_set_side_delay(ctx, 20.0)
    for prec in ref:
        y = torch.empty_like(x)
        B.bsdmrg_hpsi(ctx, site, x, y, prec)
        torch.cuda.synchronize()
        assert torch.equal(y, ref[prec]), prec
    B.bsdmrg_set_side_delay(ctx, 0.0)
    x1 = x.clone()
    e1, it1, r1, _ = B.bsdmrg_davidson(ctx, site, x1, max_iter=12, precond=1)
    assert e1 == e0 and it1 == it0 and r1 == r0
    assert torch.equal(x1, x0)
    st_ = B.bsdmrg_stats(ctx)
    assert st_["bytes_h2d"] >= host_bytes * (len(ref) * 2 + it1)
    B.bsdmrg_destroy(ctx)
