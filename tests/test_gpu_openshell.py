"""Parity in the regime of the large open-shell active space: more electrons
than orbitals and 2 S_z = 1 (as in N=113 on 76 orbitals, about 74 % filling).
The HIP product is compared with the dense definition P^T H P psi at every
two-site position, and with the block-sparse oracle when the right
environment is grown with normal operators and switched to the complementary
set at the product's right bond (the configuration the large benchmark uses).
Bars: relative 2-norm error <= 1e-10 in float64, <= 1e-6 for split-bf16 x6."""
import numpy as np
import pytest

from gpu_helpers import build_system, psi_for, rel, say
from oracle.blocks import build_left_blocks, build_right_blocks
from oracle.dense import DenseHeff
from oracle.fci import build_h_interleaved
from oracle.hpsi import BlockSparseHeff
from oracle.siteops import spin_orbital_integrals

pytestmark = pytest.mark.gpu
BARS = {0: 1e-10, 2: 1e-6}


def _products(ctx, site, psi):
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    out = {}
    for prec in BARS:
        y = torch.empty_like(x)
        B.bsdmrg_hpsi(ctx, site, x, y, prec)
        torch.cuda.synchronize()
        out[prec] = B.flat_to_psi(y.cpu().numpy(), lay)
    return out


@pytest.mark.parametrize("L,na,nb,D", [(8, 6, 5, 24), (10, 8, 7, 40)])
def test_open_shell_hpsi_matches_dense_every_site(L, na, nb, D):
    from paper_2412_04676_amd import bsdmrg as B
    H = dets = None
    for site in range(L - 1):
        say(f"open shell dense L={L} ({na},{nb}) D={D} site={site}")
        ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
        if H is None:
            dets, H = build_h_interleaved(h, eri, na, nb)
        psi = psi_for(dims, site, 300 + site)
        ref = DenseHeff(H, dets, L, T, site, (na, nb)).apply(psi)
        got = _products(ctx, site, psi)
        for prec, bar in BARS.items():
            e = rel(got[prec], ref)
            say(f"  precision {prec}: rel err {e:.3e}")
            assert e <= bar
        B.bsdmrg_destroy(ctx)


@pytest.mark.parametrize("L,na,nb,D,site", [(10, 8, 7, 60, 3), (12, 9, 8, 80, 4)])
def test_open_shell_hpsi_normal_right_matches_blocksparse_oracle(L, na, nb, D, site):
    from paper_2412_04676_amd import bsdmrg as B
    say(f"open shell block-sparse, normal right blocks: L={L} ({na},{nb}) D={D} site={site}")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site, normal_right=True)
    t, g = spin_orbital_integrals(h, eri)
    lb = build_left_blocks(T, site, t, g)[site]
    rb = build_right_blocks(T, site + 2, t, g, (na, nb))[site + 2]
    psi = psi_for(dims, site, 17)
    ref = BlockSparseHeff(lb, rb, t, g, (na, nb)).apply(psi)
    got = _products(ctx, site, psi)
    for prec, bar in BARS.items():
        e = rel(got[prec], ref)
        say(f"  precision {prec}: rel err {e:.3e}")
        assert e <= bar
    B.bsdmrg_destroy(ctx)
