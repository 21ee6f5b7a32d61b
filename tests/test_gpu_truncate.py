"""Truncation of the two-site wave function on the GPU (density-matrix
eigenproblem per symmetry sector with the global keep rule) against the
oracle's per-sector SVD: kept count, kept singular values and discarded
weight, in both sweep directions."""
import numpy as np
import pytest

from gpu_helpers import build_system, psi_for, say
from oracle.dmrg import split

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,na,nb,D,site,Dkeep", [(10, 5, 5, 100, 4, 40), (12, 6, 6, 120, 5, 200),
                                                  (24, 12, 12, 512, 11, 512)])
@pytest.mark.parametrize("direction", [0, 1])
def test_truncation_matches_oracle_svd(L, na, nb, D, site, Dkeep, direction):
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    say(f"truncate L={L} D={D} site={site} keep={Dkeep} direction={direction}")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    psi = psi_for(dims, site, 11)
    svd, keep, err = split(psi, dims[site], dims[site + 2], Dkeep)
    ref = np.sort(np.concatenate([svd[q][5][:k] for q, k in keep.items()]))[::-1]
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    e_gpu, k_gpu, sv = B.bsdmrg_truncate(ctx, site, x, Dkeep, direction)
    sv = np.sort(sv)[::-1]
    say(f"  kept {k_gpu} (oracle {len(ref)}), err {e_gpu:.3e} (oracle {err:.3e})")
    assert k_gpu == len(ref)
    # singular values come from eigenvalues of psi psi^T: absolute accuracy in
    # sigma^2 is ~1e-16 sigma_max^2
    assert np.max(np.abs(sv - ref)) < 1e-7 * ref[0]
    assert abs(e_gpu - err) < 1e-12
    B.bsdmrg_destroy(ctx)
