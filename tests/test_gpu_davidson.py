"""Davidson on the GPU against the oracle's eigensolver (scipy Lanczos on the
block-sparse oracle product): energy, eigenvector overlap (eigenvectors are
unique up to sign), Cauchy-interlacing monotonicity of the Ritz values, and the
effective-Hamiltonian diagonal against the dense definition."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from gpu_helpers import build_system, psi_for, say
from oracle.blocks import build_left_blocks, build_right_blocks
from oracle.dense import DenseHeff
from oracle.fci import build_h_interleaved
from oracle.hpsi import BlockSparseHeff
from oracle.siteops import spin_orbital_integrals
from oracle.dmrg import flatten, unflatten

pytestmark = pytest.mark.gpu


def oracle_op(h, eri, T, L, na, nb, site):
    t, g = spin_orbital_integrals(h, eri)
    lb = build_left_blocks(T, site, t, g)[site]
    rb = build_right_blocks(T, site + 2, t, g, (na, nb))[site + 2]
    return BlockSparseHeff(lb, rb, t, g, (na, nb))


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("L,na,nb,D,site", [(8, 4, 4, 64, 3), (10, 5, 5, 100, 4), (9, 5, 4, 60, 2)])
def test_davidson_matches_oracle_lanczos(L, na, nb, D, site, precond):
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    say(f"davidson L={L} D={D} site={site}")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    op = oracle_op(h, eri, T, L, na, nb, site)
    psi0 = psi_for(dims, site, 5)
    keys = sorted(psi0)
    shapes = [psi0[k].shape for k in keys]
    n = sum(a * b for a, b in shapes)
    A = sla.LinearOperator((n, n), matvec=lambda v: flatten(op.apply(unflatten(v, keys, shapes)), keys), dtype=float)
    w, V = sla.eigsh(A, k=1, which="SA", tol=1e-13, v0=flatten(psi0, keys))
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi0, lay)).cuda()
    e, it, r, ritz = B.bsdmrg_davidson(ctx, site, x, tol=1e-9, max_iter=300, precond=precond)
    say(f"  E gpu {e:.12f} oracle {w[0]:.12f} iters {it} resid {r:.2e}")
    assert abs(e - w[0]) < 1e-9
    assert r <= 1e-9
    got = B.flat_to_psi(x.cpu().numpy(), lay)
    ov = abs(np.dot(flatten(got, keys), V[:, 0]))
    assert ov > 1 - 1e-10
    assert all(ritz[k + 1] <= ritz[k] + 1e-12 * abs(ritz[k]) for k in range(len(ritz) - 1))
    B.bsdmrg_destroy(ctx)


def test_heff_diagonal_matches_dense():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 6, 3, 3, 20, 2
    say("diagonal L=6")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    dets, H = build_h_interleaved(h, eri, na, nb)
    dense = DenseHeff(H, dets, L, T, site, (na, nb))
    lay = B.bsdmrg_psi_layout(ctx, site)
    meta, off, ne = lay
    d = torch.zeros(ne, dtype=torch.float64, device="cuda")
    B.bsdmrg_hpsi_diagonal(ctx, site, d)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    tmpl = B.flat_to_psi(np.zeros(ne), lay)
    ref = np.zeros(ne)
    for i in range(ne):
        e = np.zeros(ne)
        e[i] = 1.0
        ref[i] = B.psi_to_flat(dense.apply(B.flat_to_psi(e, lay)), lay)[i]
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    B.bsdmrg_destroy(ctx)


@pytest.mark.parametrize("precision", [1, 2])
def test_split_precision_davidson_reaches_float64_energy(precision):
    # split products down to their noise level, then float64 products: the
    # energy must match the oracle's Lanczos value as the float64 run does
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 100, 4
    say(f"split davidson precision {precision}")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    op = oracle_op(h, eri, T, L, na, nb, site)
    psi0 = psi_for(dims, site, 5)
    keys = sorted(psi0)
    shapes = [psi0[k].shape for k in keys]
    n = sum(a * b for a, b in shapes)
    A = sla.LinearOperator((n, n), matvec=lambda v: flatten(op.apply(unflatten(v, keys, shapes)), keys), dtype=float)
    w, V = sla.eigsh(A, k=1, which="SA", tol=1e-13, v0=flatten(psi0, keys))
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi0, lay)).cuda()
    e, it, r, ritz = B.bsdmrg_davidson(ctx, site, x, tol=1e-9, max_iter=300, precond=1, precision=precision)
    say(f"  E {e:.12f} oracle {w[0]:.12f} iters {it} resid {r:.2e}")
    assert abs(e - w[0]) < 1e-9
    assert r < 1e-9
    B.bsdmrg_destroy(ctx)
