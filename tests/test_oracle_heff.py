"""Pins of the effective-Hamiltonian oracles: the dense P^T H P against FCI,
and the block-sparse product (renormalized normal/complementary operators)
against the dense definition on every bond."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from synthetic import make_integrals
from synthetic.mps import random_mps, random_two_site_psi
from oracle.fci import build_h_interleaved, ground_energy
from oracle.dense import DenseHeff
from oracle.siteops import spin_orbital_integrals
from oracle.blocks import build_left_blocks, build_right_blocks
from oracle.hpsi import BlockSparseHeff

_CACHE = {}


def fci(L, na, nb):
    key = (L, na, nb)
    if key not in _CACHE:
        h, eri = make_integrals(L)
        dets, H = build_h_interleaved(h, eri, na, nb)
        _CACHE[key] = (h, eri, dets, H)
    return _CACHE[key]


def flat(d, keys):
    return np.concatenate([d[k].ravel() for k in keys])


def rel(a, b):
    keys = list(b)
    x, y = flat(a, keys), flat(b, keys)
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("L,na,nb,D", [(4, 2, 2, 16), (6, 3, 3, 20), (6, 4, 2, 16), (7, 4, 3, 24)])
def test_blocksparse_equals_dense_every_bond(L, na, nb, D):
    h, eri, dets, H = fci(L, na, nb)
    t, g = spin_orbital_integrals(h, eri)
    for i in range(L - 1):
        dims, T = random_mps(L, na, nb, D, i)
        psi = random_two_site_psi(dims[i], dims[i + 2], 11 + i)
        ref = DenseHeff(H, dets, L, T, i, (na, nb)).apply(psi)
        lb = build_left_blocks(T, i, t, g)[i]
        rb = build_right_blocks(T, i + 2, t, g, (na, nb))[i + 2]
        out = BlockSparseHeff(lb, rb, t, g, (na, nb)).apply(psi)
        assert rel(out, ref) < 1e-12


@pytest.mark.parametrize("i", [3, 5])
def test_blocksparse_equals_dense_config0(i):
    L, na, nb, D = 8, 4, 4, 64
    h, eri, dets, H = fci(L, na, nb)
    t, g = spin_orbital_integrals(h, eri)
    dims, T = random_mps(L, na, nb, D, i)
    psi = random_two_site_psi(dims[i], dims[i + 2], 5)
    ref = DenseHeff(H, dets, L, T, i, (na, nb)).apply(psi)
    lb = build_left_blocks(T, i, t, g)[i]
    rb = build_right_blocks(T, i + 2, t, g, (na, nb))[i + 2]
    out = BlockSparseHeff(lb, rb, t, g, (na, nb)).apply(psi)
    assert rel(out, ref) < 1e-12


def test_heff_full_bonds_reproduces_fci():
    """With complete bond bases P is orthogonal, so min eig(P^T H P) = E_FCI."""
    L, na, nb = 6, 3, 3
    h, eri, dets, H = fci(L, na, nb)
    t, g = spin_orbital_integrals(h, eri)
    i = 2
    dims, T = random_mps(L, na, nb, 10 ** 6, i)
    psi = random_two_site_psi(dims[i], dims[i + 2], 3)
    keys = list(psi)
    shapes = [psi[k].shape for k in keys]
    n = sum(a * b for a, b in shapes)
    assert n == len(dets)
    lb = build_left_blocks(T, i, t, g)[i]
    rb = build_right_blocks(T, i + 2, t, g, (na, nb))[i + 2]
    bs = BlockSparseHeff(lb, rb, t, g, (na, nb))

    def unflat(v):
        d, o = {}, 0
        for k, s in zip(keys, shapes):
            d[k] = v[o:o + s[0] * s[1]].reshape(s)
            o += s[0] * s[1]
        return d

    mv = lambda v: flat(bs.apply(unflat(v)), keys)
    A = sla.LinearOperator((n, n), matvec=mv, dtype=float)
    w = sla.eigsh(A, k=1, which="SA", tol=1e-13)[0][0]
    assert abs(w - ground_energy(H)) < 1e-10
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=n), rng.normal(size=n)
    assert abs(x @ mv(y) - y @ mv(x)) < 1e-11 * abs(x @ mv(y))


def test_heff_truncated_is_variational():
    L, na, nb = 6, 3, 3
    h, eri, dets, H = fci(L, na, nb)
    i = 2
    dims, T = random_mps(L, na, nb, 12, i)
    op = DenseHeff(H, dets, L, T, i, (na, nb))
    psi = random_two_site_psi(dims[i], dims[i + 2], 3)
    keys = list(psi)
    v = flat(psi, keys)
    e = v @ flat(op.apply(psi), keys) / (v @ v)
    assert e >= ground_energy(H) - 1e-12


@pytest.mark.parametrize("L,na,nb,i", [(6, 3, 3, 2), (6, 4, 2, 2), (5, 3, 2, 1)])
def test_dense_heff_full_bonds_reproduces_fci(L, na, nb, i):
    """The dense definition itself: with complete bond bases P is an orthogonal
    map onto the sector, so P^T H P has exactly the FCI spectrum; its lowest
    eigenvalue is E_FCI and it is symmetric."""
    h, eri, dets, H = fci(L, na, nb)
    dims, T = random_mps(L, na, nb, 10 ** 6, i)
    op = DenseHeff(H, dets, L, T, i, (na, nb))
    psi = random_two_site_psi(dims[i], dims[i + 2], 3)
    keys = list(psi)
    shapes = [psi[k].shape for k in keys]
    n = sum(a * b for a, b in shapes)
    assert n == len(dets)

    def unflat(v):
        d, o = {}, 0
        for k, s in zip(keys, shapes):
            d[k] = v[o:o + s[0] * s[1]].reshape(s)
            o += s[0] * s[1]
        return d

    M = np.column_stack([flat(op.apply(unflat(e)), keys) for e in np.eye(n)])
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    w = np.linalg.eigvalsh(0.5 * (M + M.T))
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    assert np.allclose(w, np.linalg.eigvalsh(Hd), rtol=0, atol=1e-10)
    assert abs(w[0] - ground_energy(H)) < 1e-10
