"""Host checks of the seeded input generators: bond dimensions respect D,
exact sector counts and the isometry caps; generated tensors are left/right
isometries; two-site blocks are consistent with the bond labels."""
from math import comb

import numpy as np
import pytest

from synthetic import QS, bond_sector_dims, make_integrals
from synthetic.mps import random_mps, two_site_blocks, random_two_site_psi


@pytest.mark.parametrize("L,na,nb,D", [(8, 4, 4, 64), (24, 12, 12, 512), (12, 7, 5, 50)])
def test_bond_dims(L, na, nb, D):
    dims = bond_sector_dims(L, na, nb, D)
    assert dims[0] == {(0, 0): 1} and dims[L] == {(na, nb): 1}
    for n in range(L + 1):
        assert sum(dims[n].values()) <= D
        for (a, b), d in dims[n].items():
            assert d <= comb(n, a) * comb(n, b)
            assert d <= comb(L - n, na - a) * comb(L - n, nb - b)
            if n > 0:
                assert d <= sum(dims[n - 1].get((a - s[0], b - s[1]), 0) for s in QS)
            if n < L:
                assert d <= sum(dims[n + 1].get((a + s[0], b + s[1]), 0) for s in QS)


def test_tensors_are_isometries():
    L, na, nb, D, c = 10, 5, 5, 40, 4
    dims, T = random_mps(L, na, nb, D, c)
    for n in range(L):
        t = T[n]
        if t is None:
            continue
        if n < c:
            for qr, d in dims[n + 1].items():
                M = np.vstack([t[(qr[0] - QS[s][0], qr[1] - QS[s][1]), s] for s in range(4)
                               if ((qr[0] - QS[s][0], qr[1] - QS[s][1]), s) in t])
                assert np.allclose(M.T @ M, np.eye(d), atol=1e-12)
        else:
            for ql, d in dims[n].items():
                M = np.hstack([t[(ql, s)] for s in range(4) if (ql, s) in t])
                assert np.allclose(M @ M.T, np.eye(d), atol=1e-12)
    psi = random_two_site_psi(dims[c], dims[c + 2], 0)
    assert abs(sum(float(np.sum(b * b)) for b in psi.values()) - 1) < 1e-12
    for ql, s1, s2, qr in two_site_blocks(dims[c], dims[c + 2]):
        assert psi[(ql, s1, s2)].shape == (dims[c][ql], dims[c + 2][qr])


def test_integral_generator_is_seeded_and_shaped():
    h1, e1 = make_integrals(5)
    h2, e2 = make_integrals(5)
    assert np.array_equal(h1, h2) and np.array_equal(e1, e2)
    h3, _ = make_integrals(5, seed=1)
    assert not np.array_equal(h1, h3)
    assert e1.shape == (5,) * 4
    assert np.allclose(np.diag(h1) - np.diag((h1 + h1.T) / 2), 0)
