"""Pins of the FCI Hamiltonian (Eq. 1 in the reading stated in oracle.fci)."""
import numpy as np
import pytest

from synthetic import make_integrals
from oracle.fci import build_h_interleaved, build_h_strings, ground_energy


@pytest.mark.parametrize("L,na,nb", [(3, 2, 1), (4, 2, 2), (5, 3, 2), (6, 3, 3)])
def test_two_constructions_agree(L, na, nb):
    h, eri = make_integrals(L)
    _, H1 = build_h_interleaved(h, eri, na, nb)
    _, H2 = build_h_strings(h, eri, na, nb)
    assert abs(H1 - H2).max() < 1e-12
    assert abs(H1 - H1.T).max() < 1e-13


def test_integrals_symmetry():
    h, eri = make_integrals(6)
    assert np.allclose(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.allclose(eri, np.transpose(eri, perm))
    w = np.linalg.eigvalsh(eri.reshape(36, 36))
    assert w.min() > -1e-10


def test_noninteracting_closed_form():
    L, na, nb = 5, 3, 2
    h, _ = make_integrals(L)
    eri = np.zeros((L,) * 4)
    _, H = build_h_interleaved(h, eri, na, nb)
    e = np.linalg.eigvalsh(h)
    assert abs(ground_energy(H) - (e[:na].sum() + e[:nb].sum())) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.7, 1.3)])
def test_hubbard_dimer(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    for build in (build_h_interleaved, build_h_strings):
        _, H = build(h, eri, 1, 1)
        assert abs(ground_energy(H) - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_single_orbital_double_occupancy():
    h = np.array([[-1.3]])
    eri = np.full((1, 1, 1, 1), 0.8)
    _, H = build_h_interleaved(h, eri, 1, 1)
    assert abs(ground_energy(H) - (2 * -1.3 + 0.8)) < 1e-14


def test_same_spin_pair_exchange_sign():
    # two alpha electrons in two orbitals: one determinant, energy
    # h11 + h22 + (11|22) - (12|21)
    h, eri = make_integrals(2)
    for build in (build_h_interleaved, build_h_strings):
        _, H = build(h, eri, 2, 0)
        e = h[0, 0] + h[1, 1] + eri[0, 0, 1, 1] - eri[0, 1, 1, 0]
        assert abs(H.toarray()[0, 0] - e) < 1e-13


def test_config0_sector_dimension():
    h, eri = make_integrals(8)
    dets, H = build_h_interleaved(h, eri, 4, 4)
    assert len(dets) == 4900
