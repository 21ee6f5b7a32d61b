"""Pins of the oracle two-site DMRG: full-CI energies (exact bond dimension),
the variational bound under truncation, and sweep-energy behaviour."""
import numpy as np
import pytest

from synthetic import make_integrals
from oracle.dmrg import OracleDMRG, split
from oracle.fci import build_h_interleaved, ground_energy


def fci_energy(L, na, nb):
    h, eri = make_integrals(L)
    _, H = build_h_interleaved(h, eri, na, nb)
    return h, eri, ground_energy(H)


def test_exact_bond_dimension_reproduces_fci():
    h, eri, E = fci_energy(6, 3, 3)
    d = OracleDMRG(h, eri, 3, 3, 400)
    log = d.sweep(400)
    assert abs(log[-1][1] - E) < 1e-9
    assert all(e >= E - 1e-10 for _, e, _ in log)


def test_open_shell_fci():
    h, eri, E = fci_energy(6, 4, 2)
    d = OracleDMRG(h, eri, 4, 2, 400)
    d.sweep(400)
    log = d.sweep(400)
    assert abs(log[-1][1] - E) < 1e-9


def test_config0_sweeps_reach_fci():
    """L=8, N=8, S_z=0, D=64 (FCI dimension 4900)."""
    h, eri, E = fci_energy(8, 4, 4)
    d = OracleDMRG(h, eri, 4, 4, 64)
    d.sweep(64)
    log = d.sweep(64)
    assert abs(log[-1][1] - E) < 1e-9
    assert all(e >= E - 1e-10 for _, e, _ in log)


def test_truncated_sweeps_are_variational_and_settle():
    h, eri, E = fci_energy(6, 3, 3)
    d = OracleDMRG(h, eri, 3, 3, 8)
    sweeps = [d.sweep(4) for _ in range(3)]
    for log in sweeps:
        assert all(e >= E - 1e-10 for _, e, _ in log)
    es = [log[-1][1] for log in sweeps]
    tr = [sum(x[2] for x in log) for log in sweeps]
    for k in range(1, len(es)):
        assert es[k] <= es[k - 1] + max(1e-9, 10 * tr[k])


def test_split_keeps_degenerate_partners_and_exact_weight():
    rng = np.random.default_rng(0)
    dl = {(0, 0): 2, (1, 0): 2}
    dr = {(1, 0): 2, (2, 0): 2, (1, 1): 2, (2, 1): 2}
    psi = {((0, 0), 1, 0): rng.normal(size=(2, 2)), ((1, 0), 0, 0): rng.normal(size=(2, 2))}
    svd, keep, err = split(psi, dl, dr, 1)
    s_all = sorted(np.concatenate([v[5] for v in svd.values()]), reverse=True)
    total = sum(x * x for x in s_all)
    kept = sum(keep.values())
    assert kept >= 1
    assert abs(err - sum(x * x for x in s_all[kept:])) < 1e-14 * total
