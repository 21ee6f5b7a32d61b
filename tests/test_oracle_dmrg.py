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


def _psi_from_spectrum(dl, dr, spectrum, seed):
    """Two-site wave function built sector by sector as U diag(sigma) V^T.

    spectrum maps a middle sector q_m to its singular values.  Rows of the
    sector matrix are the (s1, q_l = q_m - q_s1) pairs present in dl, columns
    the (s2, q_r = q_m + q_s2) pairs present in dr, both in s order; U and V
    are random orthonormal columns, so the sector's singular values are exactly
    the given ones (up to rounding)."""
    from synthetic.mps import QS
    rng = np.random.default_rng(seed)
    psi = {}
    for qm, sig in spectrum.items():
        rows = [(s1, (qm[0] - QS[s1][0], qm[1] - QS[s1][1])) for s1 in range(4)]
        rows = [(s1, q) for s1, q in rows if q in dl]
        cols = [(s2, (qm[0] + QS[s2][0], qm[1] + QS[s2][1])) for s2 in range(4)]
        cols = [(s2, q) for s2, q in cols if q in dr]
        nr = sum(dl[q] for _, q in rows)
        nc = sum(dr[q] for _, q in cols)
        k = len(sig)
        assert k <= min(nr, nc)
        U = np.linalg.qr(rng.normal(size=(nr, k)))[0]
        V = np.linalg.qr(rng.normal(size=(nc, k)))[0]
        M = (U * np.asarray(sig, dtype=float)) @ V.T
        r0 = 0
        for s1, ql in rows:
            c0 = 0
            for s2, qr in cols:
                psi[(ql, s1, s2)] = M[r0:r0 + dl[ql], c0:c0 + dr[qr]].copy()
                c0 += dr[qr]
            r0 += dl[ql]
    return psi


# bonds of a two-site position in the (n_alpha, n_beta) = (1, 1) sector of a
# 2-electron problem: middle sectors (1,0), (0,1), (1,1) and (0,0) all occur
_DL = {(0, 0): 3, (1, 0): 3, (0, 1): 3}
_DR = {(1, 1): 3, (1, 0): 3, (0, 1): 3, (0, 0): 2}


def _kept_sigmas(svd, keep):
    return sorted((float(x) for qm, k in keep.items() for x in svd[qm][5][:k]), reverse=True)


def test_split_distinct_values_keep_exactly_D():
    """Distinct singular values spread over three sectors: exactly the D largest
    are kept and the error is the sum of the squares of the others."""
    spectrum = {(1, 0): [0.70, 0.31, 0.05], (0, 1): [0.52, 0.21, 0.02], (1, 1): [0.40, 0.11]}
    allsig = sorted((x for v in spectrum.values() for x in v), reverse=True)
    psi = _psi_from_spectrum(_DL, _DR, spectrum, 1)
    for D in (1, 2, 3, 5, 7):
        svd, keep, err = split(psi, _DL, _DR, D)
        got = sorted((float(x) for v in svd.values() for x in v[5] if x > 1e-12), reverse=True)
        assert np.allclose(got, allsig, rtol=0, atol=1e-13)
        assert sum(keep.values()) == D
        assert np.allclose(_kept_sigmas(svd, keep), allsig[:D], rtol=0, atol=1e-13)
        assert abs(err - sum(x * x for x in allsig[D:])) < 1e-13
    # more room than states: everything above the floor stays
    svd, keep, err = split(psi, _DL, _DR, 100)
    assert sum(keep.values()) == len(allsig)
    assert err < 1e-24


def test_split_keeps_degenerate_pair_across_sectors():
    """An exactly degenerate pair straddling position D, one partner in each of
    two sectors (the spin-flip pair of an S_z = 0 state): both are kept."""
    spectrum = {(1, 0): [0.70, 0.30, 0.05], (0, 1): [0.50, 0.30, 0.02]}
    psi = _psi_from_spectrum(_DL, _DR, spectrum, 2)
    svd, keep, err = split(psi, _DL, _DR, 3)     # 0.70, 0.50, then the 0.30 pair
    assert keep == {(1, 0): 2, (0, 1): 2}
    assert abs(err - (0.05 ** 2 + 0.02 ** 2)) < 1e-13
    # a pair split by more than the 1e-10 relative tolerance is not extended
    spectrum = {(1, 0): [0.70, 0.30, 0.05], (0, 1): [0.50, 0.30 * (1 - 1e-8), 0.02]}
    psi = _psi_from_spectrum(_DL, _DR, spectrum, 2)
    svd, keep, err = split(psi, _DL, _DR, 3)
    assert keep == {(1, 0): 2, (0, 1): 1}


def test_split_drops_values_below_floor():
    """Values at or below 1e-6 sigma_max are dropped even when fewer than D
    states exist, and a sector left with nothing disappears from the kept set;
    a value just above the floor stays."""
    spectrum = {(1, 0): [0.9, 8e-7], (0, 1): [0.4, 0.0], (1, 1): [1e-17]}
    psi = _psi_from_spectrum(_DL, _DR, spectrum, 3)
    svd, keep, err = split(psi, _DL, _DR, 64)
    assert keep == {(1, 0): 1, (0, 1): 1}
    assert abs(err - 8e-7 ** 2) < 1e-20      # sigma to ~1e-16 absolute
    spectrum = {(1, 0): [0.9, 1e-6], (0, 1): [0.4, 0.0], (1, 1): [2e-6]}
    psi = _psi_from_spectrum(_DL, _DR, spectrum, 3)
    svd, keep, err = split(psi, _DL, _DR, 64)
    assert keep == {(1, 0): 2, (0, 1): 1, (1, 1): 1}
    assert err < 1e-24


@pytest.mark.parametrize("direction,D", [(1, 400), (-1, 400), (1, 6), (-1, 6)])
def test_start_vector_carries_the_state(direction, D):
    """The start vector of the next position represents the same Fock-space
    state as the split wave function projected on the kept states: without
    truncation P' nxt == P psi exactly; with truncation <P' nxt|P psi> equals
    |nxt|^2 = |psi|^2 - discarded weight (nxt is the orthogonal projection)."""
    from oracle.dense import DenseHeff
    from synthetic.mps import random_two_site_psi
    L, na, nb = 6, 3, 3
    h, eri = make_integrals(L)
    d = OracleDMRG(h, eri, na, nb, 400)
    # move the center to position 2 (left to right from 0), then split there
    guess = random_two_site_psi(d.dims[0], d.dims[2], 5)
    for i in range(2):
        _, guess = d.move(i, d._complete(guess, i), 400, +1)
    i = 2
    psi = random_two_site_psi(d.dims[i], d.dims[i + 2], 11)
    norm2 = sum(float(np.sum(b * b)) for b in psi.values())
    psi = {k: b / np.sqrt(norm2) for k, b in psi.items()}
    before = DenseHeff(None, build_h_interleaved(h, eri, na, nb)[0], L, d.T, i, (na, nb)).expand(psi)
    err, nxt = d.move(i, psi, D, direction)
    j = i + 1 if direction > 0 else i - 1
    dets = build_h_interleaved(h, eri, na, nb)[0]
    after = DenseHeff(None, dets, L, d.T, j, (na, nb)).expand(d._complete(nxt, j))
    n2 = sum(float(np.sum(b * b)) for b in nxt.values())
    if D >= 400:
        assert err < 1e-28
        assert np.linalg.norm(after - before) < 1e-12
    else:
        assert err > 1e-6
        assert abs(n2 - (1.0 - err)) < 1e-12
        assert abs(float(after @ before) - n2) < 1e-12
        assert np.linalg.norm(after) ** 2 == pytest.approx(n2, abs=1e-12)
