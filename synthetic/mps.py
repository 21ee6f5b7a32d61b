"""Seeded synthetic MPS shapes and tensors under U(1)xU(1) symmetry.

Bond n sits between site n-1 and site n (bond 0 is the left vacuum, bond L
the right end).  A sector q = (n_alpha, n_beta) on bond n counts the electrons
on sites 0..n-1.  Sector dimensions follow a Gaussian model in (n_alpha,
n_beta) with hypergeometric variance, capped by the exact number of states on
either side, water-filled to a total of D, and then reduced until every site
tensor can be an isometry from either side.
"""

from math import comb

import numpy as np

QS = ((0, 0), (1, 0), (0, 1), (1, 1))


def mps_seed(L):
    return 2412 + L + 1


def psi_seed(L):
    return 2412 + L + 2


def _qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _qsub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def _exact_dims(L, na, nb, n):
    out = {}
    for a in range(0, min(n, na) + 1):
        for b in range(0, min(n, nb) + 1):
            ra, rb = na - a, nb - b
            if ra < 0 or rb < 0 or ra > L - n or rb > L - n:
                continue
            left = comb(n, a) * comb(n, b)
            right = comb(L - n, ra) * comb(L - n, rb)
            out[(a, b)] = min(left, right)
    return out


def _weights(L, na, nb, n, sectors):
    w = {}
    for q in sectors:
        e = 0.0
        for sig, ntot in ((0, na), (1, nb)):
            mu = n * ntot / L
            if L > 1:
                var = n * (L - n) / (L - 1) * (ntot / L) * (1 - ntot / L)
            else:
                var = 0.0
            var = max(var, 0.25)
            e += (q[sig] - mu) ** 2 / (2.0 * var)
        w[q] = np.exp(-e)
    return w


def bond_sector_dims(L, na, nb, D):
    """Return a list of L+1 dicts {q: dim} (bond 0 .. bond L)."""
    dims = []
    for n in range(L + 1):
        ex = _exact_dims(L, na, nb, n)
        if sum(ex.values()) <= D:
            dims.append(dict(ex))
            continue
        w = _weights(L, na, nb, n, ex)

        def alloc(lam):
            return {q: min(ex[q], int(np.floor(lam * w[q]))) for q in ex}

        lo, hi = 0.0, 1.0
        while sum(alloc(hi).values()) < D:
            hi *= 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if sum(alloc(mid).values()) <= D:
                lo = mid
            else:
                hi = mid
        dims.append({q: d for q, d in alloc(lo).items() if d > 0})
    # isometry caps from both sides, iterated to a fixed point
    changed = True
    while changed:
        changed = False
        for n in range(1, L + 1):
            for q in list(dims[n]):
                cap = sum(dims[n - 1].get(_qsub(q, s), 0) for s in QS)
                if dims[n][q] > cap:
                    dims[n][q] = cap
                    changed = True
            dims[n] = {q: d for q, d in dims[n].items() if d > 0}
        for n in range(L - 1, -1, -1):
            for q in list(dims[n]):
                cap = sum(dims[n + 1].get(_qadd(q, s), 0) for s in QS)
                if dims[n][q] > cap:
                    dims[n][q] = cap
                    changed = True
            dims[n] = {q: d for q, d in dims[n].items() if d > 0}
    return [dict(sorted(d.items())) for d in dims]


def _left_isometry(dl, dr, rng):
    """Random left-canonical tensor: for each right sector the stacked
    (q_left, s) rows have orthonormal columns."""
    t = {}
    for qr, ncol in dr.items():
        parts = [(s, _qsub(qr, QS[s])) for s in range(4) if _qsub(qr, QS[s]) in dl]
        nrow = sum(dl[ql] for _, ql in parts)
        g = rng.normal(size=(nrow, ncol))
        q, _ = np.linalg.qr(g)
        q = q[:, :ncol]
        off = 0
        for s, ql in parts:
            t[(ql, s)] = np.ascontiguousarray(q[off:off + dl[ql], :])
            off += dl[ql]
    return t


def _right_isometry(dl, dr, rng):
    """Random right-canonical tensor: for each left sector the concatenated
    (s, q_right) columns have orthonormal rows."""
    t = {}
    for ql, nrow in dl.items():
        parts = [(s, _qadd(ql, QS[s])) for s in range(4) if _qadd(ql, QS[s]) in dr]
        ncol = sum(dr[qr] for _, qr in parts)
        g = rng.normal(size=(ncol, nrow))
        q, _ = np.linalg.qr(g)
        q = q[:, :nrow].T
        off = 0
        for s, qr in parts:
            t[(ql, s)] = np.ascontiguousarray(q[:, off:off + dr[qr]])
            off += dr[qr]
    return t


def random_mps(L, na, nb, D, center, seed=None):
    """Random MPS in mixed-canonical form around the two-site position
    (center, center+1): sites < center are left isometries, sites > center+1
    are right isometries, and the two center sites carry no tensor.

    Returns (dims, tensors) with dims from bond_sector_dims and tensors a list
    of length L whose entries for the two center sites are None.
    """
    if seed is None:
        seed = mps_seed(L)
    rng = np.random.default_rng(seed)
    dims = bond_sector_dims(L, na, nb, D)
    tensors = [None] * L
    for n in range(L):
        if n < center:
            tensors[n] = _left_isometry(dims[n], dims[n + 1], rng)
        elif n > center + 1:
            tensors[n] = _right_isometry(dims[n], dims[n + 1], rng)
    return dims, tensors


def random_full_mps(L, na, nb, D, seed=None):
    """Random site tensors for every site: left isometries everywhere (the
    last one maps onto the single target sector).  Used as a DMRG start."""
    if seed is None:
        seed = mps_seed(L)
    rng = np.random.default_rng(seed)
    dims = bond_sector_dims(L, na, nb, D)
    tensors = [_right_isometry(dims[n], dims[n + 1], rng) for n in range(L)]
    return dims, tensors


def two_site_blocks(dl, dr):
    """Sorted block list [(q_left, s1, s2, q_right)] of a two-site wave
    function between left bond dims dl and right bond dims dr.  Both labels
    are bond labels (electrons to the left of the bond), so
    q_right = q_left + q_s1 + q_s2."""
    out = []
    for ql in sorted(dl):
        for s1 in range(4):
            for s2 in range(4):
                qr = _qadd(_qadd(ql, QS[s1]), QS[s2])
                if qr in dr:
                    out.append((ql, s1, s2, qr))
    return out


def random_two_site_psi(dl, dr, seed):
    """Gaussian two-site wave function, normalized to 1."""
    rng = np.random.default_rng(seed)
    psi = {}
    for ql, s1, s2, qr in two_site_blocks(dl, dr):
        psi[(ql, s1, s2)] = rng.normal(size=(dl[ql], dr[qr]))
    nrm = np.sqrt(sum(float(np.sum(b * b)) for b in psi.values()))
    for k in psi:
        psi[k] /= nrm
    return psi
