"""Plain two-site DMRG (Sec. II.A-B) on the block-sparse oracle operators.

One iteration step at two-site position (i, i+1): build the effective
Hamiltonian from the left block of bond i and the right block of bond i+2
(preprocessing), find its lowest eigenpair with Lanczos (scipy eigsh;
deliberately a different eigensolver from the HIP path's Davidson), split the
two-site wave function by a per-sector SVD keeping the D largest singular
values (postprocessing), renormalize the enlarged block with the new isometry,
and transform the wave function into the start vector of the next step.  A
sweep runs the cut left to right over every position and then right to left.

Truncation rule (the paper fixes none): sort the singular values of all
sectors together, keep the D largest, extend the kept set to every value
>= sigma_D (1 - 1e-10) so exact degeneracies are never split, and drop values
<= 1e-6 sigma_max (weight 1e-12 of the largest): below that a singular value
is not determined by a wave function that the eigensolver fixes only to its
residual tolerance, so whether such a state is kept would depend on rounding.
The truncation error is the discarded weight sum sigma^2.
"""

import numpy as np
import scipy.sparse.linalg as sla

from synthetic.mps import random_full_mps, random_two_site_psi
from .blocks import (build_right_blocks, enlarge_left, enlarge_right, project_left,
                     project_right, left_vacuum)
from .hpsi import BlockSparseHeff
from .siteops import QSITE, spin_orbital_integrals


def _qa(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _qs(a, b):
    return (a[0] - b[0], a[1] - b[1])


def flatten(psi, keys):
    return np.concatenate([psi[k].ravel() for k in keys])


def unflatten(v, keys, shapes):
    out, o = {}, 0
    for k, s in zip(keys, shapes):
        n = s[0] * s[1]
        out[k] = v[o:o + n].reshape(s)
        o += n
    return out


def lowest_eigenpair(heff, guess, tol=1e-12):
    keys = sorted(guess)
    if not keys:
        raise ValueError("empty two-site space: bond sectors are incompatible")
    shapes = [guess[k].shape for k in keys]
    n = sum(a * b for a, b in shapes)

    def mv(v):
        return flatten(heff.apply(unflatten(v, keys, shapes)), keys)

    v0 = flatten(guess, keys)
    if n <= 64:
        M = np.column_stack([mv(e) for e in np.eye(n)])
        w, V = np.linalg.eigh(0.5 * (M + M.T))
        e, x = w[0], V[:, 0]
    else:
        A = sla.LinearOperator((n, n), matvec=mv, dtype=float)
        w, V = sla.eigsh(A, k=1, which="SA", v0=v0, tol=tol, ncv=min(n, 40))
        e, x = w[0], V[:, 0]
    x = x / np.linalg.norm(x)
    return float(e), unflatten(x, keys, shapes)


def split(psi, dl, dr, D):
    """Per-sector SVD of psi[(q_l, s1) ; (s2, q_r)] with the global truncation
    rule.  Returns {q_mid: (U blocks by s1, s, Vt blocks by s2)}, kept dims and
    the truncation error."""
    sectors = {}
    for (ql, s1, s2), b in psi.items():
        qm = _qa(ql, QSITE[s1])
        sectors.setdefault(qm, []).append((ql, s1, s2, b))
    svd = {}
    allsig = []
    for qm, lst in sectors.items():
        rows = [(s1, _qs(qm, QSITE[s1])) for s1 in range(4) if _qs(qm, QSITE[s1]) in dl]
        cols = [(s2, _qa(qm, QSITE[s2])) for s2 in range(4) if _qa(qm, QSITE[s2]) in dr]
        nr = sum(dl[q] for _, q in rows)
        nc = sum(dr[q] for _, q in cols)
        M = np.zeros((nr, nc))
        roff, coff = {}, {}
        o = 0
        for s1, q in rows:
            roff[s1] = o
            o += dl[q]
        o = 0
        for s2, q in cols:
            coff[s2] = o
            o += dr[q]
        for ql, s1, s2, b in lst:
            M[roff[s1]:roff[s1] + b.shape[0], coff[s2]:coff[s2] + b.shape[1]] = b
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        svd[qm] = (rows, cols, roff, coff, U, s, Vt)
        allsig += [(float(x), qm) for x in s]
    sig = sorted((x for x, _ in allsig), reverse=True)
    smax = sig[0] if sig else 0.0
    if len(sig) > D:
        cut = sig[D - 1] * (1.0 - 1e-10)
    else:
        cut = -1.0
    floor = 1e-6 * smax
    keep = {}
    err = 0.0
    for qm, (rows, cols, roff, coff, U, s, Vt) in svd.items():
        k = int(np.sum((s >= cut) & (s > floor)))
        err += float(np.sum(s[k:] ** 2))
        if k > 0:
            keep[qm] = k
    return svd, keep, err


class OracleDMRG:
    """Two-site DMRG driver in float64 on the oracle's block operators."""

    def __init__(self, h, eri, na, nb, D_init, seed=None):
        self.L = h.shape[0]
        self.target = (na, nb)
        self.t, self.g = spin_orbital_integrals(h, eri)
        dims, T = random_full_mps(self.L, na, nb, D_init, seed)
        self.dims = dims
        self.T = T
        self.left = {0: left_vacuum(self.L)}
        self.right = build_right_blocks(T, 2, self.t, self.g, self.target)
        self.history = []

    def _heff(self, i):
        return BlockSparseHeff(self.left[i], self.right[i + 2], self.t, self.g, self.target)

    def step(self, i, guess, D, direction):
        heff = self._heff(i)
        e, psi = lowest_eigenpair(heff, guess)
        err, nxt = self.move(i, psi, D, direction)
        return e, err, nxt

    def move(self, i, psi, D, direction):
        """Split psi at (i, i+1) (direction > 0: new left-canonical tensor of
        site i and left block of bond i+1; else new right-canonical tensor of
        site i+1 and right block of bond i+1) and carry it into the start vector
        of the next position: S V^T B_{i+2} or A_{i-1} U S.  Returns the
        truncation error and that start vector."""
        dl, dr = self.dims[i], self.dims[i + 2]
        svd, keep, err = split(psi, dl, dr, D)
        newdims = dict(sorted(keep.items()))
        if direction > 0:
            A = {}
            nxt = {}
            for qm, k in keep.items():
                rows, cols, roff, coff, U, s, Vt = svd[qm]
                for s1, ql in rows:
                    A[(ql, s1)] = U[roff[s1]:roff[s1] + dl[ql], :k].copy()
                SV = s[:k, None] * Vt[:k, :]
                for s2, qr in cols:
                    blk = SV[:, coff[s2]:coff[s2] + dr[qr]]
                    if i + 2 < self.L:
                        B = self.T[i + 2]
                        for s3 in range(4):
                            if (qr, s3) in B:
                                nxt[(qm, s2, s3)] = nxt.get((qm, s2, s3), 0) + blk @ B[(qr, s3)]
            self.T[i] = A
            self.dims[i + 1] = newdims
            enl, ops = enlarge_left(self.left[i], self.t, self.g, 2 * self.L)
            self.left[i + 1] = project_left(self.left[i], enl, ops, A, newdims)
            return err, nxt
        else:
            B = {}
            nxt = {}
            for qm, k in keep.items():
                rows, cols, roff, coff, U, s, Vt = svd[qm]
                for s2, qr in cols:
                    B[(qm, s2)] = Vt[:k, coff[s2]:coff[s2] + dr[qr]].copy()
                US = U[:, :k] * s[None, :k]
                for s1, ql in rows:
                    blk = US[roff[s1]:roff[s1] + dl[ql], :]
                    if i > 0:
                        A = self.T[i - 1]
                        for s0 in range(4):
                            qll = _qs(ql, QSITE[s0])
                            if (qll, s0) in A:
                                nxt[(qll, s0, s1)] = nxt.get((qll, s0, s1), 0) + A[(qll, s0)] @ blk
            self.T[i + 1] = B
            self.dims[i + 1] = newdims
            enl, ops = enlarge_right(self.right[i + 2], self.t, self.g)
            self.right[i + 1] = project_right(self.right[i + 2], enl, ops, B, newdims, self.target)
            return err, nxt

    def _complete(self, guess, i):
        """Fill blocks missing from a transformed guess with zeros."""
        from synthetic.mps import two_site_blocks
        out = {}
        for ql, s1, s2, qr in two_site_blocks(self.dims[i], self.dims[i + 2]):
            k = (ql, s1, s2)
            out[k] = guess[k] if k in guess else np.zeros((self.dims[i][ql], self.dims[i + 2][qr]))
        return out

    def sweep(self, D, seed=0):
        """One full sweep (left to right, then right to left); returns the
        list of (position, energy, truncation error)."""
        L = self.L
        log = []
        guess = random_two_site_psi(self.dims[0], self.dims[2], seed) if not hasattr(self, "_guess") else self._guess
        for i in range(0, L - 2):
            e, err, nxt = self.step(i, self._complete(guess, i), D, +1)
            log.append((i, e, err))
            guess = nxt
        for i in range(L - 2, 0, -1):
            e, err, nxt = self.step(i, self._complete(guess, i), D, -1)
            log.append((i, e, err))
            guess = nxt
        self._guess = guess
        self.history += log
        return log
