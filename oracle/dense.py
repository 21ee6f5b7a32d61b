"""Dense effective-Hamiltonian product by its definition (tiny systems).

For an MPS that is left-canonical on sites 0..i-1 and right-canonical on
sites i+2..L-1, P maps a two-site wave function psi[l, s1, s2, r] to the
full (N_alpha, N_beta) determinant space (Eq. 2 with the two center sites
left open).  The effective Hamiltonian of the two-site step (Sec. II.B,
step 2) is H_eff = P^T H P, so the oracle product is H_eff psi = P^T (H (P psi)),
with H the full-CI matrix of oracle.fci.

Site-tuple codes sum_k s_k 4^(L-1-k) index the Fock basis; a site tuple is
the Jordan-Wigner ordered product of the site creation strings, which is the
same state as the interleaved determinant of oracle.fci.
"""

import numpy as np

from synthetic.mps import QS
from .fci import det_to_site_code


def _qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def left_basis(tensors, upto):
    """{q: (codes, U)} for bond `upto` from left isometries 0..upto-1."""
    basis = {(0, 0): (np.array([0], dtype=np.int64), np.ones((1, 1)))}
    for n in range(upto):
        A = tensors[n]
        new = {}
        for (ql, s), blk in A.items():
            if ql not in basis:
                continue
            qr = _qadd(ql, QS[s])
            codes, U = basis[ql]
            new.setdefault(qr, []).append((s, codes * 4 + s, U @ blk))
        basis = {}
        for qr, parts in new.items():
            parts.sort(key=lambda t: t[0])
            basis[qr] = (np.concatenate([p[1] for p in parts]),
                         np.vstack([p[2] for p in parts]))
    return basis


def right_basis(tensors, L, target, frm):
    """{q: (codes, U)} for bond `frm` from right isometries frm..L-1; q counts
    the electrons to the left of the bond; codes index sites frm..L-1."""
    basis = {target: (np.array([0], dtype=np.int64), np.ones((1, 1)))}
    for n in range(L - 1, frm - 1, -1):
        B = tensors[n]
        width = 4 ** (L - n - 1)
        new = {}
        for (ql, s), blk in B.items():
            qr = _qadd(ql, QS[s])
            if qr not in basis:
                continue
            codes, U = basis[qr]
            new.setdefault(ql, []).append((s, s * width + codes, U @ blk.T))
        basis = {}
        for ql, parts in new.items():
            parts.sort(key=lambda t: t[0])
            basis[ql] = (np.concatenate([p[1] for p in parts]),
                         np.vstack([p[2] for p in parts]))
    return basis


class DenseHeff:
    """P^T H P for the two-site position (i, i+1)."""

    def __init__(self, H, dets, L, tensors, i, target):
        self.H = H
        self.L = L
        self.i = i
        self.codes = det_to_site_code(dets, L)
        self.lb = left_basis(tensors, i)
        self.rb = right_basis(tensors, L, target, i + 2)
        self.target = target
        self.nfull = 4 ** L

    def _full_codes(self, ql, s1, s2, qr):
        lc = self.lb[ql][0]
        rc = self.rb[qr][0]
        L, i = self.L, self.i
        base = (lc * 16 + s1 * 4 + s2) * (4 ** (L - i - 2))
        return base[:, None] + rc[None, :]

    def expand(self, psi):
        """P psi as a vector over the determinants of the sector."""
        full = np.zeros(self.nfull)
        for (ql, s1, s2), blk in psi.items():
            qr = _add3(ql, s1, s2)
            full[self._full_codes(ql, s1, s2, qr)] += self.lb[ql][1] @ blk @ self.rb[qr][1].T
        return full[self.codes]

    def project(self, v, like):
        """P^T v onto the block structure of `like`."""
        full = np.zeros(self.nfull)
        full[self.codes] = v
        out = {}
        for (ql, s1, s2) in like:
            qr = _add3(ql, s1, s2)
            out[(ql, s1, s2)] = self.lb[ql][1].T @ full[self._full_codes(ql, s1, s2, qr)] @ self.rb[qr][1]
        return out

    def apply(self, psi):
        return self.project(self.H @ self.expand(psi), psi)


def _add3(ql, s1, s2):
    return (ql[0] + QS[s1][0] + QS[s2][0], ql[1] + QS[s1][1] + QS[s2][1])
