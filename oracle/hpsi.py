"""Block-sparse two-site H.psi from renormalized operators (plain numpy).

The two-site superblock L . s_i | s_{i+1} . R (Sec. II.B, Fig. 3a) is split
as X = L . s_i (left enlarged block, normal operators) and Y = s_{i+1} . R
(right enlarged block, complementary operators); both enlarged blocks are
materialized in their product bases and H.psi follows the partition rule of
oracle.blocks term by term:
    Phi = sum_t  O^X_t  (sign_t Psi)  (O^Y_t)^T
with Psi[x, y] the two-site wave function as a matrix over the two enlarged
bases and sign_t = (-1)^{|O^Y_t| n_x}.
"""

import numpy as np

from .blocksparse import qadd, qsub, qpar
from .blocks import enlarge_left, enlarge_right
from .siteops import QSITE


class BlockSparseHeff:
    """H_eff for the two-site position (i, i+1) given the left block at bond i
    and the right block at bond i+2."""

    def __init__(self, left, right, t, g, target):
        self.target = target
        nmodes = t.shape[0]
        self.X, self.xops = enlarge_left(left, t, g, nmodes)
        self.Y, self.yops = enlarge_right(right, t, g)
        self.terms = self._terms()

    def _terms(self):
        X, Y = self.xops, self.yops
        out = []
        if ("H",) in X:
            out.append((X[("H",)], None, 1.0))
        if ("H",) in Y:
            out.append((None, Y[("H",)], 1.0))
        for key, op in X.items():
            if key[0] == "cd":
                S = Y.get(("S", key[1]))
                if S is not None:
                    out.append((op, S, 1.0))
                    out.append((op.T(), S.T(), -1.0))
        for key, op in Y.items():
            if key[0] == "cd":
                S = X.get(("S", key[1]))
                if S is not None:
                    out.append((S, op.T(), 1.0))
                    out.append((S.T(), op, -1.0))
        for key, op in X.items():
            if key[0] == "A":
                P = Y.get(("P",) + key[1:])
                if P is not None:
                    out.append((op, P, 1.0))
                    out.append((op.T(), P.T(), 1.0))
            elif key[0] == "B":
                Q = Y.get(("Q",) + key[1:])
                if Q is not None:
                    out.append((op, Q, 1.0))
        return out

    def to_matrix(self, psi):
        """Two-site psi {(q_l, s1, s2): (d_l, d_r)} -> {q_x: (d_X, d_Y)}."""
        out = {}
        for (ql, s1, s2), b in psi.items():
            qx = qadd(ql, QSITE[s1])
            qy = qsub(self.target, qx)
            if qx not in out:
                out[qx] = np.zeros((self.X.dims[qx], self.Y.dims[qy]))
            ro = self.X.offset[(qx, s1)]
            co = self.Y.offset[(qy, s2)]
            out[qx][ro:ro + b.shape[0], co:co + b.shape[1]] = b
        return out

    def from_matrix(self, M, like):
        out = {}
        for (ql, s1, s2), b in like.items():
            qx = qadd(ql, QSITE[s1])
            qy = qsub(self.target, qx)
            ro = self.X.offset[(qx, s1)]
            co = self.Y.offset[(qy, s2)]
            if qx in M:
                out[(ql, s1, s2)] = M[qx][ro:ro + b.shape[0], co:co + b.shape[1]].copy()
            else:
                out[(ql, s1, s2)] = np.zeros_like(b)
        return out

    def apply_matrix(self, Psi):
        Phi = {qx: np.zeros_like(b) for qx, b in Psi.items()}
        for OX, OY, c in self.terms:
            ypar = 0 if OY is None else OY.parity
            for qx, b in Psi.items():
                qy = qsub(self.target, qx)
                if OX is None:
                    qx2, left = qx, b
                else:
                    if qx not in OX.blocks:
                        continue
                    qx2 = qadd(qx, OX.dq)
                    left = OX.blocks[qx] @ b
                if qx2 not in Phi:
                    continue
                if OY is None:
                    res = left
                else:
                    if qy not in OY.blocks:
                        continue
                    res = left @ OY.blocks[qy].T
                sign = -1.0 if (ypar and qpar(qx)) else 1.0
                Phi[qx2] += (c * sign) * res
        return Phi

    def apply(self, psi):
        return self.from_matrix(self.apply_matrix(self.to_matrix(psi)), psi)
