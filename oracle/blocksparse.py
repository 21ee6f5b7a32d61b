"""Block-sparse operators and two-site products (plain numpy, float64).

Conserved (N_alpha, N_beta) split every operator into dense sector blocks
(Sec. II.B, Fig. 4a).  An operator with quantum-number change dq is stored
as {q_in: array(d_out(q_in + dq), d_in(q_in))}.  Right-block sector labels
count the electrons inside the block (so dq is the physical change on both
sides); conversion from MPS bond labels happens at the edges.

Fermionic conventions: a product state of consecutive parts |x y> is the
Jordan-Wigner ordered product (x-string)(y-string)|0>, so an operator on the
right part that is odd picks up (-1)^{n_x} (graded tensor product).
"""

import numpy as np

from .siteops import QSITE


def qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def qsub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def qneg(a):
    return (-a[0], -a[1])


def qpar(q):
    return (q[0] + q[1]) & 1


class BlockOp:
    __slots__ = ("dq", "blocks")

    def __init__(self, dq, blocks=None):
        self.dq = dq
        self.blocks = {} if blocks is None else blocks

    @property
    def parity(self):
        return qpar(self.dq)

    def T(self):
        return BlockOp(qneg(self.dq), {qadd(q, self.dq): b.T for q, b in self.blocks.items()})

    def scaled(self, c):
        return BlockOp(self.dq, {q: c * b for q, b in self.blocks.items()})

    def norm(self):
        return np.sqrt(sum(float(np.sum(b * b)) for b in self.blocks.values()))


def identity(basis):
    return BlockOp((0, 0), {q: np.eye(d) for q, d in basis.items()})


def lincomb(terms, dq):
    """sum_k c_k O_k for operators sharing dq; returns a BlockOp."""
    out = BlockOp(dq)
    for c, op in terms:
        if c == 0.0 or op is None:
            continue
        assert op.dq == dq
        for q, b in op.blocks.items():
            if q in out.blocks:
                out.blocks[q] = out.blocks[q] + c * b
            else:
                out.blocks[q] = c * b
    return out


class Enlarged:
    """Product basis of two consecutive parts.  side='left': X = L . s with
    the site on the right; side='right': Y = s . R with the site on the left.
    parts[q] = list of (s, q_block, offset, dim) in increasing s."""

    def __init__(self, basis, side):
        self.side = side
        parts = {}
        for s in range(4):
            for qb, d in basis.items():
                q = qadd(qb, QSITE[s])
                parts.setdefault(q, []).append((s, qb, d))
        self.parts = {}
        self.dims = {}
        self.offset = {}
        for q in sorted(parts):
            off = 0
            lst = []
            for s, qb, d in sorted(parts[q]):
                lst.append((s, qb, off, d))
                self.offset[(q, s)] = off
                off += d
            self.parts[q] = lst
            self.dims[q] = off
        self.basis = basis


def materialize(terms, enl, dq):
    """Materialize sum_k (block op_k) (x) (site matrix M_k) on an Enlarged basis.

    terms: list of (op or None for identity, 4x4 matrix).  For side='left' the
    product is O^L M (site to the right): the graded sign is (-1)^{|M| n_l}.
    For side='right' it is M O^R (site to the left): the sign is
    (-1)^{|O^R| n_s}.  Entries of M are resolved one site transition at a time.
    """
    # accumulate an aggregated block operator per site transition (s', s)
    acc = {}
    for op, M in terms:
        nz = np.argwhere(M != 0.0)
        for sp_, s in nz:
            key = (int(sp_), int(s))
            lst = acc.setdefault(key, [])
            lst.append((M[sp_, s], op))
    out = BlockOp(dq)
    for (sp_, s), lst in acc.items():
        dq_site = qsub(QSITE[sp_], QSITE[s])
        dq_blk = qsub(dq, dq_site)
        site_par = qpar(dq_site)
        blk_par = qpar(dq_blk)
        agg = {}
        for c, op in lst:
            if op is None:
                if dq_blk != (0, 0):
                    raise ValueError("identity term with a non-zero block dq")
                for q, d in enl.basis.items():
                    agg[q] = agg.get(q, 0.0) + c * np.eye(d)
            else:
                if op.dq != dq_blk:
                    raise ValueError("inconsistent dq in materialize")
                for q, b in op.blocks.items():
                    agg[q] = agg[q] + c * b if q in agg else c * b
        for qb, b in agg.items():
            qb_out = qadd(qb, dq_blk)
            if qb_out not in enl.basis:
                continue
            if enl.side == "left":
                sign = -1.0 if (site_par and qpar(qb)) else 1.0
            else:
                sign = -1.0 if (blk_par and qpar(QSITE[s])) else 1.0
            q_in = qadd(qb, QSITE[s])
            q_out = qadd(qb_out, QSITE[sp_])
            if q_in not in enl.dims or q_out not in enl.dims:
                continue
            if q_in not in out.blocks:
                out.blocks[q_in] = np.zeros((enl.dims[q_out], enl.dims[q_in]))
            ro = enl.offset[(q_out, sp_)]
            co = enl.offset[(q_in, s)]
            out.blocks[q_in][ro:ro + b.shape[0], co:co + b.shape[1]] += sign * b
    return out


def left_stack(A, enl, newbasis):
    """Stack a left isometry {(q_l, s): (d_l, d_new)} into {q_new: (d_X, d_new)}."""
    out = {}
    for q, d in newbasis.items():
        if q not in enl.dims:
            continue
        m = np.zeros((enl.dims[q], d))
        for s, ql, off, dl in enl.parts[q]:
            if (ql, s) in A:
                m[off:off + dl, :] = A[(ql, s)]
        out[q] = m
    return out


def right_stack(B, enl, newbasis, target):
    """Stack a right isometry given in bond labels {(q_bond, s): (d_new, d_r)}
    into {q_new: (d_new, d_Y)} with q_new = electrons in the enlarged block."""
    out = {}
    for q, d in newbasis.items():
        if q not in enl.dims:
            continue
        m = np.zeros((d, enl.dims[q]))
        qbond = qsub(target, q)
        for s, qr, off, dr in enl.parts[q]:
            if (qbond, s) in B:
                m[:, off:off + dr] = B[(qbond, s)]
        out[q] = m
    return out


def renormalize_left(op, stack):
    """O' = A^T O A on the new left basis."""
    out = BlockOp(op.dq)
    for q, b in op.blocks.items():
        qo = qadd(q, op.dq)
        if q in stack and qo in stack:
            out.blocks[q] = stack[qo].T @ b @ stack[q]
    return out


def renormalize_right(op, stack):
    """O' = B O B^T on the new right basis."""
    out = BlockOp(op.dq)
    for q, b in op.blocks.items():
        qo = qadd(q, op.dq)
        if q in stack and qo in stack:
            out.blocks[q] = stack[qo] @ b @ stack[q].T
    return out
