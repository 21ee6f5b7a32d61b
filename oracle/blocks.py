"""Renormalized block operators: normal set on the left, complementary set on
the right, the blocking (enlargement) formulas and renormalization.

Partition rule (two parts X | Y, X to the left) used everywhere:

  H = H_X + H_Y + sum_{x in X} (a+_x S^Y_x + h.c.) + sum_{y in Y} (S^X_y a_y + h.c.)
      + sum_{p<q in X} (a+_p a+_q P^Y_pq + h.c.) + sum_{p,q in X} a+_p a_q Q^Y_pq

  S^Y_x  = sum_{y in Y} t_xy a_y + 1/2 sum_{qrs in Y} (g_xqrs - g_qxrs) a+_q a_r a_s
  S^X_y  = 1/2 sum_{pqu in X} (g_pquy - g_pqyu) a+_p a+_q a_u
  P^Y_pq = 1/2 sum_{rs in Y} (g_pqrs - g_qprs) a_r a_s
  Q^Y_pq = sum_{y,y' in Y} (g_{p y y' q} - g_{p y q y'}) a+_y a_y'

A left block (sites 0..k-1) keeps H, a+_p, A_pq = a+_p a+_q (p<q), B_pq =
a+_p a_q and S_y for every spin-orbital y to its right.  A right block keeps H,
a+_r, and S_x, P_pq (p<q), Q_pq for every spin-orbital to its left.  Blocks are
enlarged by one site (the preprocessing/renormalization of Sec. II.B) and then
projected with the MPS isometry (Eq. 2).  Ops that vanish are left out.
"""

import numpy as np

from .blocksparse import (BlockOp, Enlarged, materialize, left_stack, right_stack,
                          renormalize_left, renormalize_right, identity, qneg, qsub)
from .siteops import site_op, ID4, QSITE

QA = (1, 0)
QB = (0, 1)


def mq(p):
    """Quantum number carried by a+ on spin-orbital p."""
    return QA if p % 2 == 0 else QB


def _nz(M):
    return M is not None and np.any(M != 0.0)


class SiteOps:
    """Exact single-site operators of site k (complete 4-dim basis)."""

    def __init__(self, k, t, g):
        self.k = k
        self.modes = (2 * k, 2 * k + 1)
        self.t, self.g = t, g

    def cd(self, p):
        return site_op(True, p % 2)

    def c(self, p):
        return site_op(False, p % 2)

    def H(self):
        t, g, m = self.t, self.g, self.modes
        M = np.zeros((4, 4))
        for a in m:
            for b in m:
                M += t[a, b] * self.cd(a) @ self.c(b)
        for p in m:
            for q in m:
                for r in m:
                    for s in m:
                        if g[p, q, r, s] != 0.0:
                            M += 0.5 * g[p, q, r, s] * self.cd(p) @ self.cd(q) @ self.c(r) @ self.c(s)
        return M

    def S_yrole(self, x):
        """S^s_x for x to the left of the site (site on the Y side)."""
        t, g, m = self.t, self.g, self.modes
        M = np.zeros((4, 4))
        for a in m:
            M += t[x, a] * self.c(a)
        for q in m:
            for r in m:
                for s in m:
                    w = 0.5 * (g[x, q, r, s] - g[q, x, r, s])
                    if w != 0.0:
                        M += w * self.cd(q) @ self.c(r) @ self.c(s)
        return M

    def S_xrole(self, y):
        """S^s_y for y to the right of the site (site on the X side)."""
        g, m = self.g, self.modes
        M = np.zeros((4, 4))
        for p in m:
            for q in m:
                for u in m:
                    w = 0.5 * (g[p, q, u, y] - g[p, q, y, u])
                    if w != 0.0:
                        M += w * self.cd(p) @ self.cd(q) @ self.c(u)
        return M

    def P(self, p, q):
        g, m = self.g, self.modes
        M = np.zeros((4, 4))
        for r in m:
            for s in m:
                w = 0.5 * (g[p, q, r, s] - g[q, p, r, s])
                if w != 0.0:
                    M += w * self.c(r) @ self.c(s)
        return M

    def Q(self, p, q):
        g, m = self.g, self.modes
        M = np.zeros((4, 4))
        for y in m:
            for y2 in m:
                w = g[p, y, y2, q] - g[p, y, q, y2]
                if w != 0.0:
                    M += w * self.cd(y) @ self.c(y2)
        return M


class Block:
    """A left or right block: basis {q: dim} (electrons inside the block) and
    a dict of named BlockOps."""

    def __init__(self, side, sites, basis, ops):
        self.side = side
        self.sites = sites          # (first, last+1)
        self.basis = basis
        self.ops = ops

    @property
    def modes(self):
        return range(2 * self.sites[0], 2 * self.sites[1])

    def get(self, *key):
        return self.ops.get(key)


def left_vacuum(L):
    return Block("left", (0, 0), {(0, 0): 1}, {("H",): BlockOp((0, 0), {(0, 0): np.zeros((1, 1))})})


def right_vacuum(L):
    return Block("right", (L, L), {(0, 0): 1}, {("H",): BlockOp((0, 0), {(0, 0): np.zeros((1, 1))})})


def _keep(ops, key, op):
    if op is not None and op.blocks and op.norm() > 0.0:
        ops[key] = op


def enlarge_left(blk, t, g, nmodes):
    """X = L . s with s = site blk.sites[1]; returns (Enlarged, ops) of X in
    the left (normal) role, materialized and not yet projected."""
    k = blk.sites[1]
    site = SiteOps(k, t, g)
    enl = Enlarged(blk.basis, "left")
    Lm = list(blk.modes)
    Sm = list(site.modes)
    right = range(2 * k + 2, nmodes)
    G = blk.get
    ops = {}
    # H
    terms = [(G("H"), ID4), (None, site.H())]
    for x in Lm:
        M = site.S_yrole(x)
        if _nz(M) and G("cd", x) is not None:
            terms += [(G("cd", x), M), (G("cd", x).T(), -M.T)]
    for a in Sm:
        S = G("S", a)
        if S is not None:
            terms += [(S, site.c(a)), (S.T(), -site.cd(a))]
    for i, p in enumerate(Lm):
        for q in Lm[i + 1:]:
            A = G("A", p, q)
            if A is None:
                continue
            M = site.P(p, q)
            if _nz(M):
                terms += [(A, M), (A.T(), M.T)]
    for p in Lm:
        for q in Lm:
            B = G("B", p, q)
            if B is None:
                continue
            M = site.Q(p, q)
            if _nz(M):
                terms.append((B, M))
    _keep(ops, ("H",), materialize(terms, enl, (0, 0)))
    # a+
    for p in Lm:
        if G("cd", p) is not None:
            _keep(ops, ("cd", p), materialize([(G("cd", p), ID4)], enl, mq(p)))
    for p in Sm:
        _keep(ops, ("cd", p), materialize([(None, site.cd(p))], enl, mq(p)))
    # A, B
    X = Lm + Sm
    for i, p in enumerate(X):
        for q in X[i + 1:]:
            dq = (mq(p)[0] + mq(q)[0], mq(p)[1] + mq(q)[1])
            if q in Lm:
                tm = [(G("A", p, q), ID4)] if G("A", p, q) is not None else []
            elif p in Lm:
                tm = [(G("cd", p), site.cd(q))] if G("cd", p) is not None else []
            else:
                tm = [(None, site.cd(p) @ site.cd(q))]
            if tm:
                _keep(ops, ("A", p, q), materialize(tm, enl, dq))
    for p in X:
        for q in X:
            dq = qsub(mq(p), mq(q))
            if p in Lm and q in Lm:
                tm = [(G("B", p, q), ID4)] if G("B", p, q) is not None else []
            elif p in Lm:
                tm = [(G("cd", p), site.c(q))] if G("cd", p) is not None else []
            elif q in Lm:
                tm = [(G("cd", q).T(), -site.cd(p))] if G("cd", q) is not None else []
            else:
                tm = [(None, site.cd(p) @ site.c(q))]
            if tm:
                _keep(ops, ("B", p, q), materialize(tm, enl, dq))
    # S_y for y to the right of X
    for y in right:
        K = 0.5 * (g[:, :, :, y] - np.transpose(g[:, :, y, :], (0, 1, 2)))
        terms = []
        if G("S", y) is not None:
            terms.append((G("S", y), ID4))
        M = site.S_xrole(y)
        if _nz(M):
            terms.append((None, M))
        for u in Sm:
            for i, p in enumerate(Lm):
                for q in Lm[i + 1:]:
                    w = K[p, q, u] - K[q, p, u]
                    if w != 0.0 and G("A", p, q) is not None:
                        terms.append((G("A", p, q), w * site.c(u)))
        for a in Sm:
            for p in Lm:
                for u in Lm:
                    w = K[a, p, u] - K[p, a, u]
                    if w != 0.0 and G("B", p, u) is not None:
                        terms.append((G("B", p, u), w * site.cd(a)))
        for x in Lm:
            M = np.zeros((4, 4))
            for b in Sm:
                for c in Sm:
                    w = K[x, b, c] - K[b, x, c]
                    if w != 0.0:
                        M += w * site.cd(b) @ site.c(c)
            if _nz(M) and G("cd", x) is not None:
                terms.append((G("cd", x), M))
        for u in Lm:
            M = np.zeros((4, 4))
            for p in Sm:
                for q in Sm:
                    w = K[p, q, u]
                    if w != 0.0:
                        M += w * site.cd(p) @ site.cd(q)
            if _nz(M) and G("cd", u) is not None:
                terms.append((G("cd", u).T(), M))
        if terms:
            _keep(ops, ("S", y), materialize(terms, enl, mq(y)))
    return enl, ops


def enlarge_right(blk, t, g):
    """Y = s . R with s = site blk.sites[0]-1; returns (Enlarged, ops) of Y in
    the right (complementary) role, materialized and not yet projected."""
    k = blk.sites[0] - 1
    site = SiteOps(k, t, g)
    enl = Enlarged(blk.basis, "right")
    Rm = list(blk.modes)
    Sm = list(site.modes)
    left = list(range(0, 2 * k))
    G = blk.get
    ops = {}

    def c_r(y):
        cd = G("cd", y)
        return None if cd is None else cd.T()

    # H
    terms = [(G("H"), ID4), (None, site.H())]
    for a in Sm:
        S = G("S", a)
        if S is not None:
            terms += [(S, site.cd(a)), (S.T(), -site.c(a))]
    for r in Rm:
        M = site.S_xrole(r)
        if _nz(M) and G("cd", r) is not None:
            terms += [(c_r(r), M), (G("cd", r), -M.T)]
    for i, p in enumerate(Sm):
        for q in Sm[i + 1:]:
            P = G("P", p, q)
            if P is not None:
                M = site.cd(p) @ site.cd(q)
                terms += [(P, M), (P.T(), M.T)]
    for p in Sm:
        for q in Sm:
            Q = G("Q", p, q)
            if Q is not None:
                terms.append((Q, site.cd(p) @ site.c(q)))
    _keep(ops, ("H",), materialize(terms, enl, (0, 0)))
    # a+
    for y in Sm:
        _keep(ops, ("cd", y), materialize([(None, site.cd(y))], enl, mq(y)))
    for y in Rm:
        if G("cd", y) is not None:
            _keep(ops, ("cd", y), materialize([(G("cd", y), ID4)], enl, mq(y)))
    # S_x for x to the left of Y
    for x in left:
        terms = []
        if G("S", x) is not None:
            terms.append((G("S", x), ID4))
        M = site.S_yrole(x)
        if _nz(M):
            terms.append((None, M))
        for q in Sm:
            P = G("P", x, q)
            if P is not None:
                terms.append((P, site.cd(q)))
        for a in Sm:
            Q = G("Q", x, a)
            if Q is not None:
                terms.append((Q, site.c(a)))
        for u in Rm:
            if G("cd", u) is None:
                continue
            M1 = np.zeros((4, 4))   # (q, r in s; u in R)
            M2 = np.zeros((4, 4))   # (q, u in s; r = this R mode)
            M3 = np.zeros((4, 4))   # (r, u in s; q = this R mode)
            for a in Sm:
                for b in Sm:
                    w1 = 0.5 * (g[x, a, b, u] - g[a, x, b, u])
                    if w1 != 0.0:
                        M1 += w1 * site.cd(a) @ site.c(b)
                    w2 = 0.5 * (g[x, a, u, b] - g[a, x, u, b])
                    if w2 != 0.0:
                        M2 -= w2 * site.cd(a) @ site.c(b)
                    w3 = 0.5 * (g[x, u, a, b] - g[u, x, a, b])
                    if w3 != 0.0:
                        M3 += w3 * site.c(a) @ site.c(b)
            if _nz(M1 + M2):
                terms.append((c_r(u), M1 + M2))
            if _nz(M3):
                terms.append((G("cd", u), M3))
        if terms:
            _keep(ops, ("S", x), materialize(terms, enl, qneg(mq(x))))
    # P_pq, Q_pq for p, q to the left of Y
    for i, p in enumerate(left):
        for q in left[i + 1:]:
            dq = qneg((mq(p)[0] + mq(q)[0], mq(p)[1] + mq(q)[1]))
            terms = []
            if G("P", p, q) is not None:
                terms.append((G("P", p, q), ID4))
            M = site.P(p, q)
            if _nz(M):
                terms.append((None, M))
            for a in Sm:
                for y in Rm:
                    w = g[p, q, a, y] - g[p, q, y, a]
                    if w != 0.0 and G("cd", y) is not None:
                        terms.append((c_r(y), w * site.c(a)))
            if terms:
                _keep(ops, ("P", p, q), materialize(terms, enl, dq))
    for p in left:
        for q in left:
            dq = qsub(mq(q), mq(p))
            terms = []
            if G("Q", p, q) is not None:
                terms.append((G("Q", p, q), ID4))
            M = site.Q(p, q)
            if _nz(M):
                terms.append((None, M))
            for a in Sm:
                for y in Rm:
                    if G("cd", y) is None:
                        continue
                    w = g[p, a, y, q] - g[p, a, q, y]
                    if w != 0.0:
                        terms.append((c_r(y), w * site.cd(a)))
                    w = g[p, y, a, q] - g[p, y, q, a]
                    if w != 0.0:
                        terms.append((G("cd", y), -w * site.c(a)))
            if terms:
                _keep(ops, ("Q", p, q), materialize(terms, enl, dq))
    return enl, ops


def project_left(blk, enl, ops, A, newbasis):
    stack = left_stack(A, enl, newbasis)
    new = {}
    for key, op in ops.items():
        _keep(new, key, renormalize_left(op, stack))
    return Block("left", (0, blk.sites[1] + 1), dict(newbasis), new)


def project_right(blk, enl, ops, B, newbasis_bond, target):
    newbasis = {qsub(target, q): d for q, d in newbasis_bond.items()}
    stack = right_stack(B, enl, newbasis, target)
    new = {}
    for key, op in ops.items():
        _keep(new, key, renormalize_right(op, stack))
    return Block("right", (blk.sites[0] - 1, blk.sites[1]), newbasis, new)


def build_left_blocks(tensors, upto, t, g):
    """Left blocks for bonds 0..upto from left isometries 0..upto-1."""
    nmodes = t.shape[0]
    L = nmodes // 2
    blocks = [left_vacuum(L)]
    for n in range(upto):
        A = tensors[n]
        newbasis = {}
        for (ql, s), b in A.items():
            newbasis[(ql[0] + QSITE[s][0], ql[1] + QSITE[s][1])] = b.shape[1]
        enl, ops = enlarge_left(blocks[-1], t, g, nmodes)
        blocks.append(project_left(blocks[-1], enl, ops, A, dict(sorted(newbasis.items()))))
    return blocks


def build_right_blocks(tensors, frm, t, g, target):
    """Right blocks for bonds L..frm (returned as {bond: Block})."""
    nmodes = t.shape[0]
    L = nmodes // 2
    blocks = {L: right_vacuum(L)}
    for n in range(L - 1, frm - 1, -1):
        B = tensors[n]
        newbasis = {ql: b.shape[0] for (ql, s), b in B.items()}
        enl, ops = enlarge_right(blocks[n + 1], t, g)
        blocks[n] = project_right(blocks[n + 1], enl, ops, B, dict(sorted(newbasis.items())), target)
    return blocks
