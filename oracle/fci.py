"""Full configuration interaction in one (N_alpha, N_beta) sector.

Hamiltonian (Eq. 1, Sec. II.A) in the reading
    H = sum_{pq,s} h_pq a+_{ps} a_{qs}
        + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs},
i.e. T_ij^{ab} = h_ij d_ab and V_ijkl^{abcd} = 1/2 (il|jk) d_ad d_bc, with no
core energy.  Spin-orbital p = 2 i + sigma (sigma 0 = alpha, 1 = beta); the
Jordan-Wigner order is 0a, 0b, 1a, 1b, ... so that a site's doubly occupied
state is a+_{i alpha} a+_{i beta}|0>.

Two independent constructions are provided:
  * build_h_interleaved: applies every second-quantized term a+ a+ a a to
    all determinants as bit strings (interleaved ordering directly);
  * build_h_strings: alpha/beta string spaces, spin-summed generators
    E_pq, H = sum h E + 1/2 sum (pq|rs)(E_pq E_rs - d_qr E_ps), built in the
    alpha-first ordering and then carried to the interleaved ordering by the
    diagonal sign of the reordering permutation.
They share nothing but the sector enumeration.
"""

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def sector_determinants(L, na, nb):
    """Sorted array of interleaved occupation bit strings (bit 2i+sigma)."""
    alphas = _strings(L, na)
    betas = _strings(L, nb)
    dets = []
    for a in alphas:
        for b in betas:
            d = 0
            for i in range(L):
                if (a >> i) & 1:
                    d |= 1 << (2 * i)
                if (b >> i) & 1:
                    d |= 1 << (2 * i + 1)
            dets.append(d)
    return np.array(sorted(dets), dtype=np.int64)


def _strings(L, n):
    out = []
    for occ in combinations(range(L), n):
        s = 0
        for i in occ:
            s |= 1 << i
        out.append(s)
    return sorted(out)


def det_to_site_code(dets, L):
    """Site-tuple code sum_i s_i 4^(L-1-i) with s = n_alpha + 2 n_beta."""
    code = np.zeros_like(dets)
    for i in range(L):
        s = ((dets >> (2 * i)) & 1) + 2 * ((dets >> (2 * i + 1)) & 1)
        code = code + s * (4 ** (L - 1 - i))
    return code


# ---------------------------------------------------------------- construction (a)

def _popcount(x):
    return np.bitwise_count(x.astype(np.uint64)).astype(np.int64)


def _apply_annihilate(dets, sign, ok, p):
    occ = ((dets >> p) & 1).astype(bool)
    ok = ok & occ
    below = dets & ((1 << p) - 1)
    sign = sign * np.where(_popcount(below) % 2 == 1, -1.0, 1.0)
    dets = dets & ~(1 << p)
    return dets, sign, ok


def _apply_create(dets, sign, ok, p):
    occ = ((dets >> p) & 1).astype(bool)
    ok = ok & ~occ
    below = dets & ((1 << p) - 1)
    sign = sign * np.where(_popcount(below) % 2 == 1, -1.0, 1.0)
    dets = dets | (1 << p)
    return dets, sign, ok


def _apply_string(dets, ops):
    """ops: list of (is_creator, p) applied right to left (last first)."""
    cur = dets.copy()
    sign = np.ones(len(dets))
    ok = np.ones(len(dets), dtype=bool)
    for cre, p in reversed(ops):
        if cre:
            cur, sign, ok = _apply_create(cur, sign, ok, p)
        else:
            cur, sign, ok = _apply_annihilate(cur, sign, ok, p)
    return cur, sign, ok


def build_h_interleaved(h, eri, na, nb):
    """Sparse CSR Hamiltonian over sector_determinants(L, na, nb)."""
    L = h.shape[0]
    dets = sector_determinants(L, na, nb)
    rows, cols, vals = [], [], []
    idx = np.arange(len(dets))

    def add(ops, coef):
        new, sign, ok = _apply_string(dets, ops)
        if not ok.any():
            return
        j = np.searchsorted(dets, new[ok])
        rows.append(j)
        cols.append(idx[ok])
        vals.append(coef * sign[ok])

    for i in range(L):
        for j in range(L):
            if h[i, j] == 0.0:
                continue
            for s in range(2):
                add([(True, 2 * i + s), (False, 2 * j + s)], h[i, j])
    # 1/2 (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s}: the annihilation half
    # a_{s t} a_{q s} is applied once per (q, s, spins) and reused
    for q in range(L):
        for s_ in range(L):
            for sg in range(2):
                for tg in range(2):
                    mid, sgn0, ok0 = _apply_string(dets, [(False, 2 * s_ + tg), (False, 2 * q + sg)])
                    if not ok0.any():
                        continue
                    mid, sgn0, src_idx = mid[ok0], sgn0[ok0], idx[ok0]
                    for p in range(L):
                        for r in range(L):
                            g = eri[p, q, r, s_]
                            if g == 0.0:
                                continue
                            cur, sign, ok = mid, sgn0, np.ones(len(mid), dtype=bool)
                            cur, sign, ok = _apply_create(cur, sign, ok, 2 * r + tg)
                            cur, sign, ok = _apply_create(cur, sign, ok, 2 * p + sg)
                            if not ok.any():
                                continue
                            rows.append(np.searchsorted(dets, cur[ok]))
                            cols.append(src_idx[ok])
                            vals.append(0.5 * g * sign[ok])
    n = len(dets)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    H.sum_duplicates()
    return dets, H


# ---------------------------------------------------------------- construction (b)

def _string_generators(L, n):
    """E_pq on one spin's string space (alpha-first order inside the string):
    a+_p a_q |str> with the sign (-1)^(electrons strictly between)."""
    strs = _strings(L, n)
    index = {s: k for k, s in enumerate(strs)}
    E = {}
    for p in range(L):
        for q in range(L):
            rr, cc, vv = [], [], []
            for k, s in enumerate(strs):
                if not (s >> q) & 1:
                    continue
                t = s & ~(1 << q)
                if (t >> p) & 1:
                    continue
                sign = (-1) ** bin(t & ((1 << p) - 1)).count("1")
                sign *= (-1) ** bin(s & ((1 << q) - 1)).count("1")
                u = t | (1 << p)
                rr.append(index[u])
                cc.append(k)
                vv.append(float(sign))
            E[(p, q)] = sp.csr_matrix((vv, (rr, cc)), shape=(len(strs), len(strs)))
    return strs, E


def build_h_strings(h, eri, na, nb):
    """Same Hamiltonian via spin-summed generators; returned over
    sector_determinants(L, na, nb) in the interleaved sign convention."""
    L = h.shape[0]
    astr, Ea = _string_generators(L, na)
    bstr, Eb = _string_generators(L, nb)
    Ia = sp.identity(len(astr), format="csr")
    Ib = sp.identity(len(bstr), format="csr")
    # determinant (a, b) = alpha creators then beta creators; beta acts after
    # an even or odd number of alpha electrons: the sign is (-1)^{N_alpha}
    # for a beta single excitation moving past all alpha creators twice -> +1.
    E = {}
    for p in range(L):
        for q in range(L):
            E[(p, q)] = (sp.kron(Ea[(p, q)], Ib) + sp.kron(Ia, Eb[(p, q)])).tocsr()
    n = len(astr) * len(bstr)
    H = sp.csr_matrix((n, n))
    for p in range(L):
        for q in range(L):
            F = sp.csr_matrix((n, n))
            for r in range(L):
                for s_ in range(L):
                    if eri[p, q, r, s_] != 0.0:
                        F = F + eri[p, q, r, s_] * E[(r, s_)]
            H = H + h[p, q] * E[(p, q)] + 0.5 * (E[(p, q)] @ F)
    for p in range(L):
        for s_ in range(L):
            c = sum(eri[p, q, q, s_] for q in range(L))
            H = H - 0.5 * c * E[(p, s_)]
    # carry to the interleaved ordering
    dets = sector_determinants(L, na, nb)
    perm = np.empty(n, dtype=np.int64)
    sign = np.empty(n)
    k = 0
    for a in astr:
        for b in bstr:
            d = 0
            for i in range(L):
                if (a >> i) & 1:
                    d |= 1 << (2 * i)
                if (b >> i) & 1:
                    d |= 1 << (2 * i + 1)
            perm[k] = np.searchsorted(dets, d)
            # moving beta creator of site i left past alpha creators of sites > i
            par = 0
            for i in range(L):
                if (b >> i) & 1:
                    par += bin(a >> (i + 1)).count("1")
            sign[k] = -1.0 if par % 2 else 1.0
            k += 1
    D = sp.diags(sign)
    Hs = (D @ H @ D).tocoo()
    out = sp.csr_matrix((Hs.data, (perm[Hs.row], perm[Hs.col])), shape=(n, n))
    out.sum_duplicates()
    return dets, out


def ground_energy(H, k=1):
    """Lowest eigenvalue(s) by dense diagonalization (small sectors only)."""
    w = np.linalg.eigvalsh(H.toarray())
    return w[:k] if k > 1 else float(w[0])
