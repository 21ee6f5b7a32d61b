"""Single-site fermionic operators and spin-orbital integrals.

Local basis of a spatial orbital (Eq. 2, local dimension 4):
    0 = |0>, 1 = a+_alpha|0>, 2 = a+_beta|0>, 3 = a+_alpha a+_beta|0>.
Spin-orbital p = 2 * site + sigma.  Spin-orbital integrals follow the reading
of Eq. 1 used throughout the oracle:
    t_pq   = h_{ij} delta(sigma_p, sigma_q)
    g_pqrs = (i_p i_s | i_q i_r) delta(sigma_p, sigma_s) delta(sigma_q, sigma_r)
so that H = sum t_pq a+_p a_q + 1/2 sum g_pqrs a+_p a+_q a_r a_s.
"""

import numpy as np

CD = (np.zeros((4, 4)), np.zeros((4, 4)))
CD[0][1, 0] = 1.0
CD[0][3, 2] = 1.0
CD[1][2, 0] = 1.0
CD[1][3, 1] = -1.0
ID4 = np.eye(4)
PARITY4 = np.diag([1.0, -1.0, -1.0, 1.0])
QSITE = ((0, 0), (1, 0), (0, 1), (1, 1))


def site_op(dagger, sigma):
    return CD[sigma] if dagger else CD[sigma].T


def spin_orbital_integrals(h, eri):
    L = h.shape[0]
    n = 2 * L
    t = np.zeros((n, n))
    for s in range(2):
        t[s::2, s::2] = h
    g = np.zeros((n, n, n, n))
    # g[p,q,r,s] = eri[i_p, i_s, i_q, i_r] for matching spins
    e = np.transpose(eri, (0, 2, 3, 1))  # e[a,b,c,d] = eri[a,d,b,c]
    for sp in range(2):
        for sq in range(2):
            g[sp::2, sq::2, sq::2, sp::2] = e
    return t, g
