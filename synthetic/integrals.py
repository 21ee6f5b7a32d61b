"""Seeded synthetic one- and two-electron integrals.

Shapes follow an ab initio active space: h_pq is an L x L symmetric matrix and
(pq|rs) is an L^4 tensor in chemists' order with 8-fold permutational symmetry,
built as a sum of 2L products of symmetric "Cholesky-like" vectors, so that it
is positive semidefinite as a (pq),(rs) matrix.  Draw order:
  A ~ N(0, 0.5^2) (L x L); h = (A + A^T)/2 - diag(linspace(2.0, 0.1, L))
  B ~ N(0, 0.3^2) (2L x L x L); L^k = triu(B_k) + triu(B_k, 1)^T
  (pq|rs) = sum_k L^k_pq L^k_rs
"""

import numpy as np


def integral_seed(L):
    """Seed used for the integrals of an L-orbital system."""
    return 2412 + L


def make_integrals(L, seed=None):
    """Return (h, eri) as float64 arrays of shapes (L, L) and (L, L, L, L)."""
    if seed is None:
        seed = integral_seed(L)
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, 0.5, (L, L))
    h = (a + a.T) / 2.0 + np.diag(-np.linspace(2.0, 0.1, L))
    b = rng.normal(0.0, 0.3, (2 * L, L, L))
    lk = np.triu(b) + np.transpose(np.triu(b, 1), (0, 2, 1))
    eri = np.einsum("kpq,krs->pqrs", lk, lk)
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)
