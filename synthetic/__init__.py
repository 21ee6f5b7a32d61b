"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and lays out input shapes: one- and
two-electron integrals shaped like an ab initio active space (Hamiltonian of
Eq. 1), bond sector dimensions for an MPS (Eq. 2) under U(1)xU(1) symmetry,
random isometric site tensors, and random two-site wave functions.  It holds
none of the method's arithmetic (no Hamiltonian application, no operator
renormalization, no eigensolver, no truncation, no serialization).

Conventions shared by every consumer:
  * spatial orbital i is MPS site i, left to right;
  * local basis of a site: s = 0 |0>, 1 |up>, 2 |down>, 3 |up down>, with
    quantum numbers q_s = (n_alpha, n_beta) in QS below;
  * a quantum number q is a pair (n_alpha, n_beta) of Python ints;
  * a site tensor is a dict {(q_left, s): ndarray (d_left[q_left], d_right[q_left + q_s])}
    in float64, row-major;
  * bond n's sector label counts the electrons on sites 0..n-1;
  * a two-site wave function is a dict {(q_left, s1, s2): ndarray (d_left[q_left], d_right[q_right])}
    with q_right = q_left + q_s1 + q_s2 (both bond labels).
"""

from .integrals import make_integrals, integral_seed
from .mps import (QS, bond_sector_dims, random_mps, random_two_site_psi,
                  two_site_blocks, mps_seed, psi_seed)

__all__ = ["make_integrals", "integral_seed", "QS", "bond_sector_dims",
           "random_mps", "random_two_site_psi", "two_site_blocks", "mps_seed",
           "psi_seed"]
