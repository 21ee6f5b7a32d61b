"""CPU oracle (test infrastructure only).

A plain, slow, float64 implementation of what the HIP path computes, written
from the paper's problem statement: the ab initio Hamiltonian (Eq. 1), the MPS
ansatz (Eq. 2), the variational problem (Eq. 3), the two-site DMRG step
(Sec. II.B: preprocessing, Lanczos/Davidson diagonalization, SVD, renormalization)
and the serializer's contract (Sec. III.B.2: exact size prediction, independent
writers of disjoint intervals, identical object after deserialization; Sec.
III.B.3: self-contained segments that a reader places in any order).

Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import this package.  The product library never calls it and shares
no code with it; both sides take their inputs from the `synthetic` package.
"""
