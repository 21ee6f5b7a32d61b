"""Full two-site sweeps on the GPU (renormalization, Davidson, truncation
through the C ABI) against the oracle DMRG and full CI: sweep energies agree
within 1e-6 Eh."""
import numpy as np
import pytest

from gpu_helpers import say
from synthetic import make_integrals
from synthetic.mps import random_full_mps
from oracle.dmrg import OracleDMRG
from oracle.fci import build_h_interleaved, ground_energy

pytestmark = pytest.mark.gpu


# every precision must reproduce the oracle's sweeps within 1e-6 Eh: the split
# precisions iterate Davidson with split products and finish with float64 ones
@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-9, 1e-6), (2, 1e-9, 1e-6), (1, 1e-9, 1e-6)])
@pytest.mark.parametrize("L,na,nb,D,nsweeps", [(8, 4, 4, 64, 2), (10, 5, 5, 24, 2), (8, 5, 3, 16, 2)])
def test_gpu_sweeps_match_oracle(L, na, nb, D, nsweeps, precision, tol, bar):
    from paper_2412_04676_amd import bsdmrg as B
    from paper_2412_04676_amd import sweep as SW
    say(f"sweep L={L} ({na},{nb}) D={D} precision {precision}")
    h, eri = make_integrals(L)
    dims, T = random_full_mps(L, na, nb, D)
    ctx = B.bsdmrg_create(L, na, nb)
    B.bsdmrg_load_integrals(ctx, h, eri)
    SW.load_mps(ctx, T)
    gpu = [SW.sweep(ctx, L, D, seed=s, precision=precision, tol=tol) for s in range(nsweeps)]
    B.bsdmrg_destroy(ctx)
    ora = OracleDMRG(h, eri, na, nb, D)
    orl = [ora.sweep(D) for _ in range(nsweeps)]
    for sw in range(nsweeps):
        eg, eo = gpu[sw][-1][1], orl[sw][-1][1]
        say(f"  sweep {sw}: E gpu {eg:.10f} oracle {eo:.10f} diff {eg - eo:.2e}")
        assert abs(eg - eo) < bar
    if L <= 8:
        _, H = build_h_interleaved(h, eri, na, nb)
        E = ground_energy(H)
        assert gpu[-1][-1][1] >= E - 1e-9
        say(f"  gap to FCI {gpu[-1][-1][1] - E:.2e}")
