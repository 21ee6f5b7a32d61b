"""Full two-site sweeps on the GPU (renormalization, Davidson, truncation and
the start vector of the next step, all through the C ABI) against the oracle
DMRG and full CI: sweep energies agree within 1e-6 Eh."""
import json
import os
import time

import numpy as np
import pytest

from gpu_helpers import say
from synthetic import make_integrals
from synthetic.mps import random_full_mps
from oracle.dmrg import OracleDMRG
from oracle.fci import build_h_interleaved, ground_energy

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


# every precision must reproduce the oracle's sweeps within 1e-6 Eh: the split
# precisions iterate Davidson with split products and finish with float64 ones
@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-9, 1e-6), (2, 1e-9, 1e-6), (1, 1e-9, 1e-6)])
@pytest.mark.parametrize("L,na,nb,D,nsweeps", [(8, 4, 4, 64, 2), (10, 5, 5, 24, 2), (8, 5, 3, 16, 2),
                                               (10, 7, 6, 24, 2)])
def test_gpu_sweeps_match_oracle(L, na, nb, D, nsweeps, precision, tol, bar):
    from paper_2412_04676_amd import bsdmrg as B
    from paper_2412_04676_amd import sweep as SW
    say(f"sweep L={L} ({na},{nb}) D={D} precision {precision}")
    h, eri = make_integrals(L)
    dims, T = random_full_mps(L, na, nb, D)
    ctx = B.bsdmrg_create(L, na, nb)
    B.bsdmrg_load_integrals(ctx, h, eri)
    SW.load_mps(ctx, T)
    sw = SW.Sweeper(ctx, L, precision, tol)
    gpu = [sw.sweep(D, seed=s) for s in range(nsweeps)]
    B.bsdmrg_destroy(ctx)
    ora = OracleDMRG(h, eri, na, nb, D)
    orl = [ora.sweep(D) for _ in range(nsweeps)]
    for s in range(nsweeps):
        eg, eo = gpu[s][-1][1], orl[s][-1][1]
        say(f"  sweep {s}: E gpu {eg:.10f} oracle {eo:.10f} diff {eg - eo:.2e}")
        assert abs(eg - eo) < bar
    if L <= 8:
        _, H = build_h_interleaved(h, eri, na, nb)
        E = ground_energy(H)
        assert gpu[-1][-1][1] >= E - 1e-9
        say(f"  gap to FCI {gpu[-1][-1][1] - E:.2e}")


def test_start_vector_cuts_davidson_iterations():
    """Carrying the wave function into the next step (bsdmrg_next_guess)
    leaves the sweep energies unchanged and cuts the Davidson iterations."""
    from paper_2412_04676_amd import bsdmrg as B
    from paper_2412_04676_amd import sweep as SW
    L, na, nb, D = 10, 5, 5, 32
    h, eri = make_integrals(L)
    dims, T = random_full_mps(L, na, nb, D)
    res = {}
    for stvec in (False, True):
        ctx = B.bsdmrg_create(L, na, nb)
        B.bsdmrg_load_integrals(ctx, h, eri)
        SW.load_mps(ctx, T)
        sw = SW.Sweeper(ctx, L, B.FP64, 1e-9, stvec=stvec)
        logs = [sw.sweep(D, seed=s) for s in range(3)]
        res[stvec] = ([lg[-1][1] for lg in logs], sum(x[4] for x in logs[-1]))
        B.bsdmrg_destroy(ctx)
        say(f"  start vector {stvec}: energies {res[stvec][0]}, Davidson iterations in the last sweep "
            f"{res[stvec][1]}")
    for a, b in zip(res[False][0], res[True][0]):
        assert abs(a - b) < 1e-8
    assert res[True][1] < 0.6 * res[False][1]


@pytest.mark.timeout(1500)
@pytest.mark.parametrize("precision", [0, 2])
def test_config1_four_sweeps_match_oracle(precision):
    """L=24, N=24, S_z=0 from the seeded random MPS of bond dimension 128,
    four sweeps at D = 128, 256, 512, 512: every sweep energy within 1e-6 Eh of
    the CPU oracle's (tests/golden/make_config1_sweeps.py)."""
    from paper_2412_04676_amd import bsdmrg as B
    from paper_2412_04676_amd import sweep as SW
    path = os.path.join(HERE, "golden", "config1_sweeps.json")
    if not os.path.exists(path):
        pytest.skip("oracle sweep energies not generated")
    gold = json.load(open(path))
    L, na, nb = gold["L"], gold["n_alpha"], gold["n_beta"]
    h, eri = make_integrals(L)
    dims, T = random_full_mps(L, na, nb, gold["D_init"])
    ctx = B.bsdmrg_create(L, na, nb)
    B.bsdmrg_load_integrals(ctx, h, eri)
    SW.load_mps(ctx, T)
    sw = SW.Sweeper(ctx, L, precision, 1e-9)
    t0 = time.time()
    for n, ref in enumerate(gold["sweeps"]):
        log = sw.sweep(ref["D"], seed=n)
        e = log[-1][1]
        its = sum(x[4] for x in log)
        say(f"  sweep {n} D={ref['D']}: E gpu {e:.10f} oracle {ref['energy']:.10f} diff {e - ref['energy']:.2e}; "
            f"{its} Davidson iterations, {time.time() - t0:.0f} s")
        assert abs(e - ref["energy"]) < 1e-6
    st = B.bsdmrg_stats(ctx)
    say(f"  phases (s): " + ", ".join(f"{k} {v:.1f}" for k, v in st["seconds"].items()))
    B.bsdmrg_destroy(ctx)


def test_sweep_with_load_save_queue_is_unchanged():
    """Sweeps that offload the blocks behind the front (release) and prefetch
    the blocks ahead on a side stream (Sec. III.B.4) give the same energies as
    sweeps that keep every block on the device."""
    from paper_2412_04676_amd import bsdmrg as B
    from paper_2412_04676_amd import sweep as SW
    L, na, nb, D = 10, 5, 5, 32
    h, eri = make_integrals(L)
    dims, T = random_full_mps(L, na, nb, D)
    res = {}
    for offload in (False, True):
        ctx = B.bsdmrg_create(L, na, nb)
        B.bsdmrg_load_integrals(ctx, h, eri)
        SW.load_mps(ctx, T)
        sw = SW.Sweeper(ctx, L, B.FP64, 1e-9, offload=offload)
        res[offload] = [[x[1] for x in sw.sweep(D, seed=s)] for s in range(2)]
        st = B.bsdmrg_stats(ctx)
        say(f"  offload {offload}: last energy {res[offload][-1][-1]:.12f}; D2H {st['bytes_d2h']} B, "
            f"H2D {st['bytes_h2d']} B, exposed IO {st['io_exposed_s']:.4f} s")
        if offload:
            assert st["bytes_d2h"] > 0 and st["bytes_h2d"] > 0
        B.bsdmrg_destroy(ctx)
    for a, b in zip(res[False], res[True]):
        assert np.allclose(a, b, rtol=0, atol=1e-10)
