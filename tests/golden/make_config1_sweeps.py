"""Writes config1_sweeps.json: the CPU oracle's two-site DMRG (Sec. II.A-B)
on L=24 orbitals, N=24 electrons, S_z=0 (seeded synthetic integrals), from the
seeded random MPS of bond dimension 128, four full sweeps with the bond
dimension ramped 128, 256, 512, 512.  For every sweep it records the energy of
the last step (the sweep energy), every step's energy and the summed
truncation error.  Calls only oracle/ and the shared input generators; takes
about an hour on eight cores.  Run from the repository root:
    python tests/golden/make_config1_sweeps.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import make_integrals  # noqa: E402
from oracle.dmrg import OracleDMRG  # noqa: E402

L, NA, NB, D_INIT, SCHEDULE = 24, 12, 12, 128, (128, 256, 512, 512)


def main():
    h, eri = make_integrals(L)
    dmrg = OracleDMRG(h, eri, NA, NB, D_INIT)
    sweeps = []
    t0 = time.time()
    for n, D in enumerate(SCHEDULE):
        log = dmrg.sweep(D, seed=n)
        sweeps.append({"D": D, "energy": log[-1][1], "step_energies": [e for _, e, _ in log],
                       "trunc_err_sum": sum(err for _, _, err in log)})
        print(f"sweep {n} D={D}: E {log[-1][1]:.12f} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_sweeps.json"), "w") as f:
        json.dump({"L": L, "n_alpha": NA, "n_beta": NB, "D_init": D_INIT, "schedule": list(SCHEDULE),
                   "sweeps": sweeps}, f, indent=0)


if __name__ == "__main__":
    main()
