"""Writes config1_hpsi_samples.json: the CPU oracle's middle-site product H.psi
for L=24 orbitals, N=24 electrons, S_z=0, D=512 (seeded synthetic integrals,
seeded random mixed-canonical MPS around sites 11, 12, psi seed 1), reduced to
<psi|H psi>, |H psi| and 300 sampled elements, and config1_hpsi_full.npy: the
whole product, blocks in sorted (q_l, s1, s2) order, each row-major.  Calls
only oracle/ and the shared input generators.  Run from the repository root:
    python tests/golden/make_config1_hpsi.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synthetic import make_integrals  # noqa: E402
from synthetic.mps import random_mps, random_two_site_psi  # noqa: E402
from oracle.siteops import spin_orbital_integrals  # noqa: E402
from oracle.blocks import build_left_blocks, build_right_blocks  # noqa: E402
from oracle.hpsi import BlockSparseHeff  # noqa: E402

L, NA, NB, D, SITE, PSI_SEED = 24, 12, 12, 512, 11, 1


def main():
    h, eri = make_integrals(L)
    t, g = spin_orbital_integrals(h, eri)
    dims, T = random_mps(L, NA, NB, D, SITE)
    lb = build_left_blocks(T, SITE, t, g)[SITE]
    rb = build_right_blocks(T, SITE + 2, t, g, (NA, NB))[SITE + 2]
    op = BlockSparseHeff(lb, rb, t, g, (NA, NB))
    psi = random_two_site_psi(dims[SITE], dims[SITE + 2], PSI_SEED)
    out = op.apply(psi)
    keys = sorted(out)
    norm = float(np.sqrt(sum(np.sum(out[k] ** 2) for k in keys)))
    rq = float(sum(np.sum(out[k] * psi[k]) for k in keys))
    rng = np.random.default_rng(12345)
    samples = []
    for _ in range(300):
        k = keys[int(rng.integers(len(keys)))]
        i = int(rng.integers(out[k].shape[0]))
        j = int(rng.integers(out[k].shape[1]))
        samples.append({"ql": list(k[0]), "s1": k[1], "s2": k[2], "i": i, "j": j, "value": float(out[k][i, j])})
    here = os.path.dirname(os.path.abspath(__file__))
    np.save(os.path.join(here, "config1_hpsi_full.npy"), np.concatenate([out[k].ravel() for k in keys]))
    with open(os.path.join(here, "config1_hpsi_samples.json"), "w") as f:
        json.dump({"L": L, "n_alpha": NA, "n_beta": NB, "D": D, "site": SITE, "psi_seed": PSI_SEED,
                   "norm": norm, "rayleigh": rq, "samples": samples}, f, indent=0)


if __name__ == "__main__":
    main()
