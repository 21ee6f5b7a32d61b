"""Shared helpers of the GPU tests: build a system through the C ABI from the
seeded synthetic inputs, and move two-site wave functions in and out."""
import sys

import numpy as np

from synthetic import make_integrals
from synthetic.mps import random_mps, random_two_site_psi


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def build_system(L, na, nb, D, site, build=True, normal_right=False):
    """normal_right: right blocks beyond site+2 keep normal operators and the
    block at site+2 switches to the complementary set (as bench.py builds)."""
    from paper_2412_04676_amd import bsdmrg as B
    h, eri = make_integrals(L)
    dims, T = random_mps(L, na, nb, D, site)
    ctx = B.bsdmrg_create(L, na, nb)
    B.bsdmrg_load_integrals(ctx, h, eri)
    if normal_right:
        B.bsdmrg_set_right_normal(ctx, site + 3)
    for n, t in enumerate(T):
        if t is not None:
            B.bsdmrg_set_site_tensor(ctx, n, t)
    if build:
        B.bsdmrg_build_env(ctx, B.LEFT, site)
        B.bsdmrg_build_env(ctx, B.RIGHT, site + 2)
    return ctx, h, eri, dims, T


def build_system_front_only(L, na, nb, D, site):
    """Environments grown one bond at a time, freeing the block behind, with
    normal right blocks switched at site+2 (what bench.py does for large
    workloads): only the blocks the middle-site product reads stay."""
    from paper_2412_04676_amd import bsdmrg as B
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site, build=False, normal_right=True)
    for b in range(1, site + 1):
        B.bsdmrg_build_env(ctx, B.LEFT, b)
        if b > 1:
            B.bsdmrg_drop_block(ctx, B.LEFT, b - 1)
        if b % 8 == 0:
            say(f"  left block {b} built")
    for b in range(L - 1, site + 1, -1):
        B.bsdmrg_build_env(ctx, B.RIGHT, b)
        if b < L - 1:
            B.bsdmrg_drop_block(ctx, B.RIGHT, b + 1)
        if b % 8 == 0:
            say(f"  right block {b} built")
    return ctx, h, eri, dims, T


def hpsi_gpu(ctx, site, psi):
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    y = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y)
    torch.cuda.synchronize()
    return B.flat_to_psi(y.cpu().numpy(), lay), lay


def rel(a, b):
    keys = sorted(b)
    x = np.concatenate([np.ravel(a[k]) for k in keys])
    y = np.concatenate([np.ravel(b[k]) for k in keys])
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def psi_for(dims, site, seed):
    return random_two_site_psi(dims[site], dims[site + 2], seed)


def split_energy_check(ctx, site, x, iters, stream):
    """Float64 Davidson and the two-stage BF16X6 and BF16X3 Davidson runs from
    the same start vector with the same iteration cap, and the energy shift of
    one split product on the float64 Davidson vector (the Rayleigh quotient
    change).  BF16X6 must reach the float64 energy within 1e-6 Eh and shift it
    by at most 1e-6 Eh; the BF16X3 figures are returned for the record (the
    runs are not converged, so their energies follow different trajectories)."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    x = x / torch.linalg.norm(x)
    res = {}
    vec = None
    for p in (B.FP64, B.BF16X6, B.BF16X3):
        xs = x.clone()
        e, it, r, _ = B.bsdmrg_davidson(ctx, site, xs, max_iter=iters, tol=1e-8, precond=1, precision=p,
                                        stream=stream)
        torch.cuda.synchronize()
        res[p] = e
        if p == B.FP64:
            vec = xs
    y64 = torch.empty_like(vec)
    B.bsdmrg_hpsi(ctx, site, vec, y64, B.FP64, stream)
    shifts = {}
    for p in (B.BF16X6, B.BF16X3):
        y = torch.empty_like(vec)
        B.bsdmrg_hpsi(ctx, site, vec, y, p, stream)
        torch.cuda.synchronize()
        shifts[p] = abs(float(torch.dot(vec, y - y64))) / float(torch.dot(vec, vec))
    say(f"  Davidson {iters} it: E fp64 {res[B.FP64]:.10f}, bf16x6 dE {res[B.BF16X6] - res[B.FP64]:.2e}, "
        f"bf16x3 dE {res[B.BF16X3] - res[B.FP64]:.2e} Eh; product shift on the fp64 vector bf16x6 "
        f"{shifts[B.BF16X6]:.2e}, bf16x3 {shifts[B.BF16X3]:.2e} Eh")
    assert abs(res[B.BF16X6] - res[B.FP64]) <= 1e-6
    assert shifts[B.BF16X6] <= 1e-6
    return res, shifts
