"""Two-site DMRG sweeps driven through the C ABI (Sec. II.A-B).

Only control flow lives here: every step (renormalization, Davidson,
truncation) is a library call running HIP kernels.  A sweep visits the
two-site positions left to right (truncating into left-canonical tensors) and
then right to left (truncating into right-canonical tensors).  Start vectors are
seeded Gaussian inputs passed in from `synthetic`.
"""
import numpy as np

from . import bsdmrg as B


def load_mps(ctx, tensors):
    for n, t in enumerate(tensors):
        if t is not None:
            B.bsdmrg_set_site_tensor(ctx, n, t)


def _step(ctx, L, i, D, direction, rng_seed, precision, tol, max_iter=300, precond=1):
    import torch
    B.bsdmrg_build_env(ctx, B.LEFT, i)
    B.bsdmrg_build_env(ctx, B.RIGHT, i + 2)
    meta, off, ne = B.bsdmrg_psi_layout(ctx, i)
    guess = np.random.default_rng(rng_seed).normal(size=ne)
    x = torch.from_numpy(guess).cuda()
    e, it, r, ritz = B.bsdmrg_davidson(ctx, i, x, tol=tol, precision=precision, max_iter=max_iter,
                                       precond=precond)
    err, kept, sv = B.bsdmrg_truncate(ctx, i, x, D, direction)
    return e, err, kept, it


def sweep(ctx, L, D, seed=0, precision=B.FP64, tol=1e-9):
    """One sweep; returns [(position, energy, truncation error, kept, iterations)]."""
    log = []
    for i in range(0, L - 2):
        e, err, kept, it = _step(ctx, L, i, D, 0, seed * 1000 + i, precision, tol)
        log.append((i, e, err, kept, it))
    for i in range(L - 2, 0, -1):
        e, err, kept, it = _step(ctx, L, i, D, 1, seed * 1000 + 500 + i, precision, tol)
        log.append((i, e, err, kept, it))
    return log
