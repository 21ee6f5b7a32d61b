"""Two-site DMRG sweeps driven through the C ABI (Sec. II.A-B).

Only control flow lives here: every step (renormalization, Davidson,
truncation, the start vector of the next step) is a library call running HIP
kernels.  A sweep visits the two-site positions left to right (truncating into
left-canonical tensors) and then right to left (truncating into
right-canonical tensors).  Each step's Davidson starts from the previous
step's wave function carried over by bsdmrg_next_guess (S V^T B or A U S);
the first step of a run starts from a seeded Gaussian vector passed in from
numpy.
"""
import numpy as np

from . import bsdmrg as B


def load_mps(ctx, tensors):
    for n, t in enumerate(tensors):
        if t is not None:
            B.bsdmrg_set_site_tensor(ctx, n, t)


def positions(L):
    """(position, direction) of one sweep: 0 left to right, 1 right to left."""
    return [(i, 0) for i in range(0, L - 2)] + [(i, 1) for i in range(L - 2, 0, -1)]


class Sweeper:
    """Runs sweeps and keeps the start vector between steps (and sweeps)."""

    def __init__(self, ctx, L, precision=B.FP64, tol=1e-9, max_iter=300, precond=1, stvec=True):
        self.ctx, self.L = ctx, L
        self.precision, self.tol, self.max_iter, self.precond = precision, tol, max_iter, precond
        self.stvec = stvec
        self.guess = None      # device vector in the layout of self.guess_site
        self.guess_site = None

    def _start_vector(self, i, n, seed):
        import torch
        if self.guess is not None and self.guess_site == i and self.guess.numel() == n \
                and float(torch.linalg.norm(self.guess)) > 1e-12:
            return self.guess
        return torch.from_numpy(np.random.default_rng(seed).normal(size=n)).cuda()

    def step(self, i, direction, D, seed, next_pos=None):
        import torch
        ctx = self.ctx
        B.bsdmrg_build_env(ctx, B.LEFT, i)
        B.bsdmrg_build_env(ctx, B.RIGHT, i + 2)
        _, _, ne = B.bsdmrg_psi_layout(ctx, i)
        x = self._start_vector(i, ne, seed)
        e, it, r, _ = B.bsdmrg_davidson(ctx, i, x, tol=self.tol, precision=self.precision,
                                        max_iter=self.max_iter, precond=self.precond)
        err, kept, _ = B.bsdmrg_truncate(ctx, i, x, D, direction)
        self.guess, self.guess_site = None, None
        if self.stvec and next_pos is not None:
            j = next_pos
            if j == (i + 1 if direction == 0 else i - 1):
                B.bsdmrg_build_env(ctx, B.LEFT, j)
                B.bsdmrg_build_env(ctx, B.RIGHT, j + 2)
                _, _, nn = B.bsdmrg_psi_layout(ctx, j)
                g = torch.empty(nn, dtype=torch.float64, device="cuda")
                B.bsdmrg_next_guess(ctx, i, direction, x, g)
                self.guess, self.guess_site = g, j
        return e, err, kept, it

    def sweep(self, D, seed=0):
        """One sweep; returns [(position, energy, truncation error, kept, iterations)]."""
        pos = positions(self.L)
        log = []
        for n, (i, direction) in enumerate(pos):
            nxt = pos[n + 1][0] if n + 1 < len(pos) else pos[0][0]
            e, err, kept, it = self.step(i, direction, D, seed * 1000 + 500 * direction + i, nxt)
            log.append((i, e, err, kept, it))
        return log


def sweep(ctx, L, D, seed=0, precision=B.FP64, tol=1e-9, stvec=False):
    """One sweep with its own Sweeper (a fresh random start vector at the first
    step); returns [(position, energy, truncation error, kept, iterations)]."""
    return Sweeper(ctx, L, precision, tol, stvec=stvec).sweep(D, seed)
