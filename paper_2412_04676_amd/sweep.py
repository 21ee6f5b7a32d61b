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


class IOQueue:
    """Load/save queue of a sweep (Sec. III.B.4): blocks behind the sweep front
    are offloaded to pinned host memory and their device memory released, and
    blocks the sweep reaches two steps later are prefetched, on a side stream,
    so the copies run while Davidson works.  The blocking waits (fetching) are
    the library's; this class only decides what moves when."""

    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        self.side = torch.cuda.Stream()
        self.host = {}           # (side, bond) -> (pinned tensor, bytes)
        self.pending = []        # offloads whose copy may still run
        self.stage_out = None    # device staging of offloads
        self.stage_in = None     # device staging of prefetches
        self.offloaded = set()

    def _staging(self, which, nbytes):
        import torch
        cur = getattr(self, which)
        if cur is None or cur.numel() * 8 < nbytes:
            cur = torch.empty((nbytes + 7) // 8 + 32, dtype=torch.float64, device="cuda")
            setattr(self, which, cur)
        return cur

    def offload(self, side, bond):
        import torch
        if (side, bond) in self.offloaded or bond <= 0 or bond >= self.ctx_L:
            return
        try:
            n = B.bsdmrg_serialized_size(self.ctx, side, bond)
        except B.BsdmrgError:
            return   # not built
        pin, cap = self.host.get((side, bond), (None, 0))
        if pin is None or cap < n:
            pin = torch.empty((n + 7) // 8 + 32, dtype=torch.float64, pin_memory=True)
            self.host[(side, bond)] = (pin, pin.numel() * 8)
        st = self._staging("stage_out", n)
        B.bsdmrg_offload(self.ctx, side, bond, st, pin, n, 1, torch.cuda.current_stream(), self.side)
        self.pending.append((side, bond, n))
        self.offloaded.add((side, bond))

    def settle(self):
        """Wait for the offloads issued earlier (their memory is released)."""
        for side, bond, n in self.pending:
            B.bsdmrg_offload_wait(self.ctx, side, bond)
        self.pending = []

    def prefetch(self, side, bond):
        import torch
        if (side, bond) not in self.offloaded:
            return
        if any(p[0] == side and p[1] == bond for p in self.pending):
            self.settle()
        try:
            n = B.bsdmrg_serialized_size(self.ctx, side, bond)
        except B.BsdmrgError:
            self.offloaded.discard((side, bond))   # the block was dropped as stale
            return
        pin, _ = self.host[(side, bond)]
        st = self._staging("stage_in", n)
        B.bsdmrg_prefetch(self.ctx, side, bond, pin, st, n, torch.cuda.current_stream(), self.side)
        self.offloaded.discard((side, bond))


class Sweeper:
    """Runs sweeps and keeps the start vector between steps (and sweeps)."""

    def __init__(self, ctx, L, precision=B.FP64, tol=1e-9, max_iter=300, precond=1, stvec=True, offload=False):
        self.ctx, self.L = ctx, L
        self.precision, self.tol, self.max_iter, self.precond = precision, tol, max_iter, precond
        self.stvec = stvec
        self.guess = None      # device vector in the layout of self.guess_site
        self.guess_site = None
        self.io = IOQueue(ctx) if offload else None
        if self.io:
            self.io.ctx_L = L

    def _start_vector(self, i, n, seed):
        import torch
        if self.guess is not None and self.guess_site == i and self.guess.numel() == n \
                and float(torch.linalg.norm(self.guess)) > 1e-12:
            return self.guess
        return torch.from_numpy(np.random.default_rng(seed).normal(size=n)).cuda()

    def step(self, i, direction, D, seed, next_pos=None):
        import torch
        ctx = self.ctx
        if self.io:
            # the blocks of this position must be back before anything reads them
            self.io.prefetch(B.LEFT, i)
            self.io.prefetch(B.RIGHT, i + 2)
        B.bsdmrg_build_env(ctx, B.LEFT, i)
        B.bsdmrg_build_env(ctx, B.RIGHT, i + 2)
        if self.io:
            # two steps ahead: the copy runs during this step's Davidson
            ahead = (B.RIGHT, i + 4) if direction == 0 else (B.LEFT, i - 2)
            self.io.prefetch(*ahead)
        _, _, ne = B.bsdmrg_psi_layout(ctx, i)
        x = self._start_vector(i, ne, seed)
        e, it, r, _ = B.bsdmrg_davidson(ctx, i, x, tol=self.tol, precision=self.precision,
                                        max_iter=self.max_iter, precond=self.precond)
        if self.io:
            self.io.settle()   # offloads of the previous step: copies done, memory released
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
        if self.io:
            # behind the front: the block the next step no longer reads
            if direction == 0 and i >= 1:
                self.io.offload(B.LEFT, i)
            elif direction == 1 and i + 2 < self.L:
                self.io.offload(B.RIGHT, i + 2)
        return e, err, kept, it

    def sweep(self, D, seed=0):
        """One sweep; returns [(position, energy, truncation error, kept, iterations)]."""
        pos = positions(self.L)
        log = []
        for n, (i, direction) in enumerate(pos):
            nxt = pos[n + 1][0] if n + 1 < len(pos) else pos[0][0]
            e, err, kept, it = self.step(i, direction, D, seed * 1000 + 500 * direction + i, nxt)
            log.append((i, e, err, kept, it))
        if self.io:
            self.io.settle()
        return log


def sweep(ctx, L, D, seed=0, precision=B.FP64, tol=1e-9, stvec=False):
    """One sweep with its own Sweeper (a fresh random start vector at the first
    step); returns [(position, energy, truncation error, kept, iterations)]."""
    return Sweeper(ctx, L, precision, tol, stvec=stvec).sweep(D, seed)
