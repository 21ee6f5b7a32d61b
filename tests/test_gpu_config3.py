"""The product at the L=76, N=113, S_z=1/2, D=4096 workload (the CAS(113,76)
shape: 119 bond sectors, blocks up to 178, 54M K-segments), built the way
bench.py builds it (environments grown front-only, normal right blocks
switched at the product's right bond).  The oracle cannot build environments
of this size, so the product is checked through properties that hold at any
size: H_eff is symmetric, the product is linear, split-bf16 x6 stays within
1e-6 and x3 within 1e-5 of float64, and sampled diagonal elements e_i^T H e_i
equal the library's H_eff diagonal.  The two-stage BF16X6 Davidson reaches the
float64 Davidson energy within 1e-6 Eh from the same start vector and cap."""
import numpy as np
import pytest

from gpu_helpers import build_system_front_only, say, split_energy_check

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def test_config3_hpsi_properties():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D = 76, 57, 56, 4096
    site = L // 2 - 1
    say(f"config3 L={L} N={na + nb} D={D} site={site}: building environments")
    ctx, h, eri, dims, T = build_system_front_only(L, na, nb, D, site)
    s = torch.cuda.current_stream()
    B.bsdmrg_hpsi_prepare(ctx, site, B.FP64, 0, s)
    info = B.bsdmrg_hpsi_info(ctx, site)
    say(f"  prepared: {info['channels']} channels, {info['segments']} segments")
    lay = B.bsdmrg_psi_layout(ctx, site)
    n = int(lay[2])
    g = torch.Generator(device="cpu").manual_seed(76)
    a = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    b = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    Ha, Hb, Hc = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    B.bsdmrg_hpsi(ctx, site, a, Ha, B.FP64, s)
    B.bsdmrg_hpsi(ctx, site, b, Hb, B.FP64, s)
    B.bsdmrg_hpsi(ctx, site, a + 2.0 * b, Hc, B.FP64, s)
    torch.cuda.synchronize()
    l, r = float(torch.dot(a, Hb)), float(torch.dot(Ha, b))
    say(f"  <a,Hb> {l:.12e} <Ha,b> {r:.12e}")
    assert abs(l - r) <= 1e-12 * float(torch.linalg.norm(Ha) * torch.linalg.norm(b))
    lin = float(torch.linalg.norm(Hc - Ha - 2.0 * Hb) / torch.linalg.norm(Hc))
    say(f"  linearity {lin:.2e}")
    assert lin < 1e-13
    for prec, bar in ((B.BF16X6, 1e-6), (B.BF16X3, 1e-5)):
        y = torch.empty_like(a)
        B.bsdmrg_hpsi(ctx, site, a, y, prec, s)
        torch.cuda.synchronize()
        e = float(torch.linalg.norm(y - Ha) / torch.linalg.norm(Ha))
        say(f"  precision {prec} rel err {e:.2e}")
        assert e < bar
    diag = torch.empty_like(a)
    B.bsdmrg_hpsi_diagonal(ctx, site, diag)
    rng = np.random.default_rng(11)
    e = torch.zeros_like(a)
    He = torch.empty_like(a)
    for i in rng.choice(n, size=2, replace=False):
        e.zero_()
        e[int(i)] = 1.0
        B.bsdmrg_hpsi(ctx, site, e, He, B.FP64, s)
        torch.cuda.synchronize()
        hi, di = float(He[int(i)]), float(diag[int(i)])
        assert abs(hi - di) <= 1e-10 * max(1.0, abs(hi)), (i, hi, di)
    split_energy_check(ctx, site, a, 4, s)
    B.bsdmrg_destroy(ctx)
