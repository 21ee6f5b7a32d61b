"""Parity at the L=24, N=24, S_z=0, D=512 middle-site product, with the right
environment grown with normal operators and switched at site+2: the whole
product against the CPU oracle's (written by tests/golden/make_config1_hpsi.py,
relative 2-norm error <= 1e-10 in float64, <= 1e-6 for split-bf16 x6), its
norm, Rayleigh quotient and sampled elements, plus properties that hold at any
size (symmetry of H_eff)."""
import json
import os

import numpy as np
import pytest

from gpu_helpers import build_system, psi_for, say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def config1():
    from paper_2412_04676_amd import bsdmrg as B
    import torch
    gold = json.load(open(os.path.join(HERE, "golden", "config1_hpsi_samples.json")))
    L, na, nb, D, site = gold["L"], gold["n_alpha"], gold["n_beta"], gold["D"], gold["site"]
    say(f"config 1 full size: L={L} D={D} site={site}")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site, normal_right=True)
    lay = B.bsdmrg_psi_layout(ctx, site)
    psi = psi_for(dims, site, gold["psi_seed"])
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    yield B, ctx, site, lay, x, gold
    B.bsdmrg_destroy(ctx)


def test_config1_sampled_outputs_match_oracle(config1):
    import torch
    B, ctx, site, lay, x, gold = config1
    y = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y)
    torch.cuda.synchronize()
    out = B.flat_to_psi(y.cpu().numpy(), lay)
    norm = float(torch.linalg.norm(y))
    rq = float(torch.dot(x, y))
    say(f"  |H psi| gpu {norm:.12f} oracle {gold['norm']:.12f}; <psi|H psi> gpu {rq:.12f} oracle {gold['rayleigh']:.12f}")
    assert abs(norm - gold["norm"]) <= 1e-10 * gold["norm"]
    assert abs(rq - gold["rayleigh"]) <= 1e-10 * gold["norm"]
    for s in gold["samples"]:
        v = out[(tuple(s["ql"]), s["s1"], s["s2"])][s["i"], s["j"]]
        assert abs(v - s["value"]) <= 1e-10 * gold["norm"], s


@pytest.mark.parametrize("precision,bar", [(0, 1e-10), (2, 1e-6)])
def test_config1_full_product_matches_oracle(config1, precision, bar):
    import torch
    B, ctx, site, lay, x, gold = config1
    y = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y, precision)
    torch.cuda.synchronize()
    out = B.flat_to_psi(y.cpu().numpy(), lay)
    got = np.concatenate([out[k].ravel() for k in sorted(out)])
    ref = np.load(os.path.join(HERE, "golden", "config1_hpsi_full.npy"))
    assert got.shape == ref.shape
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    say(f"  precision {precision}: full-vector relative error {e:.3e}")
    assert e <= bar


def test_config1_heff_symmetric(config1):
    import torch
    B, ctx, site, lay, x, gold = config1
    g = torch.Generator(device="cuda").manual_seed(3)
    a = torch.randn(x.shape, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(x.shape, dtype=torch.float64, device="cuda", generator=g)
    ha, hb = torch.empty_like(a), torch.empty_like(b)
    B.bsdmrg_hpsi(ctx, site, a, ha)
    B.bsdmrg_hpsi(ctx, site, b, hb)
    torch.cuda.synchronize()
    l, r = float(torch.dot(a, hb)), float(torch.dot(ha, b))
    assert abs(l - r) <= 1e-12 * float(torch.linalg.norm(a) * torch.linalg.norm(hb))


def test_config1_split_bf16_x6_within_bar(config1):
    import torch
    B, ctx, site, lay, x, gold = config1
    y64, y6, y3 = (torch.empty_like(x) for _ in range(3))
    B.bsdmrg_hpsi(ctx, site, x, y64, B.FP64)
    B.bsdmrg_hpsi(ctx, site, x, y6, B.BF16X6)
    B.bsdmrg_hpsi(ctx, site, x, y3, B.BF16X3)
    torch.cuda.synchronize()
    e6 = float(torch.linalg.norm(y6 - y64) / torch.linalg.norm(y64))
    e3 = float(torch.linalg.norm(y3 - y64) / torch.linalg.norm(y64))
    say(f"  split-bf16 relative error x6 {e6:.2e} x3 {e3:.2e}")
    assert e6 <= 1e-6
    assert e3 <= 1e-4
