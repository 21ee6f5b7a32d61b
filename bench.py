"""Benchmark of the two-site DMRG hot path on one MI355X.

Workload (default): L=24 orbitals, N=24 electrons, S_z=0, bond dimension
D=512, seeded synthetic integrals and a seeded random MPS in mixed-canonical
form around the middle two-site position (sites 11, 12).  One step is one
effective-Hamiltonian product H.psi in float64 on the grouped-GEMM path, with
inputs resident in HBM.  Reported beside it: the serializer (pack of the left
environment block into one contiguous stream, GB/s), its offload to pinned host
memory on a side stream (GB/s), and the fraction of the offload hidden behind
back-to-back H.psi products.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
BF16_MFMA_PEAK_TFLOPS = 2516.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(L, na, nb, D, site):
    from paper_2412_04676_amd import bsdmrg as B
    from synthetic import make_integrals
    from synthetic.mps import random_mps, random_two_site_psi
    h, eri = make_integrals(L)
    dims, T = random_mps(L, na, nb, D, site)
    ctx = B.bsdmrg_create(L, na, nb)
    B.bsdmrg_load_integrals(ctx, h, eri)
    # right blocks beyond the product's right bond keep normal operators (the
    # smaller side); the block at site+2 switches to the complementary set
    B.bsdmrg_set_right_normal(ctx, site + 3)
    for n, t in enumerate(T):
        if t is not None:
            B.bsdmrg_set_site_tensor(ctx, n, t)
    # grow each environment one bond at a time and free the block behind it,
    # so that only the blocks the middle-site step reads stay on the device
    t0 = time.time()
    for b in range(1, site + 1):
        B.bsdmrg_build_env(ctx, B.LEFT, b)
        if b > 1:
            B.bsdmrg_drop_block(ctx, B.LEFT, b - 1)
    for b in range(L - 1, site + 1, -1):
        B.bsdmrg_build_env(ctx, B.RIGHT, b)
        if b < L - 1:
            B.bsdmrg_drop_block(ctx, B.RIGHT, b + 1)
    t_env = time.time() - t0
    psi = random_two_site_psi(dims[site], dims[site + 2], 1)
    return ctx, psi, dims, T, h, eri, t_env


def cpu_baseline(L, na, nb, D, site, useful_flops, budget_s=20.0):
    """The CPU oracle (plain numpy float64 block-sparse product, as it stands)
    timed on a bounded sample of the same middle-site workload: its environment
    blocks and enlarged operators are built once (untimed), then full products
    H.psi are applied back to back until the time budget is spent.  Throughput
    uses the same useful-flop count per product as the GPU figure."""
    from synthetic import make_integrals
    from synthetic.mps import random_mps, random_two_site_psi
    from oracle.siteops import spin_orbital_integrals
    from oracle.blocks import build_left_blocks, build_right_blocks
    from oracle.hpsi import BlockSparseHeff
    h, eri = make_integrals(L)
    t, g = spin_orbital_integrals(h, eri)
    dims, T = random_mps(L, na, nb, D, site)
    t0 = time.time()
    log("bench: cpu baseline: oracle left environment")
    lb = build_left_blocks(T, site, t, g)[site]
    log(f"bench: cpu baseline: oracle right environment ({time.time() - t0:.0f} s so far)")
    rb = build_right_blocks(T, site + 2, t, g, (na, nb))[site + 2]
    log(f"bench: cpu baseline: oracle enlarged operators ({time.time() - t0:.0f} s so far)")
    op = BlockSparseHeff(lb, rb, t, g, (na, nb))
    t_setup = time.time() - t0
    psi = random_two_site_psi(dims[site], dims[site + 2], 1)
    n = 0
    t0 = time.time()
    while True:
        op.apply(psi)
        n += 1
        log(f"bench: cpu baseline: {n} oracle products in {time.time() - t0:.1f} s")
        if time.time() - t0 > budget_s:
            break
    dt = time.time() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": useful_flops * n / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} full middle-site products H.psi of the oracle (numpy float64, L={L}, D={D}) in "
                      f"{dt:.1f} s after an untimed {t_setup:.0f} s environment build; throughput counts the "
                      "same useful flops per product as the GPU figure"}


def measured_traffic(kernel_label, workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration), or
    None when the summary covers another kernel or workload, or its source has
    changed since."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "*_traffic.txt")):
        kv = {}
        with open(path) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k] = v
        if not kernel_label.startswith(kv.get("kernel", "\0")) or kv.get("workload") != workload:
            continue
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), kv["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != kv["source_sha256_16"]:
                return None
        return int(kv["bytes_per_launch"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=24)
    ap.add_argument("--N", type=int, default=24)
    ap.add_argument("--D", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--ws-mb", type=int, default=0, help="H.psi workspace budget in MiB (0: library default)")
    ap.add_argument("--precision", type=int, default=0, help="0 fp64, 1 split-bf16 x3, 2 split-bf16 x6")
    ap.add_argument("--no-autotune", action="store_true", help="time the default schedules")
    ap.add_argument("--dav-iters", type=int, default=40, help="Davidson iteration cap of the site step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design "
                                   "note, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2412_04676_amd import bsdmrg as B

    L, N, D = args.L, args.N, args.D
    na, nb = (N + 1) // 2, N // 2
    site = L // 2 - 1
    torch.cuda.set_device(0)
    log(f"bench: building workload L={L} N={N} D={D} site={site}")
    ctx, psi, dims, T, h, eri, t_env = build_workload(L, na, nb, D, site)
    log(f"bench: environments built in {t_env:.1f} s")
    stream = torch.cuda.current_stream()
    B.bsdmrg_hpsi_prepare(ctx, site, B.FP64, args.ws_mb << 20, stream)
    info = B.bsdmrg_hpsi_info(ctx, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    y = torch.empty_like(x)
    log(f"bench: psi {lay[2]} elements, {info['channels']} channels, {info['segments']} K-segments, "
        f"{info['flops']:.3e} flop per product")

    shapes = {0: "<2, 2>", 1: "<1, 1>", 2: "<1, 2>", 3: "<2, 1>", 4: "<16>", 5: "<32>"}

    tuned = {}

    def time_precision(prec):
        # schedule chosen by the library's autotuner (untimed setup)
        if args.no_autotune:
            tuned[prec] = None
        else:
            best, dflt, ncand = B.bsdmrg_hpsi_autotune(ctx, site, prec, stream)
            tuned[prec] = {"candidates": ncand, "default_ms": dflt, "tuned_ms": best}
            log(f"bench: precision {prec}: autotune {ncand} schedules, default {dflt:.3f} ms -> {best:.3f} ms")
        for _ in range(args.warmup):
            B.bsdmrg_hpsi(ctx, site, x, y, prec, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            B.bsdmrg_hpsi(ctx, site, x, y, prec, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_ = e0.elapsed_time(e1) / args.steps
        out_ = y.clone()
        # dominant kernel: per-launch HIP events on the library's stream
        kinds = {}
        for _ in range(5):
            for k, t, f, nb in B.bsdmrg_hpsi_profile(ctx, site, x, y, prec, stream):
                a = kinds.setdefault(k, [0.0, 0.0, 0, 0.0])
                a[0] += t
                a[1] += f
                a[2] += 1
                a[3] += nb
        names = {0: "zero_fill_kernel", 1: "split_planes_kernel psi"}
        for ph in (1, 2):
            for c, sh in shapes.items():
                if c >= 4 and prec:
                    names[10 * ph + c] = f"wave_planes_kernel{sh[:-1]}, {3 * prec}, {2 - ph}> phase {ph}"
                elif c >= 4:
                    names[10 * ph + c] = f"wave_gemm_kernel{sh} phase {ph}"
                else:
                    names[10 * ph + c] = f"grouped_gemm_kernel{sh} phase {ph}"
        names[16], names[26] = "split_reduce_kernel phase 1", "split_reduce_kernel phase 2"
        dom = max(kinds, key=lambda k: kinds[k][0])
        per = {names[k]: v[0] / v[2] for k, v in sorted(kinds.items())}
        log(f"bench: precision {prec}: H.psi {ms_:.3f} ms, {info['flops'] / (ms_ * 1e-3) / 1e12:.2f} TFLOP/s; "
            + ", ".join(f"{n}: {t:.3f} ms" for n, t in per.items()))
        n_dom = kinds[dom][2]
        return (ms_, out_, names[dom], kinds[dom][0] / n_dom, kinds[dom][1] / n_dom, per, kinds[dom][3] / n_dom)

    res = {p: time_precision(p) for p in (B.FP64, B.BF16X3, B.BF16X6)}
    ref = res[B.FP64][1]
    errs = {p: float(torch.linalg.norm(res[p][1] - ref) / torch.linalg.norm(ref)) for p in res}
    # energy-scale error of each path on this vector, in hartree: |(H'-H)x|/|x|
    # bounds the Rayleigh-quotient change, x.(H'-H)x/|x|^2 is that change itself
    xn = float(torch.linalg.norm(x))
    de_bound = {p: float(torch.linalg.norm(res[p][1] - ref)) / xn for p in res}
    de_rq = {p: abs(float(torch.dot(x, res[p][1] - ref))) / xn ** 2 for p in res}
    log(f"bench: relative error vs fp64: x3 {errs[B.BF16X3]:.2e}, x6 {errs[B.BF16X6]:.2e}; "
        f"dE(Rayleigh) x3 {de_rq[B.BF16X3]:.2e} Eh, x6 {de_rq[B.BF16X6]:.2e} Eh")
    # the reported path: the fastest one within 1e-6 relative 2-norm error of the
    # float64 product whose energy (Rayleigh quotient) moves by at most 1e-6 Eh
    ok = [p for p in res if errs[p] <= 1e-6 and de_rq[p] <= 1e-6]
    chosen = min(ok, key=lambda p: res[p][0])
    ms, _, dname, t_dom, f_dom, per_launch, b_dom = res[chosen]
    tflops = info["flops"] / (ms * 1e-3) / 1e12
    # algorithmic flops of the dominant kernel: the split-bf16 products issue 3 or
    # 6 bf16 MFMA products per float64 multiply-add
    mult = {B.FP64: 1.0, B.BF16X3: 3.0, B.BF16X6: 6.0}[chosen]
    peak_f = FP64_MFMA_PEAK_TFLOPS if chosen == B.FP64 else BF16_MFMA_PEAK_TFLOPS
    ach_f = mult * f_dom / (t_dom * 1e-3) / 1e12
    ach_b = b_dom / (t_dom * 1e-3) / 1e9
    # the roof that bounds the kernel at its algorithmic intensity
    intensity = mult * f_dom / b_dom
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = measured_traffic(dname, f"L={L} N={N} D={D}")
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": ach_b, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_b / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma", "achieved": ach_f, "peak": peak_f, "unit": "TFLOP/s", "frac": ach_f / peak_f}
    roof.update({"traffic": traffic, "kernel": dname, "kernel_ms": t_dom, "kernel_useful_flops": f_dom,
                 "algorithmic_flops_per_useful_flop": mult, "algorithmic_bytes": b_dom,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "mfma_tflops": ach_f, "mfma_peak": peak_f, "mfma_frac": ach_f / peak_f,
                 "hbm_GBps": ach_b, "hbm_frac": ach_b / HBM_PEAK_GBS,
                 "traffic_GBps": traffic / (t_dom * 1e-3) / 1e9 if traffic else None})

    # serializer and offload of the left environment block
    nbytes = B.bsdmrg_serialized_size(ctx, B.LEFT, site)
    staging = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    pinned = torch.empty(nbytes // 8 + 64, dtype=torch.float64, pin_memory=True)
    side = torch.cuda.Stream()
    B.bsdmrg_pack(ctx, B.LEFT, site, staging, staging.numel() * 8, stream)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.time()
    for _ in range(reps):
        B.bsdmrg_pack(ctx, B.LEFT, site, staging, staging.numel() * 8, stream)
    torch.cuda.synchronize()
    t_pack = (time.time() - t0) / reps
    pack_gbs = 2 * nbytes / t_pack / 1e9
    # offload alone
    t0 = time.time()
    B.bsdmrg_offload(ctx, B.LEFT, site, staging, pinned, nbytes, 0, stream, side)
    B.bsdmrg_offload_wait(ctx, B.LEFT, site)
    torch.cuda.synchronize()
    t_io = time.time() - t0
    t0 = time.time()
    side.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(side):
        ev0.record(side)
        pinned.copy_(staging, non_blocking=True)
        ev1.record(side)
    torch.cuda.synchronize()
    d2h_gbs = nbytes / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    # compute alone and compute with the offload in flight
    nrep = max(4, int(np.ceil(t_io / (ms * 1e-3))) + 2)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(nrep):
        B.bsdmrg_hpsi(ctx, site, x, y, chosen, stream)
    torch.cuda.synchronize()
    t_comp = time.time() - t0
    t0 = time.time()
    B.bsdmrg_offload(ctx, B.LEFT, site, staging, pinned, nbytes, 0, stream, side)
    for _ in range(nrep):
        B.bsdmrg_hpsi(ctx, site, x, y, chosen, stream)
    B.bsdmrg_offload_wait(ctx, B.LEFT, site)
    torch.cuda.synchronize()
    t_both = time.time() - t0
    hidden = 1.0 - max(0.0, t_both - t_comp) / t_io
    hidden = min(1.0, max(0.0, hidden))
    log(f"bench: pack {nbytes / 1e6:.1f} MB in {t_pack * 1e3:.2f} ms ({pack_gbs:.0f} GB/s HBM), "
        f"D2H {d2h_gbs:.1f} GB/s, offload alone {t_io * 1e3:.1f} ms, hidden {hidden * 100:.1f}%")

    # one full middle-site step: Davidson (H.psi products + float64 vector work),
    # truncation to D, renormalization of the enlarged left block
    torch.cuda.synchronize()
    xs = x.clone()
    t0 = time.time()
    e_dav, it_dav, r_dav, _ = B.bsdmrg_davidson(ctx, site, xs, max_iter=args.dav_iters, tol=1e-8, precond=1,
                                                precision=chosen, stream=stream)
    torch.cuda.synchronize()
    t_dav = time.time() - t0
    t0 = time.time()
    err_tr, kept, _ = B.bsdmrg_truncate(ctx, site, xs, D, 0, stream)
    torch.cuda.synchronize()
    t_tr = time.time() - t0
    t0 = time.time()
    B.bsdmrg_build_env(ctx, B.LEFT, site + 1, stream)
    torch.cuda.synchronize()
    t_ren = time.time() - t0
    log(f"bench: site step: Davidson {it_dav} it {t_dav * 1e3:.1f} ms (E {e_dav:.8f}, |r| {r_dav:.1e}), "
        f"truncation {t_tr * 1e3:.1f} ms (kept {kept}, err {err_tr:.2e}), renormalization {t_ren * 1e3:.1f} ms")

    out = {
        "metric": "H·ψ TFLOP/s split-BF16 vs FP64 at ΔE≤1e-6 Eh; serializer+offload GB/s, % hidden",
        "value": tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if chosen == B.FP64 else "bf16",   # MFMA operand type; config.precision_path names the scheme
        "data": "synthetic",
        "config": {"workload": f"middle-site two-site H.psi, L={L} N={N} S_z={(na - nb) / 2} D={D} "
                               "(synthetic integrals, random mixed-canonical MPS)",
                   "site": site, "psi_elements": int(lay[2]), "channels": info["channels"],
                   "k_segments": info["segments"], "flops_per_step": info["flops"],
                   "precision_path": {0: "fp64", 1: "bf16x3", 2: "bf16x6"}[chosen], "env_build_s": t_env},
        "precisions": {name: {"ms": res[p][0], "tflops": info["flops"] / (res[p][0] * 1e-3) / 1e12,
                              "rel_err_vs_fp64": errs[p], "dHx_over_x_Eh": de_bound[p],
                              "d_rayleigh_Eh": de_rq[p], "per_launch_ms": res[p][5]}
                       for name, p in (("fp64", B.FP64), ("bf16x3", B.BF16X3), ("bf16x6", B.BF16X6))},
        "speedup_bf16x6_vs_fp64": res[B.FP64][0] / res[B.BF16X6][0],
        "autotune": {name: tuned[p] for name, p in (("fp64", B.FP64), ("bf16x3", B.BF16X3), ("bf16x6", B.BF16X6))},
        "roofline": roof,
        "site_step": {"davidson_precision": {0: "fp64", 1: "bf16x3", 2: "bf16x6"}[chosen],
                      "davidson_iters": it_dav, "davidson_ms": t_dav * 1e3, "energy": e_dav,
                      "residual": r_dav, "truncate_ms": t_tr * 1e3, "kept": kept, "trunc_err": err_tr,
                      "renormalize_ms": t_ren * 1e3},
        "serializer": {"bytes": nbytes, "pack_ms": t_pack * 1e3, "pack_hbm_GBps": pack_gbs,
                       "d2h_GBps": d2h_gbs, "offload_ms": t_io * 1e3, "hidden_frac": hidden},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        try:
            out["cpu_baseline"] = cpu_baseline(L, na, nb, D, site, info["flops"], args.cpu_budget)
        except Exception as e:  # report, never hide
            out["cpu_baseline"] = {"error": repr(e)}
    B.bsdmrg_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
