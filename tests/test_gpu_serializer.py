"""Serializer on the GPU: the packed stream is byte-identical to the reference
serializer's, unpacking restores the object bit for bit (padding untouched),
corrupted streams are rejected without writing, and a block offloaded to pinned
host memory and prefetched back gives bit-identical products."""
import numpy as np
import pytest

from gpu_helpers import build_system, psi_for, say
from oracle import serializer as S

pytestmark = pytest.mark.gpu


def random_families(rng, nfam=5, pad=3):
    fams_dev, fams_ref, keep = [], [], []
    import torch
    for k in range(nfam):
        nb = int(rng.integers(0, 7))
        rows = rng.integers(0, 40, nb).astype(np.int32)
        cols = rng.integers(0, 40, nb).astype(np.int32)
        if nb > 2:
            rows[1], cols[1] = 300, 129   # a block large enough for row slices
        ld = (cols + rng.integers(0, pad, nb)).astype(np.int32)
        off = np.zeros(nb, dtype=np.int64)
        o = 0
        for b in range(nb):
            off[b] = o
            o += int(rows[b]) * int(ld[b]) + 2 * int(rng.integers(0, 2))
        stride = o + 8
        nl = int(rng.integers(0, 4))
        mem = rng.normal(size=max(1, nl * stride))
        if mem.size > 5:
            mem[:5] = [-0.0, np.inf, -np.inf, 5e-324, np.nan]
        dev = torch.from_numpy(mem).cuda()
        keep.append(dev)
        data = np.zeros((nl, int(np.sum(rows.astype(np.int64) * cols))))
        for l in range(nl):
            pos = 0
            for b in range(nb):
                blk = mem[l * stride + off[b]: l * stride + off[b] + rows[b] * ld[b]].reshape(rows[b], ld[b])[:, :cols[b]]
                data[l, pos:pos + blk.size] = blk.ravel()
                pos += blk.size
        q = [[int(rng.integers(-3, 4)), int(rng.integers(-3, 4))] for _ in range(nb)]
        fams_dev.append({"tag": 1000 + k, "dq": (k % 3 - 1, 1), "n_layers": nl, "block_q": q, "rows": rows,
                         "cols": cols, "ld": ld, "elem_offset": off, "layer_stride": stride, "data": dev})
        fams_ref.append({"tag": 1000 + k, "dq": (k % 3 - 1, 1),
                         "blocks": [((q[b][0], q[b][1]), int(rows[b]), int(cols[b])) for b in range(nb)],
                         "data": data})
    return fams_dev, fams_ref, keep


def test_pack_matches_reference_bytes_and_round_trips():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    rng = np.random.default_rng(7)
    fams, ref, keep = random_families(rng)
    n = B.bsdmrg_serialized_size_desc(fams)
    expect = S.serialize(ref)
    assert n == len(expect)
    say(f"pack {n} bytes")
    dst = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
    B.bsdmrg_pack_desc(fams, dst, dst.numel() * 8)
    got = dst.cpu().numpy().view(np.uint8)[:n].tobytes()
    assert got == expect
    # round trip into fresh memory filled with a sentinel
    fresh = []
    for f in fams:
        x = torch.full_like(f["data"], 12345.0)
        g = dict(f)
        g["data"] = x
        fresh.append(g)
    B.bsdmrg_unpack_desc(fresh, dst, n)
    torch.cuda.synchronize()
    for f, g in zip(fams, fresh):
        a = f["data"].cpu().numpy().view(np.uint64)
        b = g["data"].cpu().numpy()
        mask = np.zeros(a.size, dtype=bool)
        for l in range(f["n_layers"]):
            for r, c, ld, o in zip(f["rows"], f["cols"], f["ld"], f["elem_offset"]):
                for i in range(r):
                    s0 = l * f["layer_stride"] + o + i * ld
                    mask[s0:s0 + c] = True
        assert np.array_equal(a[mask], b.view(np.uint64)[mask])
        assert np.all(b[~mask] == 12345.0)


def test_corrupted_stream_is_rejected_without_writes():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    rng = np.random.default_rng(8)
    fams, ref, keep = random_families(rng, nfam=3)
    n = B.bsdmrg_serialized_size_desc(fams)
    dst = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
    B.bsdmrg_pack_desc(fams, dst, dst.numel() * 8)
    raw = dst.cpu().numpy().view(np.uint8).copy()
    for where in (0, 12, 64 + 8, 64 * 4 + 8):
        bad = raw.copy()
        bad[where] ^= 0x55
        tb = torch.from_numpy(bad.view(np.float64)).cuda()
        tgt = []
        for f in fams:
            g = dict(f)
            g["data"] = torch.full_like(f["data"], 7.0)
            tgt.append(g)
        with pytest.raises(B.BsdmrgError) as e:
            B.bsdmrg_unpack_desc(tgt, tb, n)
        assert e.value.code == B.ECORRUPT
        for g in tgt:
            assert torch.all(g["data"] == 7.0)
    with pytest.raises(B.BsdmrgError):
        B.bsdmrg_unpack_desc(fams, dst, n - 256)


def test_block_offload_release_prefetch_bit_identical():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("offload/prefetch")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    psi = psi_for(dims, site, 2)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi, lay)).cuda()
    y0 = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y0)
    torch.cuda.synchronize()
    for side, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        n = B.bsdmrg_serialized_size(ctx, side, bond)
        staging = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        pinned = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
        comp, sidestream = torch.cuda.current_stream(), torch.cuda.Stream()
        assert B.bsdmrg_block_bytes(ctx, side, bond) > 0
        B.bsdmrg_offload(ctx, side, bond, staging, pinned, n, 1, comp, sidestream)
        B.bsdmrg_offload_wait(ctx, side, bond)
        assert B.bsdmrg_block_bytes(ctx, side, bond) == 0
        y = torch.empty_like(x)
        with pytest.raises(B.BsdmrgError) as e:
            B.bsdmrg_hpsi(ctx, site, x, y)
        assert e.value.code in (B.EBUSY, B.ESTATE)
        staging.zero_()
        B.bsdmrg_prefetch(ctx, side, bond, pinned, staging, n, comp, sidestream)
        torch.cuda.synchronize()
    y1 = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    B.bsdmrg_destroy(ctx)


def test_davidson_bit_identical_with_offload_in_flight():
    """Hiding the offload must not change results: a float64 Davidson run while
    both environment blocks are packed and copied to pinned host memory on a
    side stream gives the same energy and vector, bit for bit, as a run
    without the offload."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("davidson with offload in flight")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x0 = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 8), lay)).cuda()
    comp = torch.cuda.current_stream()
    xa = x0.clone()
    ea, ita, ra, _ = B.bsdmrg_davidson(ctx, site, xa, max_iter=30, tol=1e-10, stream=comp)
    bufs = []
    sidestream = torch.cuda.Stream()
    for side, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        n = B.bsdmrg_serialized_size(ctx, side, bond)
        staging = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        pinned = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
        bufs.append((staging, pinned))
        B.bsdmrg_offload(ctx, side, bond, staging, pinned, n, 0, comp, sidestream)
    xb = x0.clone()
    eb, itb, rb, _ = B.bsdmrg_davidson(ctx, site, xb, max_iter=30, tol=1e-10, stream=comp)
    for side, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        B.bsdmrg_offload_wait(ctx, side, bond)
    torch.cuda.synchronize()
    say(f"  E {ea:.12f} vs {eb:.12f}, iterations {ita} vs {itb}")
    assert ea == eb and ita == itb and ra == rb
    assert torch.equal(xa, xb)
    B.bsdmrg_destroy(ctx)


def _offloaded_copies(B, ctx, site, comp, side):
    """Pinned host copies of both environment blocks (offload without release)."""
    import torch
    out = {}
    for sd, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        n = B.bsdmrg_serialized_size(ctx, sd, bond)
        st = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        pin = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
        B.bsdmrg_offload(ctx, sd, bond, st, pin, n, 0, comp, side)
        B.bsdmrg_offload_wait(ctx, sd, bond)
        out[(sd, bond)] = (n, pin)
    return out


def test_release_and_prefetch_keep_product_plans():
    """Offload with release returns the block's physical memory; the prefetch
    restores it at the same addresses, so the prepared product is replayed as
    it was (no new Tables step) and gives the same result bit for bit."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("release + prefetch keep plans")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 3), lay)).cuda()
    y0 = torch.empty_like(x)
    for prec in (B.FP64, B.BF16X6):
        B.bsdmrg_hpsi(ctx, site, x, y0, prec)
    B.bsdmrg_hpsi(ctx, site, x, y0)
    torch.cuda.synchronize()
    tables = B.bsdmrg_stats(ctx)["seconds"]["Tables"]
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    copies = _offloaded_copies(B, ctx, site, comp, side)
    for (sd, bond), (n, pin) in copies.items():
        st = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        B.bsdmrg_offload(ctx, sd, bond, st, pin, n, 1, comp, side)
        B.bsdmrg_offload_wait(ctx, sd, bond)
        assert B.bsdmrg_block_bytes(ctx, sd, bond) == 0
        B.bsdmrg_prefetch(ctx, sd, bond, pin, st, n, comp, side)
        B.bsdmrg_prefetch_wait(ctx, sd, bond)
    y1 = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    st = B.bsdmrg_stats(ctx)
    say(f"  Tables {tables:.3f} s -> {st['seconds']['Tables']:.3f} s; IO {st['seconds']['IO']:.3f} s")
    assert st["seconds"]["Tables"] == tables
    B.bsdmrg_destroy(ctx)


def test_prefetches_sharing_one_staging_buffer():
    """Two prefetches through one staging buffer with products queued between
    them: the second copy waits for the first unpack, so both blocks come back
    intact and every product equals the reference bit for bit."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("two prefetches, one staging buffer")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 4), lay)).cuda()
    ref = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, ref)
    torch.cuda.synchronize()
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    copies = _offloaded_copies(B, ctx, site, comp, side)
    nmax = max(n for n, _ in copies.values())
    staging = torch.empty(nmax // 8 + 32, dtype=torch.float64, device="cuda")
    (nl, pin_l), (nr, pin_r) = copies[(B.LEFT, site)], copies[(B.RIGHT, site + 2)]
    outs = [torch.empty_like(x) for _ in range(3)]
    for rep in range(2):
        # the left block's memory is returned, so only its unpack restores it
        B.bsdmrg_offload(ctx, B.LEFT, site, staging, pin_l, nl, 1, comp, side)
        B.bsdmrg_offload_wait(ctx, B.LEFT, site)
        B.bsdmrg_prefetch(ctx, B.LEFT, site, pin_l, staging, nl, comp, side)
        B.bsdmrg_hpsi(ctx, site, x, outs[0], B.FP64, comp)
        # the right block's stream goes through the same staging buffer
        B.bsdmrg_prefetch(ctx, B.RIGHT, site + 2, pin_r, staging, nr, comp, side)
        B.bsdmrg_hpsi(ctx, site, x, outs[1], B.FP64, comp)
        torch.cuda.synchronize()
        for o in outs[:2]:
            assert torch.equal(o, ref), rep
    B.bsdmrg_destroy(ctx)


def test_forced_side_delay_is_counted_as_exposed_io():
    """With a host delay queued before each side-stream copy, the blocking
    waits (fetching) see it, the statistics count it as exposed IO, and the
    data still arrive intact."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 8, 4, 4, 40, 3
    say("forced side delay")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 5), lay)).cuda()
    ref = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, ref)
    torch.cuda.synchronize()
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    n = B.bsdmrg_serialized_size(ctx, B.LEFT, site)
    st = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
    pin = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
    B.bsdmrg_stats(ctx, reset=True)
    B.bsdmrg_set_side_delay(ctx, 300.0)
    B.bsdmrg_offload(ctx, B.LEFT, site, st, pin, n, 1, comp, side)
    w1 = B.bsdmrg_offload_wait(ctx, B.LEFT, site)
    B.bsdmrg_prefetch(ctx, B.LEFT, site, pin, st, n, comp, side)
    w2 = B.bsdmrg_prefetch_wait(ctx, B.LEFT, site)
    B.bsdmrg_set_side_delay(ctx, 0.0)
    y = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y)
    torch.cuda.synchronize()
    s = B.bsdmrg_stats(ctx)
    say(f"  waited {w1:.3f} s and {w2:.3f} s, exposed IO {s['io_exposed_s']:.3f} s")
    assert w1 >= 0.25 and w2 >= 0.25
    assert s["io_exposed_s"] >= w1 + w2 - 1e-9
    assert torch.equal(y, ref)
    B.bsdmrg_destroy(ctx)


def _split_segments(raw):
    """Segments of a segmented stream: (header, payload incl. padding) byte arrays."""
    out, at = [], 0
    while at < len(raw):
        payload = int(np.frombuffer(raw[at + 32:at + 40].tobytes(), dtype=np.uint64)[0])
        ln = 256 + (payload + 255) // 256 * 256
        out.append(raw[at:at + ln].copy())
        at += ln
    return out


def test_segments_round_trip_in_any_order():
    """Synchronous small-buffer segments (Fig. 4b) are self-contained: packed
    through a small staging area, shuffled, and read back into the released
    block, they restore it exactly; a corrupted, missing or repeated segment
    is rejected before anything is written."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("segments in any order")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    lay = B.bsdmrg_psi_layout(ctx, site)
    x = torch.from_numpy(B.psi_to_flat(psi_for(dims, site, 7), lay)).cuda()
    ref = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, ref)
    torch.cuda.synchronize()
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    rng = np.random.default_rng(1)
    for sd, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        staging_bytes = None
        for sb in (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22):
            try:
                total, nseg = B.bsdmrg_segments_size(ctx, sd, bond, sb)
                staging_bytes = sb
                break
            except B.BsdmrgError as e:
                assert e.code == B.ENOMEM
        assert staging_bytes is not None
        say(f"  side {sd}: {nseg} segments, {total} bytes through a {staging_bytes} byte staging area")
        assert nseg >= 2
        staging = torch.empty(staging_bytes // 8, dtype=torch.float64, device="cuda")
        pin = torch.empty(total // 8, dtype=torch.float64, pin_memory=True)
        written, k = B.bsdmrg_pack_segments(ctx, sd, bond, staging, staging_bytes, pin, total, comp, side)
        assert written == total and k == nseg
        segs = _split_segments(pin.numpy().view(np.uint8))
        assert len(segs) == nseg
        order = rng.permutation(nseg)
        shuffled = torch.from_numpy(np.concatenate([segs[i] for i in order]).view(np.float64)).pin_memory()
        # release the block: only the segments can restore it
        n = B.bsdmrg_serialized_size(ctx, sd, bond)
        st1 = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        pin1 = torch.empty(n // 8 + 32, dtype=torch.float64, pin_memory=True)
        B.bsdmrg_offload(ctx, sd, bond, st1, pin1, n, 1, comp, side)
        B.bsdmrg_offload_wait(ctx, sd, bond)
        bad_sets = []
        b1 = np.concatenate([segs[i] for i in order]).copy()
        b1[40] ^= 0x01                      # fingerprint byte of the first segment
        bad_sets.append(b1)
        bad_sets.append(np.concatenate([segs[i] for i in order[1:]]))           # one missing
        bad_sets.append(np.concatenate([segs[i] for i in order] + [segs[order[0]]]))   # one repeated
        for bad in bad_sets:
            tb = torch.from_numpy(bad.view(np.float64)).pin_memory()
            with pytest.raises(B.BsdmrgError) as e:
                B.bsdmrg_unpack_segments(ctx, sd, bond, tb, tb.numel() * 8, staging, staging_bytes, comp, side)
            assert e.value.code == B.ECORRUPT
            assert B.bsdmrg_block_bytes(ctx, sd, bond) == 0
        B.bsdmrg_unpack_segments(ctx, sd, bond, shuffled, total, staging, staging_bytes, comp, side)
        assert B.bsdmrg_block_bytes(ctx, sd, bond) > 0
    y = torch.empty_like(x)
    B.bsdmrg_hpsi(ctx, site, x, y)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    B.bsdmrg_destroy(ctx)


def test_segments_match_the_oracle_bytes():
    """The segments a block packs through a small staging area are, byte for
    byte, the reference serializer's segments of the same block (headers,
    skeleton fingerprints, layer runs, zero padding), read from the block's
    one-stream form, at two staging sizes."""
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("segments vs oracle bytes")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    comp, side = torch.cuda.current_stream(), torch.cuda.Stream()
    for sd, bond in ((B.LEFT, site), (B.RIGHT, site + 2)):
        n = B.bsdmrg_serialized_size(ctx, sd, bond)
        dst = torch.empty(n // 8 + 32, dtype=torch.float64, device="cuda")
        B.bsdmrg_pack(ctx, sd, bond, dst, dst.numel() * 8)
        torch.cuda.synchronize()
        fams = S.deserialize(dst.cpu().numpy().view(np.uint8)[:n].tobytes())
        need = max(S.layer_elems(f) * 8 for f in fams if f["data"].shape[0])
        smallest = 2 * ((need + 255) // 256 * 256)
        for staging_bytes in (smallest, 4 * smallest):
            expect = b"".join(S.segments(fams, staging_bytes))
            total, nseg = B.bsdmrg_segments_size(ctx, sd, bond, staging_bytes)
            say(f"  side {sd} staging {staging_bytes}: {nseg} segments, {total} bytes")
            assert total == len(expect)
            assert nseg == len(S.segment_runs(fams, staging_bytes))
            staging = torch.empty(staging_bytes // 8, dtype=torch.float64, device="cuda")
            pin = torch.full((total // 8,), 7.0, dtype=torch.float64, pin_memory=True)
            written, k = B.bsdmrg_pack_segments(ctx, sd, bond, staging, staging_bytes, pin, total, comp, side)
            assert written == total and k == nseg
            assert pin.numpy().view(np.uint8).tobytes() == expect
    B.bsdmrg_destroy(ctx)


def test_pack_is_independent_of_the_workgroup_count():
    import torch
    from paper_2412_04676_amd import bsdmrg as B
    L, na, nb, D, site = 10, 5, 5, 60, 4
    say("pack vs workgroup count")
    ctx, h, eri, dims, T = build_system(L, na, nb, D, site)
    n = B.bsdmrg_serialized_size(ctx, B.LEFT, site)
    outs = []
    try:
        for wg in (0, 1, 7, 1024):
            B.bsdmrg_set_copy_workgroups(wg)
            dst = torch.full((n // 8 + 32,), float(wg), dtype=torch.float64, device="cuda")
            B.bsdmrg_pack(ctx, B.LEFT, site, dst, dst.numel() * 8)
            outs.append(dst[: n // 8].clone())
            B.bsdmrg_unpack(ctx, B.LEFT, site, dst, n)
    finally:
        B.bsdmrg_set_copy_workgroups(0)
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o.view(torch.int64), outs[0].view(torch.int64))
    B.bsdmrg_destroy(ctx)
