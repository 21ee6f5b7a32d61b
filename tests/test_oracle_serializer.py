"""Pins of the reference serializer against the paper's contract (Sec. III.B.2):
exact size before writing, disjoint independent intervals, identical object
after deserialization; and against the byte format written in its header."""
import struct

import numpy as np
import pytest

from oracle import serializer as S


def fam(tag, dq, shapes, nl, rng):
    blocks = [((i, i + 1), r, c) for i, (r, c) in enumerate(shapes)]
    le = sum(r * c for r, c in shapes)
    return {"tag": tag, "dq": dq, "blocks": blocks, "data": rng.normal(size=(nl, le))}


def test_tiny_family_bytes():
    f = {"tag": 7, "dq": (1, -1), "blocks": [((2, 3), 1, 2)],
         "data": np.array([[1.5, -2.0]])}
    b = S.serialize([f])
    assert len(b) == 512 == S.serialized_size([f])
    assert b[:8] == b"BSDMRG01"
    assert struct.unpack_from("<IIQQQ", b, 8) == (1, 1, 512, 256, 256)
    assert struct.unpack_from("<QiiII", b, 64) == (7, 1, -1, 1, 1)
    assert struct.unpack_from("<QQQ", b, 96) == (128, 256, 2)
    assert struct.unpack_from("<iiiiQ", b, 128) == (2, 3, 1, 2, 0)
    assert struct.unpack_from("<dd", b, 256) == (1.5, -2.0)
    assert b[272:] == bytes(240)
    assert b[160:256] == bytes(96)


def test_round_trip_bit_exact_special_values():
    rng = np.random.default_rng(0)
    f = fam(1, (0, 1), [(3, 5), (1, 1), (0, 4), (7, 2)], 3, rng)
    special = np.array([-0.0, np.inf, -np.inf, 5e-324, np.nan], dtype=np.float64)
    f["data"][0, :5] = special
    f["data"].view(np.uint64)[1, 0] = 0x7FF0000000000123  # NaN payload
    g = S.deserialize(S.serialize([f]))[0]
    assert g["tag"] == 1 and g["dq"] == (0, 1) and g["blocks"] == f["blocks"]
    assert np.array_equal(g["data"].view(np.uint64), f["data"].view(np.uint64))


def test_size_prediction_and_disjoint_intervals():
    rng = np.random.default_rng(1)
    fams = [fam(k, (k % 2, 0), [(rng.integers(0, 9), rng.integers(0, 9)) for _ in range(k + 1)],
                k % 3 + 1, rng) for k in range(6)]
    meta, entries, total = S.layout(fams)
    b = S.serialize(fams)
    assert len(b) == total == S.serialized_size(fams)
    # every family's interval is self-contained: writing it alone into the
    # predicted interval of an empty buffer reproduces the same bytes
    for f, e in zip(fams, entries):
        n = e["n_layers"] * e["layer_elems"] * 8
        assert b[e["payload_off"]:e["payload_off"] + n] == np.ascontiguousarray(f["data"]).tobytes()
        assert e["payload_off"] % 256 == 0
    out = S.deserialize(b)
    for f, g in zip(fams, out):
        assert np.array_equal(f["data"], g["data"])


def test_empty_and_zero_layer_families():
    rng = np.random.default_rng(2)
    fams = [fam(0, (0, 0), [], 2, rng), fam(1, (1, 0), [(2, 2)], 0, rng)]
    b = S.serialize(fams)
    out = S.deserialize(b)
    assert out[0]["data"].shape == (2, 0) and out[1]["data"].shape == (0, 4)


@pytest.mark.parametrize("where", [0, 8, 16, 64 + 40, 128 + 16])
def test_corruption_detected(where):
    rng = np.random.default_rng(3)
    b = bytearray(S.serialize([fam(5, (0, 0), [(2, 3), (4, 1)], 2, rng)]))
    b[where] ^= 0x5A
    with pytest.raises(S.CorruptStream):
        S.deserialize(bytes(b))


# ---------------------------------------------------------------- segments
# Pins of the segmented, self-contained form (Sec. III.A strategy 1 with the
# packages of Sec. III.B.3): the published FNV-1a test vectors, the byte
# layout of a worked example, exact cover of the one-stream payload (itself
# pinned above), and order-free reassembly that refuses bad sets.

@pytest.mark.parametrize("text,value", [(b"", 0xcbf29ce484222325), (b"a", 0xaf63dc4c8601ec8c),
                                        (b"foobar", 0x85944171f73967e8)])
def test_fnv1a64_published_vectors(text, value):
    assert S.fnv1a64(text) == value


def test_segment_tiny_bytes():
    data = np.arange(48, dtype=np.float64).reshape(3, 16) * 0.5 - 3.0
    f = {"tag": (5 << 20) | 3, "dq": (1, -1), "blocks": [((2, 3), 2, 8)], "data": data}
    # 128 bytes a layer; a 512-byte staging area has 256-byte halves: two layers each
    segs = S.segments([f], 512)
    assert [len(s) for s in segs] == [512, 512]
    for i, (s, l0, n) in enumerate(zip(segs, (0, 2), (2, 1))):
        assert s[:8] == b"BSDSEG01"
        assert struct.unpack_from("<QIIIIQ", s, 8) == (5 << 20, 0, 1, l0, n, 128 * n)
        assert struct.unpack_from("<Q", s, 48)[0] == i
        assert s[56:256] == bytes(200)
        assert np.array_equal(np.frombuffer(s, dtype="<f8", count=16 * n, offset=256),
                              data[l0:l0 + n].ravel())
        assert s[256 + 128 * n:] == bytes(256 - 128 * n)
    # the fingerprint spelled out: dq, layers, then sector, rows, cols of the block
    spelled = b"".join(v.to_bytes(8, "little", signed=True) for v in (1, -1, 3, 2, 3, 2, 8))
    assert struct.unpack_from("<Q", segs[0], 40)[0] == S.fnv1a64(spelled)
    # below 512 bytes the halves hold 0 bytes
    with pytest.raises(ValueError):
        S.segments([f], 511)


def test_fingerprint_sees_the_skeleton_only():
    rng = np.random.default_rng(3)
    f = fam(1, (0, 1), [(3, 5), (2, 2)], 4, rng)
    p = S.skeleton_print(f)
    g = dict(f, data=rng.normal(size=f["data"].shape))
    assert S.skeleton_print(g) == p
    variants = [dict(f, dq=(1, 0)), dict(f, data=f["data"][:3]),
                dict(f, blocks=[((0, 2), 3, 5), ((1, 2), 2, 2)]),
                dict(f, blocks=[((0, 1), 5, 3), ((1, 2), 2, 2)])]
    assert len({S.skeleton_print(v) for v in variants} | {p}) == 5


@pytest.mark.parametrize("staging", [512, 1024, 4096, 1 << 16])
def test_segments_cover_the_one_stream_payload(staging):
    rng = np.random.default_rng(staging)
    fams = [fam((9 << 20) | 0, (0, 1), [(3, 5), (1, 1), (0, 4)], 7, rng),
            fam((9 << 20) | 1, (1, 0), [(4, 4)], 0, rng),
            fam((9 << 20) | 2, (1, 1), [(2, 3), (5, 1)], 11, rng),
            fam((9 << 20) | 3, (0, 0), [(0, 3)], 5, rng)]
    stream = S.serialize(fams)
    _, entries, _ = S.layout(fams)
    segs = S.segments(fams, staging)
    half = staging // 2 // 256 * 256
    count = 0
    for k, (f, e) in enumerate(zip(fams, entries)):
        lb = e["layer_elems"] * 8
        mine = [s for s in segs if struct.unpack_from("<I", s, 16)[0] == k]
        if lb == 0 or e["n_layers"] == 0:
            assert not mine
            continue
        per = max(1, half // lb)
        assert len(mine) == -(-e["n_layers"] // per)
        count += len(mine)
        joined = b"".join(s[256:256 + struct.unpack_from("<Q", s, 32)[0]] for s in mine)
        assert joined == stream[e["payload_off"]:e["payload_off"] + e["n_layers"] * lb]
        assert all(struct.unpack_from("<Q", s, 32)[0] <= half for s in mine)
    assert count == len(segs)
    assert [struct.unpack_from("<Q", s, 48)[0] for s in segs] == list(range(len(segs)))


def test_layer_above_half_the_staging_area_is_refused():
    f = fam(0, (0, 0), [(8, 8)], 2, np.random.default_rng(0))    # 512-byte layers
    assert len(S.segments([f], 1024)) == 2
    with pytest.raises(ValueError):
        S.segments([f], 1023)


def test_reassembly_in_any_order_and_refusals():
    rng = np.random.default_rng(11)
    fams = [fam((4 << 20) | 0, (0, 1), [(3, 5), (2, 2)], 9, rng),
            fam((4 << 20) | 1, (1, 1), [(6, 1)], 6, rng)]
    segs = S.segments(fams, 512)
    assert len(segs) >= 4
    order = rng.permutation(len(segs))
    got = S.reassemble(b"".join(segs[i] for i in order), fams)
    for f, d in zip(fams, got):
        assert d.view(np.uint64).tobytes() == f["data"].view(np.uint64).tobytes()
    first = segs[order[0]]
    bad = []
    for at in (0, 8, 16, 24, 40):             # magic, owner, family, layer0, fingerprint
        b = bytearray(first)
        b[at] ^= 0x01
        bad.append(bytes(b) + b"".join(segs[i] for i in order[1:]))
    bad.append(b"".join(segs[i] for i in order[1:]))                         # one missing
    bad.append(b"".join(segs[i] for i in order) + first)                     # one repeated
    other = [dict(fams[0], blocks=[((0, 1), 5, 3), ((1, 2), 2, 2)]), fams[1]]
    bad.append(b"".join(S.segments(other, 512)))                             # another skeleton
    for b in bad:
        with pytest.raises(S.CorruptStream):
            S.reassemble(b, fams)
