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
