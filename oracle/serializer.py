"""Reference serializer for layered block-sparse operator families.

Follows the contract of Sec. III.B.2: the exact size of the byte stream is
known before anything is written, every part's byte interval is fixed in
advance (so independent writers can fill disjoint intervals of one buffer),
and deserialization restores an identical object.  Layered operators sharing
one block-sparse skeleton (Fig. 4a) are serialized as one family; the stream
is a header, a "pointer/grid structure" (family and block tables, Sec. III.A
strategy 2) and the payload.  The paper gives no byte format; this one is the
project's own, little-endian throughout:

  Header, 64 bytes
    0  magic        8 bytes  b"BSDMRG01"
    8  version      u32      1
   12  n_families   u32
   16  total_bytes  u64      whole stream
   24  payload      u64      sum of aligned family payloads
   32  meta_bytes   u64      offset of the first payload = align256(64 + 64 F + 32 sum n_blocks)
   40  reserved     24 zero bytes
  Family table, 64 bytes per family f, at 64 + 64 f
    0  tag          u64      caller-defined identifier
    8  dq           i32 x 2  (d n_alpha, d n_beta) of every layer
   16  n_layers     u32
   20  n_blocks     u32
   24  esize        u32      8 (float64)
   28  reserved     u32      0
   32  blocks_off   u64      byte offset of the family's block table
   40  payload_off  u64      byte offset of the family's payload (256-aligned)
   48  layer_elems  u64      sum over blocks of rows * cols
   56  reserved     u64      0
  Block tables, 32 bytes per block, families in order
    0  q_in         i32 x 2  input sector
    8  rows         i32
   12  cols         i32
   16  elem_off     u64      exclusive prefix sum of rows * cols within a layer
   24  reserved     u64      0
  Zero padding up to meta_bytes, then each family's payload: n_layers layers,
  each layer the blocks in table order, each block row-major and compact;
  zero padding to the next 256-byte boundary after every family.

The segmented form (self-contained packages for a small staging buffer) is
described and built at the end of this module.

A family here is a dict {"tag": int, "dq": (a, b), "blocks": [(q_in, rows,
cols)], "data": float64 array (n_layers, layer_elems)}.
"""

import struct

import numpy as np

MAGIC = b"BSDMRG01"
VERSION = 1
ALIGN = 256


def align(n, a=ALIGN):
    return (n + a - 1) // a * a


def layer_elems(fam):
    return sum(r * c for _, r, c in fam["blocks"])


def layout(families):
    """Byte offsets of every part; everything is known before writing."""
    nb = sum(len(f["blocks"]) for f in families)
    meta = align(64 + 64 * len(families) + 32 * nb)
    fam_entries = []
    boff = 64 + 64 * len(families)
    poff = meta
    for f in families:
        le = layer_elems(f)
        nl = f["data"].shape[0]
        fam_entries.append({"blocks_off": boff, "payload_off": poff, "layer_elems": le,
                            "n_layers": nl})
        boff += 32 * len(f["blocks"])
        poff += align(nl * le * 8)
    return meta, fam_entries, poff


def serialized_size(families):
    return layout(families)[2]


def serialize(families):
    meta, entries, total = layout(families)
    buf = bytearray(total)
    struct.pack_into("<8sIIQQQ", buf, 0, MAGIC, VERSION, len(families), total,
                     total - meta, meta)
    for k, (f, e) in enumerate(zip(families, entries)):
        struct.pack_into("<QiiIIIIQQQQ", buf, 64 + 64 * k, f["tag"], f["dq"][0], f["dq"][1],
                         e["n_layers"], len(f["blocks"]), 8, 0, e["blocks_off"],
                         e["payload_off"], e["layer_elems"], 0)
        off = 0
        for j, (q, r, c) in enumerate(f["blocks"]):
            struct.pack_into("<iiiiQQ", buf, e["blocks_off"] + 32 * j, q[0], q[1], r, c, off, 0)
            off += r * c
        data = np.ascontiguousarray(f["data"], dtype="<f8")
        assert data.shape == (e["n_layers"], e["layer_elems"])
        raw = data.tobytes()
        buf[e["payload_off"]:e["payload_off"] + len(raw)] = raw
    return bytes(buf)


class CorruptStream(ValueError):
    pass


def deserialize(stream):
    if len(stream) < 64:
        raise CorruptStream("short stream")
    magic, ver, nf, total, payload, meta = struct.unpack_from("<8sIIQQQ", stream, 0)
    if magic != MAGIC or ver != VERSION:
        raise CorruptStream("bad magic or version")
    if total != len(stream) or meta > total or 64 + 64 * nf > meta:
        raise CorruptStream("bad sizes")
    fams = []
    nblk_total = 0
    exp_boff = 64 + 64 * nf
    for k in range(nf):
        nblk_total += struct.unpack_from("<I", stream, 64 + 64 * k + 20)[0]
    if align(64 + 64 * nf + 32 * nblk_total) != meta:
        raise CorruptStream("bad metadata size")
    exp_poff = meta
    for k in range(nf):
        tag, da, db, nl, nblk, es, _, boff, poff, le, _ = struct.unpack_from(
            "<QiiIIIIQQQQ", stream, 64 + 64 * k)
        if es != 8 or boff != exp_boff or poff != exp_poff or poff + nl * le * 8 > total:
            raise CorruptStream("bad family entry")
        exp_boff += 32 * nblk
        exp_poff += align(nl * le * 8)
        blocks = []
        off = 0
        for j in range(nblk):
            qa, qb, r, c, eo, _ = struct.unpack_from("<iiiiQQ", stream, boff + 32 * j)
            if eo != off or r < 0 or c < 0:
                raise CorruptStream("bad block entry")
            blocks.append(((qa, qb), r, c))
            off += r * c
        if off != le:
            raise CorruptStream("layer size mismatch")
        data = np.frombuffer(stream, dtype="<f8", count=nl * le, offset=poff).reshape(nl, le).copy()
        fams.append({"tag": tag, "dq": (da, db), "blocks": blocks, "data": data})
    if exp_poff != total or payload != total - meta:
        raise CorruptStream("payload size mismatch")
    return fams


def family_from_ops(tag, ops):
    """Build a family from a list of BlockOps that share dq and block set."""
    dq = ops[0].dq
    qs = sorted(ops[0].blocks)
    blocks = [(q, ops[0].blocks[q].shape[0], ops[0].blocks[q].shape[1]) for q in qs]
    data = np.stack([np.concatenate([op.blocks[q].ravel() for q in qs]) for op in ops])
    return {"tag": tag, "dq": dq, "blocks": blocks, "data": data}


# ---------------------------------------------------------------- segments
# Self-contained packages (Sec. III.B.3) cut for a small staging buffer (Sec.
# III.A strategy 1, Fig. 4b).  The paper fixes the properties, not the bytes:
# every segment says by itself which family and which layers it holds, so a
# reader places segments in any order and can refuse a set that does not
# cover the block exactly once.  The project's format, little-endian:
#
#   Segment header, 256 bytes
#     0  magic        8 bytes  b"BSDSEG01"
#     8  owner        u64      the block's family tags with the low 20 bits
#                              (the family index) cleared
#    16  family       u32      index of the family in the block
#    20  n_families   u32
#    24  layer0       u32      first layer held
#    28  n_layers     u32      layers held (at least one)
#    32  payload      u64      n_layers * layer_elems * 8
#    40  print        u64      FNV-1a fingerprint of the family's skeleton
#    48  index        u64      position of the segment in the writer's order
#    56  zero bytes up to 256
#   Payload: the layers, each laid out as in the one-stream payload, then zero
#   bytes to the next 256-byte boundary.
#
# A family's layers are cut into runs of as many whole layers as fit half the
# staging area (half = floor(staging / 2) rounded down to 256 bytes); a family
# whose single layer exceeds that half cannot be segmented.  Families with no
# layers or no elements give no segment.  Writer order: families in order,
# runs in layer order.

SEG_MAGIC = b"BSDSEG01"
SEG_HEADER = 256
FNV_OFFSET = 14695981039346656037
FNV_PRIME = 1099511628211
INDEX_BITS = 20


def fnv1a64(data):
    """The 64-bit FNV-1a hash of a byte string (Fowler, Noll and Vo): start
    from the offset basis, and for every byte xor it in, then multiply by the
    FNV prime modulo 2^64."""
    h = FNV_OFFSET
    for byte in bytes(data):
        h ^= byte
        h = (h * FNV_PRIME) % (1 << 64)
    return h


def skeleton_print(fam):
    """Fingerprint of a family's block-sparse skeleton: FNV-1a over the 8-byte
    little-endian two's-complement encodings of dq (both charges), the layer
    count, and for every block in table order its input sector (both charges),
    rows and cols.  Layer values do not enter."""
    vals = [fam["dq"][0], fam["dq"][1], fam["data"].shape[0]]
    for q, r, c in fam["blocks"]:
        vals += [q[0], q[1], r, c]
    return fnv1a64(b"".join(struct.pack("<q", v) for v in vals))


def owner_of(families):
    return families[0]["tag"] & ~((1 << INDEX_BITS) - 1) if families else 0


def segment_half(staging_bytes):
    return staging_bytes // 2 // ALIGN * ALIGN


def segment_runs(families, staging_bytes):
    """(family, layer0, n_layers) of every segment, in writer order."""
    half = segment_half(staging_bytes)
    runs = []
    for f, fam in enumerate(families):
        nl, lb = fam["data"].shape[0], layer_elems(fam) * 8
        if nl == 0 or lb == 0:
            continue
        if lb > half:
            raise ValueError("half the staging area is smaller than one layer")
        per = max(1, half // lb)
        for l0 in range(0, nl, per):
            runs.append((f, l0, min(per, nl - l0)))
    return runs


def segments(families, staging_bytes):
    """The segments of a block, as one list of byte strings in writer order."""
    owner = owner_of(families)
    out = []
    for i, (f, l0, n) in enumerate(segment_runs(families, staging_bytes)):
        fam = families[f]
        raw = np.ascontiguousarray(fam["data"][l0:l0 + n], dtype="<f8").tobytes()
        head = bytearray(SEG_HEADER)
        struct.pack_into("<8sQIIIIQQQ", head, 0, SEG_MAGIC, owner, f, len(families), l0, n,
                         len(raw), skeleton_print(fam), i)
        out.append(bytes(head) + raw + bytes(align(len(raw)) - len(raw)))
    return out


def split_segments(stream):
    """Cut a concatenation of segments back into single segments, using only
    each header's payload size."""
    out, at = [], 0
    while at < len(stream):
        if len(stream) - at < SEG_HEADER:
            raise CorruptStream("short segment header")
        payload = struct.unpack_from("<Q", stream, at + 32)[0]
        n = SEG_HEADER + align(payload)
        if len(stream) - at < n:
            raise CorruptStream("short segment")
        out.append(bytes(stream[at:at + n]))
        at += n
    return out


def reassemble(stream, skeleton):
    """Read a concatenation of segments, in any order, into the layers of a
    block whose skeleton (families with tag, dq, blocks and the data shape) is
    known.  Every header is checked and every layer must be held exactly once
    before any layer is returned."""
    owner = owner_of(skeleton)
    data = [np.full(f["data"].shape, np.nan) for f in skeleton]
    seen = [np.zeros(f["data"].shape[0], dtype=int) for f in skeleton]
    parts = []
    for seg in split_segments(stream):
        magic, own, f, nf, l0, n, payload, fp, _ = struct.unpack_from("<8sQIIIIQQQ", seg, 0)
        if magic != SEG_MAGIC or own != owner or nf != len(skeleton) or f >= nf:
            raise CorruptStream("segment of another block")
        fam = skeleton[f]
        if fp != skeleton_print(fam) or n == 0 or l0 + n > fam["data"].shape[0] \
                or payload != n * layer_elems(fam) * 8:
            raise CorruptStream("segment does not fit the family")
        seen[f][l0:l0 + n] += 1
        parts.append((f, l0, n, seg))
    for f, fam in enumerate(skeleton):
        if layer_elems(fam) > 0 and np.any(seen[f] != 1):
            raise CorruptStream("layers missing or repeated")
    for f, l0, n, seg in parts:
        le = layer_elems(skeleton[f])
        data[f][l0:l0 + n] = np.frombuffer(seg, dtype="<f8", count=n * le,
                                           offset=SEG_HEADER).reshape(n, le)
    return data
