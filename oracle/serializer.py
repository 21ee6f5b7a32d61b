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
