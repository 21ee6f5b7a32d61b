"""Thin ctypes binding of libbsdmrg.so (include/bsdmrg.h).

Functions keep the C names; this module only marshals arguments (numpy arrays
for host data, torch tensors for device buffers and streams).  Every compute
step runs in the library's HIP kernels; if the shared library is missing the
import fails loudly.
"""

import ctypes
import os

import numpy as np
# torch first: it ships its own HIP runtime under the same soname as the one the
# library is linked against, and whichever loads first serves the process.
# Loading torch's keeps a single runtime that both torch and the library use.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbsdmrg.so")

OK, EINVAL, ESTATE, ESHAPE, ENOMEM, EHIP, EBUSY, ECORRUPT = range(8)
LEFT, RIGHT = 0, 1
FP64, BF16X3, BF16X6 = 0, 1, 2
QS = ((0, 0), (1, 0), (0, 1), (1, 1))


class BsdmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bsdmrg error {code}: {msg}")
        self.code = code


if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with paper_2412_04676_amd/build.py")
_lib = ctypes.CDLL(LIBPATH)

c_int, c_i32p, c_i64p, c_dp, c_vp, c_sz = (ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_size_t)


class FamilyDesc(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("dq", ctypes.c_int32 * 2), ("n_layers", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("block_q", c_vp), ("rows", c_vp), ("cols", c_vp),
                ("ld", c_vp), ("elem_offset", c_vp), ("layer_stride", ctypes.c_int64), ("data", c_vp)]


class Config(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_alpha", ctypes.c_int32), ("n_beta", ctypes.c_int32),
                ("D_max", ctypes.c_int32), ("hpsi_ws_bytes", ctypes.c_size_t),
                ("renorm_ws_bytes", ctypes.c_size_t), ("hbm_budget_bytes", ctypes.c_size_t),
                ("right_normal_from", ctypes.c_int32), ("flags", ctypes.c_int32)]


PHASES = ("Tables", "Diag_H", "Ren_l", "Ren_r", "SVD", "StVec", "IO")


class Stats(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double * 8), ("io_exposed_s", ctypes.c_double),
                ("hpsi_flops", ctypes.c_double), ("renorm_flops", ctypes.c_double),
                ("hpsi_calls", ctypes.c_int64), ("davidson_calls", ctypes.c_int64),
                ("davidson_iters", ctypes.c_int64), ("truncations", ctypes.c_int64),
                ("renorm_steps", ctypes.c_int64), ("bytes_packed", ctypes.c_int64),
                ("bytes_unpacked", ctypes.c_int64), ("bytes_d2h", ctypes.c_int64),
                ("bytes_h2d", ctypes.c_int64)]


class GemmDesc(ctypes.Structure):
    _fields_ = [("A", c_vp), ("B", c_vp), ("C", c_vp), ("M", ctypes.c_int32), ("N", ctypes.c_int32),
                ("K", ctypes.c_int32), ("transA", ctypes.c_int32), ("transB", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64),
                ("ldc", ctypes.c_int64), ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


_SIGS = {
    "bsdmrg_last_error": ([], ctypes.c_char_p),
    "bsdmrg_create": ([ctypes.POINTER(c_vp), c_vp], c_int),
    "bsdmrg_get_site_tensor": ([c_vp, c_int, ctypes.POINTER(c_int), c_i64p, c_vp, c_vp], c_int),
    "bsdmrg_renormalize": ([c_vp, c_int, c_int, c_vp], c_int),
    "bsdmrg_family_count": ([c_vp, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)], c_int),
    "bsdmrg_stats": ([c_vp, c_vp, c_int], c_int),
    "bsdmrg_destroy": ([c_vp], c_int),
    "bsdmrg_load_integrals": ([c_vp, c_vp, c_vp, ctypes.c_double], c_int),
    "bsdmrg_set_site_tensor": ([c_vp, c_int, c_int, c_vp, c_vp], c_int),
    "bsdmrg_build_env": ([c_vp, c_int, c_int, c_vp], c_int),
    "bsdmrg_set_renorm_workspace": ([c_vp, c_sz], c_int),
    "bsdmrg_drop_block": ([c_vp, c_int, c_int], c_int),
    "bsdmrg_set_right_normal": ([c_vp, c_int], c_int),
    "bsdmrg_renorm_stats": ([c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), c_i64p], c_int),
    "bsdmrg_psi_layout": ([c_vp, c_int, ctypes.POINTER(c_int), c_i64p, c_vp, c_vp], c_int),
    "bsdmrg_hpsi_prepare": ([c_vp, c_int, c_int, c_sz, c_vp], c_int),
    "bsdmrg_hpsi": ([c_vp, c_int, c_vp, c_vp, c_int, c_vp], c_int),
    "bsdmrg_hpsi_autotune": ([c_vp, c_int, c_int, c_vp, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int)], c_int),
    "bsdmrg_hpsi_schedule": ([c_vp, c_int, c_int, ctypes.c_double, c_int, c_int], c_int),
    "bsdmrg_hpsi_info": ([c_vp, c_int, c_int, ctypes.POINTER(ctypes.c_double), c_i64p, c_i64p,
                          c_i64p, c_i64p, c_i64p], c_int),
    "bsdmrg_hpsi_profile": ([c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_int, c_vp, c_vp, c_vp, c_vp,
                             ctypes.POINTER(c_int)], c_int),
    "bsdmrg_davidson": ([c_vp, c_int, c_vp, c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int),
                         ctypes.POINTER(ctypes.c_double), c_vp, c_int, c_vp], c_int),
    "bsdmrg_hpsi_diagonal": ([c_vp, c_int, c_vp, c_vp], c_int),
    "bsdmrg_next_guess": ([c_vp, c_int, c_int, c_vp, c_vp, c_vp], c_int),
    "bsdmrg_truncate": ([c_vp, c_int, c_vp, c_int, c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int),
                         c_vp, c_int, c_vp], c_int),
    "bsdmrg_get_block_op": ([c_vp, c_int, c_int, ctypes.c_char, c_int, c_int, ctypes.POINTER(c_int),
                             c_i64p, c_vp, c_vp], c_int),
    "bsdmrg_block_gemm": ([c_int, c_vp, c_int, c_vp], c_int),
    "bsdmrg_serialized_size_desc": ([c_int, c_vp, ctypes.POINTER(c_sz)], c_int),
    "bsdmrg_pack_desc": ([c_int, c_vp, c_vp, c_sz, c_vp], c_int),
    "bsdmrg_unpack_desc": ([c_int, c_vp, c_vp, c_sz, c_vp], c_int),
    "bsdmrg_serialized_size": ([c_vp, c_int, c_int, ctypes.POINTER(c_sz)], c_int),
    "bsdmrg_pack": ([c_vp, c_int, c_int, c_vp, c_sz, c_vp], c_int),
    "bsdmrg_unpack": ([c_vp, c_int, c_int, c_vp, c_sz, c_vp], c_int),
    "bsdmrg_offload": ([c_vp, c_int, c_int, c_vp, c_vp, c_sz, c_int, c_vp, c_vp], c_int),
    "bsdmrg_offload_wait": ([c_vp, c_int, c_int, ctypes.POINTER(ctypes.c_double)], c_int),
    "bsdmrg_prefetch": ([c_vp, c_int, c_int, c_vp, c_vp, c_sz, c_vp, c_vp], c_int),
    "bsdmrg_block_bytes": ([c_vp, c_int, c_int, ctypes.POINTER(c_sz)], c_int),
    "bsdmrg_prefetch_wait": ([c_vp, c_int, c_int, ctypes.POINTER(ctypes.c_double)], c_int),
    "bsdmrg_set_side_delay": ([c_vp, ctypes.c_double], c_int),
    "bsdmrg_set_hbm_budget": ([c_vp, c_sz, c_sz], c_int),
    "bsdmrg_segments_size": ([c_vp, c_int, c_int, c_sz, ctypes.POINTER(c_sz), ctypes.POINTER(c_int)], c_int),
    "bsdmrg_pack_segments": ([c_vp, c_int, c_int, c_vp, c_sz, c_vp, c_sz, ctypes.POINTER(c_sz),
                              ctypes.POINTER(c_int), c_vp, c_vp], c_int),
    "bsdmrg_unpack_segments": ([c_vp, c_int, c_int, c_vp, c_sz, c_vp, c_sz, c_vp, c_vp], c_int),
    "bsdmrg_set_copy_workgroups": ([c_int], c_int),
    "bsdmrg_set_split_policy": ([c_vp, c_int], c_int),
    "bsdmrg_pack_desc_noalloc": ([c_int, c_vp, c_vp, c_sz, c_vp], c_int),
    "bsdmrg_noalloc_scratch_bytes": ([ctypes.POINTER(c_sz)], c_int),
    "bsdmrg_hpsi_streamed": ([c_vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_sz), ctypes.POINTER(c_int)], c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def _check(rc):
    if rc != OK:
        raise BsdmrgError(rc, _lib.bsdmrg_last_error().decode())


def _ptr(x):
    """Device pointer of a torch tensor, host pointer of a numpy array, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


def _stream(s):
    if s is None:
        return None
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def bsdmrg_last_error():
    return _lib.bsdmrg_last_error().decode()


def bsdmrg_create(L, n_alpha, n_beta, D_max=0, hpsi_ws_bytes=0, renorm_ws_bytes=0, hbm_budget_bytes=0,
                  right_normal_from=0, flags=0):
    cfg = Config(L, n_alpha, n_beta, D_max, hpsi_ws_bytes, renorm_ws_bytes, hbm_budget_bytes,
                 right_normal_from, flags)
    h = c_vp()
    _check(_lib.bsdmrg_create(ctypes.byref(h), ctypes.byref(cfg)))
    return h


def bsdmrg_get_site_tensor(ctx, site):
    """Returns {(q_left, s): block} of a site tensor (host copies)."""
    n = c_int()
    ne = ctypes.c_int64()
    _check(_lib.bsdmrg_get_site_tensor(ctx, site, ctypes.byref(n), ctypes.byref(ne), None, None))
    meta = np.zeros((n.value, 5), dtype=np.int32)
    data = np.zeros(max(1, ne.value))
    _check(_lib.bsdmrg_get_site_tensor(ctx, site, ctypes.byref(n), ctypes.byref(ne), _ptr(meta), _ptr(data)))
    out, o = {}, 0
    for m in meta:
        r, c = int(m[3]), int(m[4])
        out[((int(m[0]), int(m[1])), int(m[2]))] = data[o:o + r * c].reshape(r, c).copy()
        o += r * c
    return out


def bsdmrg_renormalize(ctx, side, bond, stream=None):
    _check(_lib.bsdmrg_renormalize(ctx, side, bond, _stream(stream)))


def bsdmrg_family_count(ctx, side, bond):
    """Returns (families, operators) of a renormalized block."""
    f, o = c_int(), c_int()
    _check(_lib.bsdmrg_family_count(ctx, side, bond, ctypes.byref(f), ctypes.byref(o)))
    return f.value, o.value


def bsdmrg_stats(ctx, reset=False):
    """Returns the context statistics as a dict (seconds per Fig. 9 phase name)."""
    st = Stats()
    _check(_lib.bsdmrg_stats(ctx, ctypes.byref(st), int(bool(reset))))
    out = {"seconds": {name: st.seconds[i] for i, name in enumerate(PHASES)}}
    for name, _ in Stats._fields_[1:]:
        out[name] = getattr(st, name)
    return out


def bsdmrg_destroy(ctx):
    _check(_lib.bsdmrg_destroy(ctx))


def bsdmrg_load_integrals(ctx, h, eri, e_core=0.0):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    _check(_lib.bsdmrg_load_integrals(ctx, _ptr(h), _ptr(eri), e_core))


def site_tensor_arrays(tensor):
    """{(q_left, s): block} -> (meta int32 n x 5, data float64)."""
    keys = sorted(tensor)
    meta = np.array([[ql[0], ql[1], s, tensor[(ql, s)].shape[0], tensor[(ql, s)].shape[1]]
                     for ql, s in keys], dtype=np.int32)
    data = np.concatenate([np.ascontiguousarray(tensor[k], dtype=np.float64).ravel() for k in keys])
    return meta, data


def bsdmrg_set_site_tensor(ctx, site, tensor):
    meta, data = site_tensor_arrays(tensor)
    _check(_lib.bsdmrg_set_site_tensor(ctx, site, len(meta), _ptr(meta), _ptr(data)))


def bsdmrg_renorm_stats(ctx):
    """(flops, wall seconds, device seconds, steps) of all renormalizations so far."""
    f, w, d, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(_lib.bsdmrg_renorm_stats(ctx, ctypes.byref(f), ctypes.byref(w), ctypes.byref(d), ctypes.byref(n)))
    return f.value, w.value, d.value, n.value


def bsdmrg_set_right_normal(ctx, bond):
    _check(_lib.bsdmrg_set_right_normal(ctx, bond))


def bsdmrg_drop_block(ctx, side, bond):
    _check(_lib.bsdmrg_drop_block(ctx, side, bond))


def bsdmrg_set_renorm_workspace(ctx, nbytes):
    _check(_lib.bsdmrg_set_renorm_workspace(ctx, nbytes))


def bsdmrg_build_env(ctx, side, bond, stream=None):
    _check(_lib.bsdmrg_build_env(ctx, side, bond, _stream(stream)))


def bsdmrg_psi_layout(ctx, site):
    """Returns (meta int32 n x 8, offsets int64 n, n_elems)."""
    n = c_int()
    ne = ctypes.c_int64()
    _check(_lib.bsdmrg_psi_layout(ctx, site, ctypes.byref(n), ctypes.byref(ne), None, None))
    meta = np.zeros((n.value, 8), dtype=np.int32)
    off = np.zeros(n.value, dtype=np.int64)
    _check(_lib.bsdmrg_psi_layout(ctx, site, ctypes.byref(n), ctypes.byref(ne), _ptr(meta), _ptr(off)))
    return meta, off, ne.value


def psi_to_flat(psi, layout):
    """Two-site psi dict {(q_l, s1, s2): block} -> flat float64 array in the library layout."""
    meta, off, ne = layout
    out = np.zeros(ne)
    for m, o in zip(meta, off):
        b = psi[((int(m[0]), int(m[1])), int(m[2]), int(m[3]))]
        out[o:o + b.size] = b.ravel()
    return out


def flat_to_psi(flat, layout):
    meta, off, _ = layout
    return {((int(m[0]), int(m[1])), int(m[2]), int(m[3])):
            np.asarray(flat[o:o + m[6] * m[7]]).reshape(m[6], m[7]) for m, o in zip(meta, off)}


def bsdmrg_hpsi_prepare(ctx, site, precision=FP64, ws_bytes=0, stream=None):
    _check(_lib.bsdmrg_hpsi_prepare(ctx, site, precision, ws_bytes, _stream(stream)))


def bsdmrg_hpsi(ctx, site, psi_dev, out_dev, precision=FP64, stream=None):
    _check(_lib.bsdmrg_hpsi(ctx, site, _ptr(psi_dev), _ptr(out_dev), precision, _stream(stream)))


def bsdmrg_hpsi_info(ctx, site, precision=FP64):
    fl = ctypes.c_double()
    a, b, c, d, e = (ctypes.c_int64() for _ in range(5))
    _check(_lib.bsdmrg_hpsi_info(ctx, site, precision, ctypes.byref(fl), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c), ctypes.byref(d), ctypes.byref(e)))
    return {"flops": fl.value, "channels": a.value, "segments": b.value, "aggregates": c.value,
            "ws_bytes": d.value, "op_elems": e.value}


def bsdmrg_hpsi_schedule(ctx, site, precision, target_waves=8192.0, xcd_order=1, wave_max=64):
    _check(_lib.bsdmrg_hpsi_schedule(ctx, site, precision, float(target_waves), int(xcd_order), int(wave_max)))


def bsdmrg_hpsi_autotune(ctx, site, precision=FP64, stream=None):
    """Returns (best ms, default ms, candidates tried); the best schedule is kept."""
    best, dflt, n = ctypes.c_double(), ctypes.c_double(), c_int()
    _check(_lib.bsdmrg_hpsi_autotune(ctx, site, precision, _stream(stream), ctypes.byref(best), ctypes.byref(dflt),
                                     ctypes.byref(n)))
    return best.value, dflt.value, n.value


def bsdmrg_hpsi_profile(ctx, site, psi_dev, out_dev, precision=FP64, stream=None, cap=256):
    """Returns a list of (kind, ms, flops, bytes) per kernel launch of one product."""
    ms = np.zeros(cap)
    fl = np.zeros(cap)
    by = np.zeros(cap)
    kd = np.zeros(cap, dtype=np.int32)
    n = c_int()
    _check(_lib.bsdmrg_hpsi_profile(ctx, site, _ptr(psi_dev), _ptr(out_dev), precision, _stream(stream), cap,
                                    _ptr(ms), _ptr(fl), _ptr(by), _ptr(kd), ctypes.byref(n)))
    return [(int(kd[i]), float(ms[i]), float(fl[i]), float(by[i])) for i in range(min(n.value, cap))]


class DavOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("max_subspace", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tol", ctypes.c_double), ("precond_floor", ctypes.c_double),
                ("precond", ctypes.c_int32), ("pad", ctypes.c_int32)]


def bsdmrg_davidson(ctx, site, psi_dev, max_iter=50, max_subspace=24, restart=4, tol=1e-8,
                    precond_floor=1e-4, precision=FP64, precond=0, stream=None):
    """Returns (energy, iterations, residual norm, list of Ritz values); psi_dev is overwritten."""
    o = DavOpts(max_iter, max_subspace, restart, precision, tol, precond_floor, precond, 0)
    e = ctypes.c_double()
    it = c_int()
    r = ctypes.c_double()
    ritz = np.zeros(max_iter + 1)
    _check(_lib.bsdmrg_davidson(ctx, site, _ptr(psi_dev), ctypes.byref(o), ctypes.byref(e), ctypes.byref(it),
                                ctypes.byref(r), _ptr(ritz), len(ritz), _stream(stream)))
    return e.value, it.value, r.value, list(ritz[:it.value])


def bsdmrg_next_guess(ctx, site, direction, psi_dev, guess_dev, stream=None):
    _check(_lib.bsdmrg_next_guess(ctx, site, direction, _ptr(psi_dev), _ptr(guess_dev), _stream(stream)))


def bsdmrg_hpsi_diagonal(ctx, site, diag_dev, stream=None):
    _check(_lib.bsdmrg_hpsi_diagonal(ctx, site, _ptr(diag_dev), _stream(stream)))


def bsdmrg_truncate(ctx, site, psi_dev, D, direction, stream=None, cap=None):
    """Returns (truncation error, kept count, kept singular values)."""
    cap = cap or 4 * D + 64
    err = ctypes.c_double()
    k = c_int()
    sv = np.zeros(cap)
    _check(_lib.bsdmrg_truncate(ctx, site, _ptr(psi_dev), D, direction, ctypes.byref(err), ctypes.byref(k),
                                _ptr(sv), cap, _stream(stream)))
    return err.value, k.value, sv[:min(k.value, cap)].copy()


def bsdmrg_get_block_op(ctx, side, bond, kind, p=-1, q=-1):
    """Returns {q_in: block} of one stored operator, or None if it is not stored."""
    n = c_int()
    ne = ctypes.c_int64()
    rc = _lib.bsdmrg_get_block_op(ctx, side, bond, kind.encode(), p, q, ctypes.byref(n), ctypes.byref(ne),
                                  None, None)
    if rc == ESTATE:
        return None
    _check(rc)
    meta = np.zeros((n.value, 6), dtype=np.int32)
    data = np.zeros(max(1, ne.value))
    _check(_lib.bsdmrg_get_block_op(ctx, side, bond, kind.encode(), p, q, ctypes.byref(n), ctypes.byref(ne),
                                    _ptr(meta), _ptr(data)))
    out = {}
    o = 0
    for m in meta:
        r, c = int(m[4]), int(m[5])
        out[(int(m[0]), int(m[1]))] = data[o:o + r * c].reshape(r, c).copy()
        o += r * c
    return out


def bsdmrg_block_gemm(problems, precision=FP64, stream=None):
    """problems: list of dicts with torch tensors A, B, C and M, N, K, lda, ldb, ldc,
    transA, transB, alpha, beta."""
    arr = (GemmDesc * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = GemmDesc(_ptr(p["A"]), _ptr(p["B"]), _ptr(p["C"]), p["M"], p["N"], p["K"],
                          int(p.get("transA", 0)), int(p.get("transB", 0)), 0, p["lda"], p["ldb"], p["ldc"],
                          p.get("alpha", 1.0), p.get("beta", 0.0))
    _check(_lib.bsdmrg_block_gemm(len(problems), arr, precision, _stream(stream)))


def make_family_descs(fams):
    """fams: list of dicts {tag, dq, n_layers, block_q (n,2), rows, cols, ld, elem_offset,
    layer_stride, data (device tensor)} -> ctypes array (keeps numpy arrays alive)."""
    arr = (FamilyDesc * max(1, len(fams)))()
    keep = []
    for i, f in enumerate(fams):
        bq = np.ascontiguousarray(f["block_q"], dtype=np.int32).reshape(-1, 2)
        rows = np.ascontiguousarray(f["rows"], dtype=np.int32)
        cols = np.ascontiguousarray(f["cols"], dtype=np.int32)
        ld = np.ascontiguousarray(f["ld"], dtype=np.int32)
        eo = np.ascontiguousarray(f["elem_offset"], dtype=np.int64)
        keep += [bq, rows, cols, ld, eo]
        d = FamilyDesc()
        d.tag = f["tag"]
        d.dq[0], d.dq[1] = f["dq"]
        d.n_layers = f["n_layers"]
        d.n_blocks = len(rows)
        d.block_q, d.rows, d.cols, d.ld, d.elem_offset = (_ptr(x) for x in (bq, rows, cols, ld, eo))
        d.layer_stride = f["layer_stride"]
        d.data = _ptr(f["data"])
        arr[i] = d
    return arr, keep


def bsdmrg_serialized_size_desc(fams):
    arr, keep = make_family_descs(fams)
    n = c_sz()
    _check(_lib.bsdmrg_serialized_size_desc(len(fams), arr, ctypes.byref(n)))
    return n.value


def bsdmrg_pack_desc(fams, dst, cap, stream=None):
    arr, keep = make_family_descs(fams)
    _check(_lib.bsdmrg_pack_desc(len(fams), arr, _ptr(dst), cap, _stream(stream)))


def bsdmrg_pack_desc_noalloc(fams, dst, cap, stream=None):
    arr, keep = make_family_descs(fams)
    _check(_lib.bsdmrg_pack_desc_noalloc(len(fams), arr, _ptr(dst), cap, _stream(stream)))


def bsdmrg_noalloc_scratch_bytes():
    n = c_sz()
    _check(_lib.bsdmrg_noalloc_scratch_bytes(ctypes.byref(n)))
    return n.value


def bsdmrg_unpack_desc(fams, src, nbytes, stream=None):
    arr, keep = make_family_descs(fams)
    _check(_lib.bsdmrg_unpack_desc(len(fams), arr, _ptr(src), nbytes, _stream(stream)))


def bsdmrg_serialized_size(ctx, side, bond):
    n = c_sz()
    _check(_lib.bsdmrg_serialized_size(ctx, side, bond, ctypes.byref(n)))
    return n.value


def bsdmrg_pack(ctx, side, bond, dst, cap, stream=None):
    _check(_lib.bsdmrg_pack(ctx, side, bond, _ptr(dst), cap, _stream(stream)))


def bsdmrg_unpack(ctx, side, bond, src, nbytes, stream=None):
    _check(_lib.bsdmrg_unpack(ctx, side, bond, _ptr(src), nbytes, _stream(stream)))


def bsdmrg_offload(ctx, side, bond, staging, pinned, cap, release, compute, side_stream):
    _check(_lib.bsdmrg_offload(ctx, side, bond, _ptr(staging), _ptr(pinned), cap, int(release),
                               _stream(compute), _stream(side_stream)))


def bsdmrg_offload_wait(ctx, side, bond):
    w = ctypes.c_double()
    _check(_lib.bsdmrg_offload_wait(ctx, side, bond, ctypes.byref(w)))
    return w.value


def bsdmrg_prefetch(ctx, side, bond, pinned, staging, nbytes, compute, side_stream):
    _check(_lib.bsdmrg_prefetch(ctx, side, bond, _ptr(pinned), _ptr(staging), nbytes, _stream(compute),
                                _stream(side_stream)))


def bsdmrg_block_bytes(ctx, side, bond):
    n = c_sz()
    _check(_lib.bsdmrg_block_bytes(ctx, side, bond, ctypes.byref(n)))
    return n.value


def bsdmrg_prefetch_wait(ctx, side, bond):
    w = ctypes.c_double()
    _check(_lib.bsdmrg_prefetch_wait(ctx, side, bond, ctypes.byref(w)))
    return w.value


def bsdmrg_set_side_delay(ctx, ms):
    _check(_lib.bsdmrg_set_side_delay(ctx, float(ms)))


def bsdmrg_set_hbm_budget(ctx, nbytes, chunk_bytes=0):
    _check(_lib.bsdmrg_set_hbm_budget(ctx, int(nbytes), int(chunk_bytes)))


def bsdmrg_hpsi_streamed(ctx, site):
    """Returns (streamed, pinned host bytes copied per product, chunks)."""
    st, hb, nc = c_int(), c_sz(), c_int()
    _check(_lib.bsdmrg_hpsi_streamed(ctx, site, ctypes.byref(st), ctypes.byref(hb), ctypes.byref(nc)))
    return bool(st.value), hb.value, nc.value


def bsdmrg_segments_size(ctx, side, bond, staging_bytes):
    """Returns (bytes, segments) of the segmented form for a staging size."""
    n, k = c_sz(), c_int()
    _check(_lib.bsdmrg_segments_size(ctx, side, bond, staging_bytes, ctypes.byref(n), ctypes.byref(k)))
    return n.value, k.value


def bsdmrg_pack_segments(ctx, side, bond, staging, staging_bytes, pinned, cap, compute=None, side_stream=None):
    """Returns (bytes written, segments)."""
    n, k = c_sz(), c_int()
    _check(_lib.bsdmrg_pack_segments(ctx, side, bond, _ptr(staging), staging_bytes, _ptr(pinned), cap,
                                     ctypes.byref(n), ctypes.byref(k), _stream(compute), _stream(side_stream)))
    return n.value, k.value


def bsdmrg_unpack_segments(ctx, side, bond, pinned, nbytes, staging, staging_bytes, compute=None, side_stream=None):
    _check(_lib.bsdmrg_unpack_segments(ctx, side, bond, _ptr(pinned), nbytes, _ptr(staging), staging_bytes,
                                       _stream(compute), _stream(side_stream)))


def bsdmrg_set_copy_workgroups(n):
    _check(_lib.bsdmrg_set_copy_workgroups(int(n)))


def bsdmrg_set_split_policy(ctx, fp64_heavy=1):
    _check(_lib.bsdmrg_set_split_policy(ctx, int(fp64_heavy)))
