"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments, and predicts serialized sizes exactly
like the reference serializer (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from synthetic import make_integrals

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "bsdmrg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsdmrg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2412_04676_amd import bsdmrg as B
    lib = ctypes.CDLL(B.LIBPATH)
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(B.EXPORTED)


def test_integral_validation():
    from paper_2412_04676_amd import bsdmrg as B
    ctx = B.bsdmrg_create(4, 2, 2)
    h, eri = make_integrals(4)
    B.bsdmrg_load_integrals(ctx, h, eri)
    bad = eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_load_integrals(ctx, h, bad)
    assert e.value.code == B.EINVAL
    hb = h.copy()
    hb[0, 1] += 1.0
    with pytest.raises(B.BsdmrgError):
        B.bsdmrg_load_integrals(ctx, hb, eri)
    with pytest.raises(B.BsdmrgError):
        B.bsdmrg_load_integrals(ctx, h, eri, 1.0)
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_psi_layout(ctx, 1)
    assert e.value.code == B.ESTATE


def test_create_rejects_bad_sizes():
    from paper_2412_04676_amd import bsdmrg as B
    for args in [(1, 0, 0), (4, 5, 0), (4, -1, 1)]:
        with pytest.raises(B.BsdmrgError):
            B.bsdmrg_create(*args)


def test_serialized_size_matches_reference():
    from paper_2412_04676_amd import bsdmrg as B
    from oracle import serializer as S
    rng = np.random.default_rng(0)
    fams_o, fams_b = [], []
    for k in range(5):
        nb = int(rng.integers(0, 6))
        rows = rng.integers(0, 9, nb)
        cols = rng.integers(0, 9, nb)
        nl = int(rng.integers(0, 4))
        ld = cols + rng.integers(0, 3, nb)
        off = np.concatenate([[0], np.cumsum(rows * ld)])[:-1] if nb else np.zeros(0, dtype=np.int64)
        le = int(sum(rows * cols))
        fams_o.append({"tag": k, "dq": (1, 0), "blocks": [((i, 0), int(rows[i]), int(cols[i])) for i in range(nb)],
                       "data": np.zeros((nl, le))})
        fams_b.append({"tag": k, "dq": (1, 0), "n_layers": nl, "block_q": [[i, 0] for i in range(nb)],
                       "rows": rows, "cols": cols, "ld": ld, "elem_offset": off,
                       "layer_stride": int(sum(rows * ld)) + 4, "data": 256})
    assert B.bsdmrg_serialized_size_desc(fams_b) == S.serialized_size(fams_o)


def test_block_and_schedule_calls_validate_arguments():
    from paper_2412_04676_amd import bsdmrg as B
    ctx = B.bsdmrg_create(6, 3, 3)
    assert B.bsdmrg_renorm_stats(ctx) == (0.0, 0.0, 0.0, 0)
    for bond in (0, 6, -1):   # the vacuum blocks stay; out of range
        with pytest.raises(B.BsdmrgError) as e:
            B.bsdmrg_drop_block(ctx, B.LEFT, bond)
        assert e.value.code == B.EINVAL
    B.bsdmrg_drop_block(ctx, B.RIGHT, 3)   # not built: nothing to free
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_drop_block(ctx, 7, 3)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_set_right_normal(ctx, 0)
    assert e.value.code == B.EINVAL
    B.bsdmrg_set_right_normal(ctx, 4)
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_hpsi_schedule(ctx, 2, B.FP64, 8192, 1, 64)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_hpsi_schedule(ctx, 2, B.FP64, 10.0, 1, 64)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_hpsi_schedule(ctx, 2, 9, 8192, 1, 64)
    assert e.value.code == B.EINVAL
    B.bsdmrg_destroy(ctx)


def test_config_and_state_calls_validate_arguments():
    from paper_2412_04676_amd import bsdmrg as B
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_create(6, 3, 3, flags=1)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_create(6, 3, 3, D_max=-1)
    assert e.value.code == B.EINVAL
    ctx = B.bsdmrg_create(6, 3, 3, D_max=64, hpsi_ws_bytes=1 << 30, renorm_ws_bytes=1 << 30,
                          right_normal_from=5)
    st = B.bsdmrg_stats(ctx)
    assert all(v == 0.0 for v in st["seconds"].values()) and st["hpsi_calls"] == 0
    assert set(st["seconds"]) == {"Tables", "Diag_H", "Ren_l", "Ren_r", "SVD", "StVec", "IO"}
    # vacuum blocks exist and hold no operators; other blocks are not built
    assert B.bsdmrg_family_count(ctx, B.LEFT, 0) == (0, 0)
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_family_count(ctx, B.LEFT, 2)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_get_site_tensor(ctx, 1)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_get_site_tensor(ctx, 6)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:   # integrals not loaded
        B.bsdmrg_renormalize(ctx, B.LEFT, 0)
    assert e.value.code == B.ESTATE
    h, eri = make_integrals(6)
    B.bsdmrg_load_integrals(ctx, h, eri)
    for side, bond in ((B.LEFT, 6), (B.RIGHT, 0), (3, 1)):
        with pytest.raises(B.BsdmrgError) as e:
            B.bsdmrg_renormalize(ctx, side, bond)
        assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:   # site tensor missing
        B.bsdmrg_renormalize(ctx, B.LEFT, 0)
    assert e.value.code == B.ESTATE
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_next_guess(ctx, 2, 2, 256, 256)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BsdmrgError) as e:   # environment blocks not built
        B.bsdmrg_next_guess(ctx, 2, 0, 256, 256)
    assert e.value.code == B.ESTATE
    B.bsdmrg_destroy(ctx)


def test_noalloc_pack_limits_are_checked_on_the_host():
    """The allocation-free pack states its fixed scratch size and refuses,
    before any device call, descriptor tables that do not fit it and
    destinations below the exact serialized size."""
    from paper_2412_04676_amd import bsdmrg as B
    assert B.bsdmrg_noalloc_scratch_bytes() == 16 << 20

    def family(nb):
        return {"tag": 0, "dq": (0, 0), "n_layers": 1, "block_q": np.zeros((nb, 2), dtype=np.int32),
                "rows": np.ones(nb), "cols": np.ones(nb), "ld": np.ones(nb),
                "elem_offset": np.arange(nb), "layer_stride": nb, "data": 256}

    big = family(600_000)   # one descriptor and one offset per block: above 16 MiB
    n = B.bsdmrg_serialized_size_desc([big])
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_pack_desc_noalloc([big], 4096, n)
    assert e.value.code == B.EINVAL and "exceed the no-allocation scratch" in str(e.value)
    small = family(3)
    n = B.bsdmrg_serialized_size_desc([small])
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_pack_desc_noalloc([small], 4096, n - 1)
    assert e.value.code == B.ENOMEM
    with pytest.raises(B.BsdmrgError) as e:
        B.bsdmrg_pack_desc_noalloc([small], 4096 + 8, n)
    assert e.value.code == B.EINVAL
