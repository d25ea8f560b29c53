"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments on the host, and generates the same
projection as the oracle's independent implementation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import prng
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "bvs.h")


@pytest.fixture(scope="module")
def bvs():
    from paper_2412_03301_amd import bvs as b
    if not os.path.exists(b.LIB_PATH):
        pytest.skip("libbvs.so not built")
    b.lib()
    return b


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bvs_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(bvs):
    names = declared_functions()
    assert len(names) >= 20
    lib = bvs.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(bvs.EXPORTED)


def test_version_and_defaults(bvs):
    assert b"gfx950" in bvs.lib().bvs_version()
    p = bvs.Params()
    bvs.lib().bvs_params_default(C.byref(p))
    assert (p.code_bits, p.wta_k, p.access_lists, p.min_count) == (1024, 64, 3, 1)
    assert bvs.lib().bvs_params_check(C.byref(p)) == bvs.BVS_ENOTSUP   # dim unset
    p.dim = 128
    bvs.params_check(p)


@pytest.mark.parametrize("field,value,status", [
    ("dim", 0, -6), ("dim", 2048, -6), ("code_bits", 1000, -6), ("code_bits", 128, -6),
    ("code_bits", 8192, -6), ("fan_in", 0, -1), ("fan_in", 200, -1), ("wta_k", 0, -1),
    ("wta_k", 5000, -1), ("access_lists", 0, -1), ("access_lists", 9, -1), ("min_count", 256, -1),
    ("top_t", 0, -6), ("top_t", 5000, -6), ("flags", 1, -1),
])
def test_param_validation(bvs, field, value, status):
    p = bvs.Params.make(dim=128, code_bits=1024, fan_in=8, wta_k=32, top_t=200)
    setattr(p, field, value)
    assert bvs.lib().bvs_params_check(C.byref(p)) == status
    assert bvs.lib().bvs_last_error() != b""


def test_wta_key_width_limit(bvs):
    # s * 8192 must stay below 2^(32 - log2 L).
    ok = bvs.Params.make(dim=384, code_bits=4096, fan_in=127, wta_k=64)
    bad = bvs.Params.make(dim=384, code_bits=4096, fan_in=128, wta_k=64)
    assert bvs.lib().bvs_params_check(C.byref(bad)) == bvs.BVS_ENOTSUP
    # 4096 * 128 (rounded fan-in) > 65536 entries of the LDS table as well
    assert bvs.lib().bvs_params_check(C.byref(ok)) == bvs.BVS_ENOTSUP
    assert bvs.lib().bvs_params_check(C.byref(bvs.Params.make(dim=384, code_bits=4096, fan_in=16))) == 0


@pytest.mark.parametrize("seed,d,L,s", [(0, 128, 1024, 8), (0, 384, 4096, 16), (12345, 768, 4096, 16),
                                        (7, 17, 256, 17), (2 ** 64 - 1, 64, 512, 3)])
def test_projection_matches_oracle(bvs, seed, d, L, s):
    p = bvs.Params.make(dim=d, code_bits=L, fan_in=s, wta_k=8, seed=seed)
    lib_idx = bvs.projection(p)
    ora_idx = prng.projection_rows(seed, d, L, s)
    assert np.array_equal(lib_idx.astype(np.int64), ora_idx)


def test_index_and_workspace_sizes(bvs):
    p = bvs.Params.make(dim=384, code_bits=4096, fan_in=16, wta_k=64, top_t=1000)
    out = C.c_uint64()
    assert bvs.lib().bvs_index_bytes(C.byref(p), 1_000_000, 52_500_000, C.byref(out)) == 0
    # planes 2 B/element + norms and screening pairs 12 B/vector + counts
    # L B/set + bits L/8 B/set + membership bitmaps L/8 B/set + set weights
    # 2 B/set + offsets
    approx = 52_500_000 * (384 * 2 + 12) + 1_000_192 * (4096 + 512 + 512 + 2) + 8 * 1_000_001
    assert abs(out.value - approx) < 1 << 20
    assert bvs.lib().bvs_build_workspace_bytes(C.byref(p), 1000, 5000, C.byref(out)) == 0
    assert out.value >= 1000 * (4096 + 512)


def _build(bvs, p, offsets, idx_bytes=1 << 30, ws_bytes=1 << 30):
    off = np.asarray(offsets, np.uint64)
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)
    st = bvs.lib().bvs_build_index(C.byref(p), fake, off.ctypes.data_as(bvs.PU64), len(off) - 1, fake,
                                   idx_bytes, fake, ws_bytes, None, C.byref(h))
    return st, h


def test_build_rejects_bad_offsets_on_host(bvs):
    p = bvs.Params.make(dim=32, code_bits=256, fan_in=4, wta_k=8, top_t=10)
    assert _build(bvs, p, [1, 2, 3])[0] == bvs.BVS_EINVAL            # offsets[0] != 0
    assert _build(bvs, p, [0, 2, 2, 5])[0] == bvs.BVS_EINVAL         # empty set
    assert _build(bvs, p, [0, 3, 2])[0] == bvs.BVS_EINVAL            # decreasing
    assert _build(bvs, p, [0, 10, 266])[0] == bvs.BVS_ERANGE         # 256 vectors in a set
    assert _build(bvs, p, [0, 4, 8], idx_bytes=16)[0] == bvs.BVS_ENOSPC
    assert _build(bvs, p, [0, 4, 8], ws_bytes=16)[0] == bvs.BVS_ENOSPC
    st, h = _build(bvs, p, [0, 4, 8])
    assert h.value is None
    p.flags = 3
    assert _build(bvs, p, [0, 4, 8])[0] == bvs.BVS_EINVAL


def test_calls_reject_null_index(bvs):
    L = bvs.lib()
    out = C.c_uint64()
    assert L.bvs_search_workspace_bytes(None, 1, 1, C.byref(out)) == bvs.BVS_EINVAL
    off = np.array([0, 3], np.uint64)
    fake = C.c_void_p(0x1000)
    assert L.bvs_search(None, fake, off.ctypes.data_as(bvs.PU64), 1, 10, fake, 1 << 20, fake, fake, fake,
                        None) == bvs.BVS_EINVAL
    assert L.bvs_bruteforce(None, fake, off.ctypes.data_as(bvs.PU64), 1, 10, fake, 1 << 20, fake, fake, fake,
                            None) == bvs.BVS_EINVAL
    assert L.bvs_sketch_views(None, None, None) == bvs.BVS_EINVAL


def test_batch_calls_reject_null_handles(bvs):
    L = bvs.lib()
    off = np.array([0, 3, 5], np.uint64)
    h = C.c_void_p()
    assert L.bvs_batch_create(None, off.ctypes.data_as(bvs.PU64), 2, 10, None, C.byref(h)) == bvs.BVS_EINVAL
    assert h.value is None
    assert L.bvs_batch_create(None, off.ctypes.data_as(bvs.PU64), 2, 10, None, None) == bvs.BVS_EINVAL
    fake = C.c_void_p(0x1000)
    assert L.bvs_batch_bind(None, fake, fake, 1 << 20, fake, fake, fake, None) == bvs.BVS_EINVAL
    assert L.bvs_batch_launch(None, None) == bvs.BVS_EINVAL
    assert L.bvs_batch_status(None, None) == bvs.BVS_EINVAL
    info = bvs.BatchInfo()
    assert L.bvs_batch_get_info(None, C.byref(info)) == bvs.BVS_EINVAL
    L.bvs_batch_destroy(None)


def test_metric_calls_reject_unknown_metric_on_the_host(bvs):
    lib = bvs.lib()
    for fn in (lib.bvs_search_metric, lib.bvs_bruteforce_metric):
        assert fn(None, 7, None, None, 1, 10, None, 0, None, None, None, None) == bvs.BVS_EINVAL
        assert b"metric" in lib.bvs_last_error()
        assert fn(None, -1, None, None, 1, 10, None, 0, None, None, None, None) == bvs.BVS_EINVAL


def test_search_params_setter_validates_on_the_host(bvs):
    lib = bvs.lib()
    assert lib.bvs_index_set_search_params(None, 3, 1, 1000) == bvs.BVS_EINVAL
