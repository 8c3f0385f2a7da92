"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/miaug.h, its host sampler equals the oracle's sampler bit
for bit, and argument validation reports the documented status codes without
touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "miaug.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(miaug_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def miaug():
    import paper_1809_06839_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1809_06839_amd import build
        build.build()
    m.lib()
    return m


def test_every_declared_symbol_is_exported(miaug):
    syms = declared_symbols()
    assert len(syms) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", miaug.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (miaug_[a-z0-9_]+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    for s in syms:
        getattr(miaug.lib(), s)


def test_status_strings(miaug):
    L = miaug.lib()
    assert L.miaug_version() >= 10000
    assert L.miaug_status_str(0) == b"ok"
    assert L.miaug_status_str(-6) == b"workspace too small"


def test_sampler_matches_the_oracle_bit_for_bit(miaug):
    import oracle
    for seed, first, n in [(1809068391, 0, 500), (7, 10**12, 50), (2**63 + 5, 3, 20)]:
        f1, a1 = miaug.sample_d4bc(seed, first, n)
        f2, a2 = oracle.sample_d4bc(seed, first, n)
        assert np.array_equal(f1, f2) and np.array_equal(a1.view(np.uint32), a2.view(np.uint32))
        c1, k1 = miaug.sample_c2(seed, first, n)
        c2, k2 = oracle.sample_c2(seed, first, n)
        assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32)) and np.array_equal(k1, k2)
        assert np.array_equal(miaug.sample_wc(seed, first, n).view(np.uint32),
                              oracle.sample_wc(seed, first, n).view(np.uint32))
        assert np.array_equal(miaug.sample_grid(seed, first, n).view(np.uint64),
                              oracle.sample_grid(seed, first, n).view(np.uint64))


def test_validation_errors_without_a_gpu(miaug):
    L = miaug.lib()
    assert L.miaug_sample_d4bc(1, 0, -1, None, None) == miaug.EINVAL
    assert L.miaug_sample_d4bc(1, 0, 3, None, None) == miaug.EINVAL
    assert b"bad arguments" in L.miaug_last_error()
    assert L.miaug_sample_grid(1, 0, 1, 1.5, None) == miaug.EINVAL
    assert L.miaug_d4_bc_u8(None, 1, 4, 4, 2, None, None, None, None) == miaug.ESHAPE
    assert L.miaug_d4_bc_u8(None, 1, 4, 4, 3, None, None, None, None) == miaug.EINVAL
    assert L.miaug_d4_bc_u8(None, 0, 4, 4, 3, None, None, None, None) == miaug.OK  # empty batch is a no-op
    assert L.miaug_d4_bc_u8(None, -1, 4, 4, 3, None, None, None, None) == miaug.EINVAL
    a = miaug.RaggedArgs()
    a.n, a.out_h, a.out_w = 2, 224, 224
    assert L.miaug_ragged_apply(None, ctypes.byref(a), None) == miaug.EINVAL
    dummy = ctypes.c_void_p(1)
    assert L.miaug_ragged_apply(dummy, ctypes.byref(a), None) == miaug.EINVAL  # NULL image pointers
    a.out_h = 0
    assert L.miaug_ragged_apply(dummy, ctypes.byref(a), None) == miaug.ESHAPE
    assert L.miaug_ragged_set_variant(dummy, 99) == miaug.EINVAL
    assert L.miaug_warpcolor_bwd(None, 1, 3, 8, 8, None, None, None, None, None, 0, None) == miaug.EINVAL
    assert L.miaug_elastic_fields(1, 0, 1, 8, 8, 50.0, 1000, 0, ctypes.c_void_p(8), None, 0, None) == miaug.ESHAPE
    assert L.miaug_image_stats_u8(None, 1, 10, 5, None, None, None, None, None) == miaug.ESHAPE
    assert L.miaug_ragged_variant_count() >= 4
    assert L.miaug_ragged_variant_name(0)
    # launch forms switched off are named "off: ..." and cannot be forced
    off = [v for v in range(L.miaug_ragged_variant_count()) if L.miaug_ragged_variant_name(v).startswith(b"off: ")]
    assert off and 0 not in off
    assert L.miaug_ragged_set_variant(dummy, off[0]) == miaug.EUNSUPPORTED
    assert b"switched off" in L.miaug_last_error()


def test_ctx_create_reports_a_missing_device(miaug):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = miaug.lib().miaug_ctx_create(0, None, ctypes.byref(h))
    assert st == miaug.EDEVICE and not h.value


def test_c2_compile_matches_the_oracle_setup(miaug):
    import oracle
    m = miaug
    f, k = m.sample_c2(5, 0, 64)
    rec = m.compile_c2(f, k, 512, 512, 448)
    for i in range(64):
        aq = np.frombuffer(rec[i, :48].tobytes(), np.int64)
        assert np.array_equal(aq, oracle.ssr_matrix_q32(*f[i][:4], 512, 512))
        assert np.array_equal(rec[i, 72:], oracle.gamma_lut(f[i][4]))
