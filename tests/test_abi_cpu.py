"""The C ABI library loads and exports every symbol the header declares, and
its host-side validation behaves as documented.  No call here reaches a
device: every case returns before the first HIP call."""

from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "linview.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1403_6968_amd import linview
    if not os.path.exists(linview.LIB_PATH):
        from paper_1403_6968_amd import build_lib
        build_lib.build()
    return linview.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lv_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(lib):
    from paper_1403_6968_amd import linview
    names = _declared()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), f"{name} declared in linview.h but not exported"
    assert set(names) == set(linview.EXPORTED)


def test_status_strings(lib):
    from paper_1403_6968_amd import linview as L
    assert L.lv_status_str(0) == "LV_OK"
    assert L.lv_status_str(1) == "LV_EINVAL"
    assert L.lv_status_str(3) == "LV_EDEVICE"


def test_footprint_rules(lib):
    from paper_1403_6968_amd import linview as L
    f = L.lv_view_footprint
    # the stored powers alone: (m + 1) padded float matrices
    assert f(8192, 16, 1, L.LV_FP32) >= 5 * 8192 * 8192 * 4
    assert f(8192, 16, 1, L.LV_FP64) >= 5 * 8192 * 8192 * 8
    assert f(1000, 16, 1, L.LV_FP32) == f(1024, 16, 1, L.LV_FP32)     # padded to 256
    assert f(1025, 16, 1, L.LV_FP32) > f(1024, 16, 1, L.LV_FP32)
    assert f(1000, 1, 1, L.LV_FP64) >= 1024 * 1024 * 8
    for bad in [(0, 16, 1, 1), (100, 3, 1, 1), (100, 12, 1, 1), (100, 16, 0, 1),
                (100, 16, 1, 7), (100, 2048, 1, 1), (100, 16, 64, 1)]:
        assert f(*bad) == 0, bad
    assert L.lv_reeval_footprint(1000, 1, L.LV_FP32) >= 2 * 1024 * 1024 * 4
    assert L.lv_reeval_footprint(0, 1, L.LV_FP32) == 0


def test_wide_factor_rules(lib):
    """Top factors up to 512 columns (k * r_max rounded up) for plain float
    views only; FP64, sums and allocation-free re-evaluation stop at 256."""
    from paper_1403_6968_amd import linview as L
    f = L.lv_view_footprint
    for mode in (L.LV_FP32, L.LV_FP32_BF16SHADOW):
        assert f(1000, 16, 32, mode) > f(1000, 16, 16, mode) > 0
        assert f(1000, 32, 16, mode) > 0
        assert f(1000, 16, 33, mode) == 0                 # rounds up to 64: width 1024
    assert f(1000, 16, 16, L.LV_FP64) > 0
    assert f(1000, 16, 32, L.LV_FP64) == 0
    assert f(1000, 16, 16, L.LV_FP32, L.LV_WITH_SUMS) > 0
    assert f(1000, 16, 32, L.LV_FP32, L.LV_WITH_SUMS) == 0
    assert L.lv_reeval_footprint(1000, 256, L.LV_FP32) > 0
    assert L.lv_reeval_footprint(1000, 257, L.LV_FP32) == 0


def test_create_validation_before_device(lib):
    from paper_1403_6968_amd import linview as L
    h = ctypes.c_void_p()
    # NULL A / workspace
    st = lib.lv_view_create(None, 64, 64, 4, 1, L.LV_FP32, None, 0, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "NULL" in L.lv_last_error()
    # k not a power of two
    st = lib.lv_view_create(0x1000, 64, 64, 6, 1, L.LV_FP32, 0x1000, 1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "power of two" in L.lv_last_error()
    # lda < n
    st = lib.lv_view_create(0x1000, 64, 32, 4, 1, L.LV_FP32, 0x1000, 1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL
    # misaligned workspace
    st = lib.lv_view_create(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1001, 1 << 30, None, ctypes.byref(h))
    assert st == L.LV_ENOMEM
    # workspace too small
    need = L.lv_view_footprint(64, 4, 1, L.LV_FP32)
    st = lib.lv_view_create(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, need - 1, None, ctypes.byref(h))
    assert st == L.LV_ENOMEM and str(need) in L.lv_last_error()
    assert not h.value
    # null out
    st = lib.lv_view_create(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, need, None, None)
    assert st == L.LV_EINVAL


def test_null_view_calls(lib):
    from paper_1403_6968_amd import linview as L
    assert lib.lv_view_update(None, 0x1000, 0x1000, 1, 1, 1, None) == L.LV_EINVAL
    assert lib.lv_view_update_batch(None, 0x1000, 0x1000, 1, 2, 1, 1, 64, 64, None) == L.LV_EINVAL
    assert lib.lv_view_update_batch(None, 0x1000, 0x1000, 1, -1, 1, 1, 64, 64, None) == L.LV_EINVAL
    assert lib.lv_view_read(None, 1, 0x1000, 1, None) == L.LV_EINVAL
    assert lib.lv_view_reanchor(None, None) == L.LV_EINVAL
    assert lib.lv_view_data(None, 1, None) is None
    s = L.lv_stats()
    assert lib.lv_view_stats(None, ctypes.byref(s)) == L.LV_EINVAL
    lib.lv_view_destroy(None)


def test_reeval_validation(lib):
    from paper_1403_6968_amd import linview as L
    st = lib.lv_reeval(0x1000, 64, 64, 5, None, None, 0, 0, 0, L.LV_FP32, 0x1000, 64, 0x1000, 1 << 30, None)
    assert st == L.LV_EINVAL
    st = lib.lv_reeval(0x1000, 64, 64, 4, None, None, 1, 1, 1, L.LV_FP32, 0x1000, 64, 0x1000, 1 << 30, None)
    assert st == L.LV_EINVAL   # r = 1 with NULL U/V
    st = lib.lv_reeval(0x1000, 64, 64, 4, None, None, 0, 0, 0, L.LV_FP32, 0x1000, 64, 0x1000, 16, None)
    assert st == L.LV_ENOMEM


def test_shadow_mode_footprint(lib):
    """LV_FP32_BF16SHADOW adds one bfloat16 copy of each power below the top
    (2 bytes per padded element) to the FP32 footprint."""
    from paper_1403_6968_amd import linview as L
    for n, k in [(1000, 16), (8192, 16), (300, 2), (513, 1)]:
        n_pad = -(-n // 256) * 256
        m = k.bit_length() - 1
        extra = L.lv_view_footprint(n, k, 1, L.LV_FP32_BF16SHADOW) - L.lv_view_footprint(n, k, 1, L.LV_FP32)
        assert m * n_pad * n_pad * 2 <= extra <= m * (n_pad * n_pad * 2 + 256), (n, k, extra)
    assert L.lv_reeval_footprint(1000, 1, L.LV_FP32_BF16SHADOW) == 0


def test_tile_and_tuning_calls_validate(lib):
    from paper_1403_6968_amd import linview as L
    rows = ctypes.c_int()
    assert lib.lv_view_tile_rows(None, 0, ctypes.byref(rows)) == L.LV_EINVAL
    assert lib.lv_view_set_tile_rows(None, 0, 512) == L.LV_EINVAL
    assert lib.lv_batch_tuning(None, None, None) == L.LV_EINVAL
    assert lib.lv_view_set_pipeline(None, 1) == L.LV_EINVAL
    assert lib.lv_view_autotune(None, 1, 24, None, None) == L.LV_EINVAL


def test_sums_footprint_and_flags(lib):
    from paper_1403_6968_amd import linview as L
    for n, k, r in [(1000, 16, 1), (300, 8, 4), (513, 1, 2)]:
        plain = L.lv_view_footprint(n, k, r, L.LV_FP32)
        assert L.lv_view_footprint(n, k, r, L.LV_FP32, 0) == plain
        sums = L.lv_view_footprint(n, k, r, L.LV_FP32, L.LV_WITH_SUMS)
        n_pad = -(-n // 256) * 256
        m = k.bit_length() - 1
        assert sums >= plain + (m + 1) * n_pad * n_pad * 4      # the stored sums S_1 .. S_k
    assert L.lv_view_footprint(1000, 16, 1, L.LV_FP32, 4) == 0  # unknown flag
    h = ctypes.c_void_p()
    st = lib.lv_view_create_ex(0x1000, 64, 64, 4, 1, L.LV_FP32, 8, 0x1000, 1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "flags" in L.lv_last_error()
    assert lib.lv_view_read_sum(None, 1, 0x1000, 64, None) == L.LV_EINVAL


def test_general_footprint_and_validation(lib):
    from paper_1403_6968_amd import linview as L
    for n, k, r, p in [(1000, 16, 1, 1), (300, 8, 4, 5), (513, 1, 2, 64)]:
        sums = L.lv_view_footprint(n, k, r, L.LV_FP32, L.LV_WITH_SUMS)
        gen = L.lv_view_footprint_general(n, k, r, L.LV_FP32, p)
        n_pad = -(-n // 256) * 256
        pp = 1 << (p - 1).bit_length()
        m = k.bit_length() - 1
        # T_1 .. T_k, T_0, B and the two deltas in storage type, four FP64 n x p buffers
        assert gen >= sums + (m + 5) * n_pad * pp * 4 + 4 * n_pad * pp * 8
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 0) == 0
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 65) == 0
    assert L.lv_view_footprint_general(1000, 6, 1, L.LV_FP32, 4) == 0
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 4, 7) == 0            # unknown strategy
    F = L.LV_GENERAL_FACTORED
    fac = L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 1000, F)
    # T_1 .. T_16, T_0, B in storage type (p padded to 1024) and four FP64 n x p creation buffers
    assert fac >= L.lv_view_footprint(1000, 16, 1, L.LV_FP32, L.LV_WITH_SUMS) + 7 * 1024 * 1024 * 4 + 4 * 1024 * 1024 * 8
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 4096, F) > 0
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 4097, F) == 0
    assert L.lv_view_footprint_general(1000, 16, 16, L.LV_FP32, 4, F) == 0            # k * r_pad > 128
    h = ctypes.c_void_p()
    st = lib.lv_view_create_general(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 65, 0, 0, 0x1000, 1 << 30,
                                    None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "p = 65" in L.lv_last_error()
    st = lib.lv_view_create_general(0x1000, 64, 64, 4, 1, L.LV_FP32, None, 4, 0x1000, 4, 4, 0, 0, 0x1000, 1 << 30,
                                    None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "NULL" in L.lv_last_error()
    st = lib.lv_view_create_general(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 3, 0x1000, 4, 4, 0, 0, 0x1000, 1 << 30,
                                    None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "ldt" in L.lv_last_error()
    st = lib.lv_view_create_general(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, 3, 0, 0x1000, 1 << 30,
                                    None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "strategy" in L.lv_last_error()
    need = L.lv_view_footprint_general(64, 4, 1, L.LV_FP32, 4)
    st = lib.lv_view_create_general(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, 0, 0, 0x1000, need - 1,
                                    None, ctypes.byref(h))
    assert st == L.LV_ENOMEM and str(need) in L.lv_last_error()
    assert lib.lv_view_read_general(None, 1, 0x1000, 4, None) == L.LV_EINVAL
    assert lib.lv_server_set_hold(None, 1, 0.0) == L.LV_EINVAL


def test_general_skip_footprint_and_validation(lib):
    from paper_1403_6968_amd import linview as L
    F = L.LV_GENERAL_FACTORED
    exp16 = L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 8, F)
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 8, F, 16) == exp16        # s = k: exponential
    sk = L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 8, F, 4)
    exp4 = L.lv_view_footprint_general(1000, 4, 1, L.LV_FP32, 8, F)
    # three more T (T_8, T_12, T_16) with their factor slabs, no powers beyond P_4
    assert exp4 + 3 * 1024 * 128 * 4 < sk < exp16
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 8, F, 3) == 0             # s not a power of two
    assert L.lv_view_footprint_general(1000, 12, 1, L.LV_FP32, 8, F, 8) == 0             # s does not divide k
    assert L.lv_view_footprint_general(1000, 12, 1, L.LV_FP32, 8, F, 4) > 0
    assert L.lv_view_footprint_general(1000, 16, 1, L.LV_FP32, 8, L.LV_GENERAL_HYBRID, 4) == 0
    assert L.lv_view_footprint_general(1000, 64, 2, L.LV_FP32, 8, F, 2) == 0             # (2k - 1 - 2s) r > 128
    assert L.lv_view_footprint_general(1000, 32, 2, L.LV_FP32, 8, F, 8) > 0              # 47 * 2 <= 128
    h = ctypes.c_void_p()
    st = lib.lv_view_create_general(0x1000, 64, 64, 16, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, 0, 4, 0x1000,
                                    1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "factored" in L.lv_last_error()
    st = lib.lv_view_create_general(0x1000, 64, 64, 16, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, F, 6, 0x1000,
                                    1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "s = 6" in L.lv_last_error()


def test_chain_footprint_and_validation(lib):
    from paper_1403_6968_amd import linview as L
    n_pad = 1024
    mat = n_pad * n_pad * 4
    lin = L.load().lv_chain_footprint(1000, 16, 1, L.LV_FP32, L.LV_MODEL_LIN, 0)
    exp = L.load().lv_chain_footprint(1000, 16, 1, L.LV_FP32, L.LV_MODEL_EXP, 0)
    skip = L.load().lv_chain_footprint(1000, 16, 1, L.LV_FP32, L.LV_MODEL_SKIP, 4)
    # Table 2 (space): k, log k + 1 and log s + k/s stored matrices
    assert lin >= 16 * mat and exp >= 5 * mat and skip >= 6 * mat
    assert lin > skip > exp
    f = L.load().lv_chain_footprint
    assert f(1000, 12, 1, L.LV_FP32, L.LV_MODEL_LIN, 0) > 0           # linear: any k
    assert f(1000, 12, 1, L.LV_FP32, L.LV_MODEL_EXP, 0) == 0          # exponential: power of two
    assert f(1000, 16, 1, L.LV_FP32, L.LV_MODEL_SKIP, 3) == 0         # s not a power of two
    assert f(1000, 16, 1, L.LV_FP32, L.LV_MODEL_SKIP, 32) == 0        # s > k
    assert f(1000, 12, 1, L.LV_FP32, L.LV_MODEL_SKIP, 8) == 0         # s does not divide k
    assert f(1000, 128, 1, L.LV_FP32, L.LV_MODEL_LIN, 0) > 0
    assert f(1000, 129, 1, L.LV_FP32, L.LV_MODEL_LIN, 0) == 0         # width k * r_pad > 128
    assert f(1000, 16, 1, L.LV_FP32_BF16SHADOW, L.LV_MODEL_LIN, 0) == 0
    assert f(1000, 16, 1, L.LV_FP32, 7, 0) == 0
    h = ctypes.c_void_p()
    st = lib.lv_chain_create(0x1000, 64, 64, 12, 1, L.LV_FP32, L.LV_MODEL_SKIP, 8, 0x1000, 1 << 30, None,
                             ctypes.byref(h))
    assert st == L.LV_EINVAL and "skip" in L.lv_last_error()
    need = f(64, 8, 1, L.LV_FP32, L.LV_MODEL_LIN, 0)
    st = lib.lv_chain_create(0x1000, 64, 64, 8, 1, L.LV_FP32, L.LV_MODEL_LIN, 0, 0x1000, need - 1, None,
                             ctypes.byref(h))
    assert st == L.LV_ENOMEM and str(need) in L.lv_last_error()
    assert lib.lv_chain_update(None, 0x1000, 0x1000, 1, 1, 1, None) == L.LV_EINVAL
    assert lib.lv_chain_read(None, 1, 0x1000, 64, None) == L.LV_EINVAL
    assert lib.lv_chain_powers(None, None, 0) == -1


def test_ols_footprint_and_validation(lib):
    from paper_1403_6968_amd import linview as L
    f = L.load().lv_ols_footprint
    a = f(2000, 1000, 4, L.LV_FP32)
    # X (m x n), W (n x n) and the four double n x n creation buffers
    assert a >= 2048 * 1024 * 4 + 1024 * 1024 * 4 + 4 * 1024 * 1024 * 8
    assert f(2000, 1000, 4, L.LV_FP64) > a
    assert f(999, 1000, 4, L.LV_FP32) == 0          # m < n
    assert f(2000, 1000, 65, L.LV_FP32) == 0        # p > 64
    assert f(2000, 1000, 0, L.LV_FP32) == 0
    assert f(70000, 40000, 1, L.LV_FP32) == 0       # n > 32768
    assert f(2000, 1000, 4, L.LV_FP32_BF16SHADOW) == 0
    h = ctypes.c_void_p()
    st = lib.lv_ols_create(0x1000, 10, 20, 20, 0x1000, 1, 1, L.LV_FP32, 0x1000, 1 << 30, None, ctypes.byref(h))
    assert st == L.LV_EINVAL and "m = 10" in L.lv_last_error()
    need = f(512, 256, 2, L.LV_FP32)
    st = lib.lv_ols_create(0x1000, 512, 256, 256, 0x1000, 2, 2, L.LV_FP32, 0x1000, need - 1, None, ctypes.byref(h))
    assert st == L.LV_ENOMEM and str(need) in L.lv_last_error()
    assert lib.lv_ols_update(None, 0x1000, 0x1000, None) == L.LV_EINVAL
    assert lib.lv_ols_update_row(None, 0, 0x1000, None) == L.LV_EINVAL
    assert lib.lv_ols_read(None, 0, 0x1000, 1, None) == L.LV_EINVAL


def test_glin_footprint_and_validation(lib):
    from paper_1403_6968_amd import linview as L
    f = L.load().lv_glin_footprint
    n_pad = 1024
    re = f(1000, 16, 1, L.LV_FP32, 4, L.LV_GLIN_REEVAL)
    hy = f(1000, 16, 1, L.LV_FP32, 4, L.LV_GLIN_HYBRID)
    inc = f(1000, 16, 1, L.LV_FP32, 4, L.LV_GLIN_INCR)
    # A (FP32) and its FP64 copy, T_0 .. T_16 and B
    assert re >= n_pad * n_pad * 12 + 18 * n_pad * 4 * 4
    assert hy > re and inc > re
    assert f(1000, 12, 1, L.LV_FP32, 4, L.LV_GLIN_HYBRID) > 0            # any k
    assert f(1000, 257, 1, L.LV_FP32, 4, L.LV_GLIN_HYBRID) == 0
    assert f(1000, 16, 1, L.LV_FP32, 4097, L.LV_GLIN_REEVAL) == 0
    assert f(1000, 16, 16, L.LV_FP32, 4, L.LV_GLIN_INCR) == 0             # k * r_pad > 128
    assert f(1000, 16, 1, L.LV_FP32, 4, 3) == 0
    assert f(1000, 16, 1, L.LV_FP32_BF16SHADOW, 4, L.LV_GLIN_HYBRID) == 0
    h = ctypes.c_void_p()
    st = lib.lv_glin_create(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, 5, 0x1000, 1 << 30, None,
                            ctypes.byref(h))
    assert st == L.LV_EINVAL and "strategy" in L.lv_last_error()
    need = f(64, 4, 1, L.LV_FP32, 4, L.LV_GLIN_INCR)
    st = lib.lv_glin_create(0x1000, 64, 64, 4, 1, L.LV_FP32, 0x1000, 4, 0x1000, 4, 4, L.LV_GLIN_INCR, 0x1000,
                            need - 1, None, ctypes.byref(h))
    assert st == L.LV_ENOMEM and str(need) in L.lv_last_error()
    assert lib.lv_glin_update(None, 0x1000, 0x1000, 1, 1, 1, None) == L.LV_EINVAL
    assert lib.lv_glin_read(None, 1, 0x1000, 4, None) == L.LV_EINVAL


def test_tune_cache_json_roundtrip(lib, tmp_path):
    """The autotuner's cache persists as a flat JSON object; loading merges,
    saving writes every entry back, bad tile rows are refused."""
    import json
    from paper_1403_6968_amd import linview as L
    L.lv_tune_cache_clear()
    src = tmp_path / "tune.json"
    src.write_text(json.dumps({"gfx950|m1|R8|n:1024:4096": 512, "gfx950|m1|R1|n:8192": 256}))
    assert L.lv_tune_cache_load(str(src)) == 2
    out = tmp_path / "out.json"
    L.lv_tune_cache_save(str(out))
    assert json.loads(out.read_text()) == {"gfx950|m1|R8|n:1024:4096": 512, "gfx950|m1|R1|n:8192": 256}
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"gfx950|m1|R2|n:512": 300}))
    with pytest.raises(L.LinviewError):
        L.lv_tune_cache_load(str(bad))
    with pytest.raises(L.LinviewError):
        L.lv_tune_cache_load(str(tmp_path / "missing.json"))
    L.lv_tune_cache_save(str(out))                     # the failed loads changed nothing
    assert len(json.loads(out.read_text())) == 2
    L.lv_tune_cache_clear()
    L.lv_tune_cache_save(str(out))
    assert json.loads(out.read_text()) == {}
