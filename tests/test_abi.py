"""The C-ABI library loads and exports every symbol include/kvop.h declares; host-only
calls (no GPU needed) behave as documented."""
import ctypes
import os
import re

import pytest

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "kvop.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kvop_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "kvop_op_eval" in names and "kvop_kv_build" in names
    lib = ctypes.CDLL(K.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_function():
    names = declared_functions()
    missing = [n for n in names if not hasattr(K, n) and n not in ("kvop_last_error",)]
    assert not missing, missing


@pytest.mark.parametrize("shape", [synth.TINY, synth.SCALE])
def test_weights_numel_matches_packing(shape):
    assert K.kvop_weights_numel(K.make_cfg(shape)) == shape.numel()


def test_model_create_rejects_bad_shapes_before_touching_the_device():
    bad = K.make_cfg(synth.TINY)
    bad.head_dim = 48
    out = ctypes.c_void_p()
    st = K.lib().kvop_model_create(ctypes.byref(bad), ctypes.c_void_p(1), 1, 0, None, ctypes.byref(out))
    assert st == K.KVOP_EINVAL and b"head_dim" in K.lib().kvop_last_error()
    bad = K.make_cfg(synth.TINY)
    bad.n_kv_heads = 3
    st = K.lib().kvop_model_create(ctypes.byref(bad), ctypes.c_void_p(1), 1, 0, None, ctypes.byref(out))
    assert st == K.KVOP_EINVAL
    good = K.make_cfg(synth.TINY)
    st = K.lib().kvop_model_create(ctypes.byref(good), ctypes.c_void_p(1), 5, 0, None, ctypes.byref(out))
    assert st == K.KVOP_EINVAL and b"count" in K.lib().kvop_last_error()


def test_gemm_tile_table_is_named():
    for dt in (K.KVOP_F32, K.KVOP_BF16):
        n = K.kvop_gemm_num_tiles(dt)
        assert n >= 3
        names = [K.kvop_gemm_tile_name(dt, t) for t in range(n)]
        assert len(set(names)) == n and all(names)


def test_tuning_table_text_roundtrip():
    """The tuning table is host state: import/export need no device."""
    name = K.kvop_gemm_tile_name(K.KVOP_BF16, 1)
    K.kvop_tuning_import(f"1 2 11264 2048 17 {name}\n")
    assert f"1 2 11264 2048 17 {name}" in K.kvop_tuning_export()
    with pytest.raises(K.KvopError):
        K.kvop_tuning_import("1 2 11264 2048 17 no_such_tile\n")
    K.kvop_gemm_set_tile(K.KVOP_BF16, 2, 11264, 2048, 131072, 0)     # M=131072 -> bucket 17
    assert f"1 2 11264 2048 17 {K.kvop_gemm_tile_name(K.KVOP_BF16, 0)}" in K.kvop_tuning_export()


def test_tile_choice_is_the_tuned_bucket_else_the_default():
    """A projection takes the tuned tile of its own bucket floor(log2 M) only; a row count in
    an untuned bucket, even next to a tuned one, keeps the built-in default for its M (the
    tile that suits M rows, since tile counts and rounds change with M)."""
    bf, N, Kd = K.KVOP_BF16, 11264, 4096        # a shape no other test tunes
    default_big = K.kvop_gemm_pick_tile(bf, 2, 131072, N, Kd)
    default_small = K.kvop_gemm_pick_tile(bf, 2, 4062, N, Kd)
    t17, t12 = 0, 1
    assert default_big not in (t17, t12) and default_small not in (t17, t12)
    K.kvop_gemm_set_tile(bf, 2, N, Kd, 131072, t17)    # bucket 17
    K.kvop_gemm_set_tile(bf, 2, N, Kd, 4096, t12)      # bucket 12
    assert K.kvop_gemm_pick_tile(bf, 2, 131072, N, Kd) == t17
    assert K.kvop_gemm_pick_tile(bf, 2, 262143, N, Kd) == t17     # still bucket 17
    assert K.kvop_gemm_pick_tile(bf, 2, 8191, N, Kd) == t12       # still bucket 12
    assert K.kvop_gemm_pick_tile(bf, 2, 129984, N, Kd) == default_big     # bucket 16
    assert K.kvop_gemm_pick_tile(bf, 2, 4062, N, Kd) == default_small     # bucket 11
    assert K.kvop_gemm_pick_tile(bf, 0, 131072, N, Kd) == default_big     # another epilogue
    assert K.kvop_gemm_pick_tile(bf, 3, 131072, N, Kd) == default_big     # rotary: the store tuning
    K.kvop_gemm_set_tile(bf, 0, N, Kd, 131072, t12)
    assert K.kvop_gemm_pick_tile(bf, 3, 131072, N, Kd) == t12
    assert K.kvop_gemm_pick_tile(bf, 2, 0, N, Kd) == -1 and K.kvop_gemm_pick_tile(7, 2, 64, N, Kd) == -1


def test_attention_kernel_knob_is_host_state_and_checked():
    assert K.kvop_get_attention_kernel() == 2          # default: direct loads, 32-key tiles, 3 stages
    for v in (-1, 0, 1, 2):
        K.kvop_set_attention_kernel(v)
        assert K.kvop_get_attention_kernel() == v
    with pytest.raises(K.KvopError):
        K.kvop_set_attention_kernel(3)
    assert K.kvop_get_attention_kernel() == 2


def test_retained_count_rule_matches_the_input_generator():
    """The library's k(r, L) (used by kvop_ea_select) is the count rule of the seeded lists."""
    for L in (1, 2, 3, 4, 5, 9, 10, 64, 999, 1000, 4096, 65535):
        for r in (0.0, 0.1, 0.25, 0.3, 0.5, 0.8, 0.999, 1.0):
            assert K.kvop_retained_count(r, L) == synth.retained_count(r, L), (r, L)
    assert K.kvop_retained_count(0.5, 0) == -1 and K.kvop_retained_count(1.5, 10) == -1
