"""Properties of the seeded input generators (host logic, CPU only)."""
import numpy as np
import pytest

from paper_2602_04430_amd import synth


def test_retained_count_rule():
    assert synth.retained_count(1.0, 517) == 517
    assert synth.retained_count(0.5, 517) == 259          # (500*517+500)//1000
    assert synth.retained_count(0.1, 70) == 7
    assert synth.retained_count(0.1, 30) == 4             # never below the first four rows
    assert synth.retained_count(0.1, 3) == 3              # never above L
    assert synth.retained_count(0.25, 1) == 1
    for L in range(1, 300):
        for r in (0.1, 0.25, 0.5, 1.0):
            k = synth.retained_count(r, L)
            assert min(4, L) <= k <= L


def test_retained_lists_sorted_unique_head_nested():
    L = synth.lengths_lognormal(300, 64, 2, 400, seed=0)
    prev = None
    for r in (1.0, 0.5, 0.25, 0.1):
        idx, off = synth.retained_lists(L, r, seed=0)
        assert off[0] == 0 and off[-1] == len(idx)
        sets = []
        for i, l in enumerate(L):
            s = idx[off[i]:off[i + 1]]
            assert len(s) == synth.retained_count(r, int(l))
            assert np.all(np.diff(s) > 0) and s[0] == 0 and s[-1] < l
            assert np.array_equal(s[:min(4, l)], np.arange(min(4, l)))
            sets.append(set(s.tolist()))
        if prev is not None:
            assert all(a <= b for a, b in zip(sets, prev))        # nested across r
        prev = sets
    full, fo = synth.retained_lists(L, 1.0, seed=0)
    ref, ro = synth.full_lists(L)
    np.testing.assert_array_equal(full, ref)
    np.testing.assert_array_equal(fo, ro)


def test_lengths_and_tokens_deterministic_and_in_range():
    a = synth.make_docs_lognormal(500, 512, 64, 4096, 32000, seed=3)
    b = synth.make_docs_lognormal(500, 512, 64, 4096, 32000, seed=3)
    np.testing.assert_array_equal(a.tokens, b.tokens)
    assert a.lengths.min() >= 64 and a.lengths.max() <= 4096
    assert a.tokens.min() >= 0 and a.tokens.max() < 32000
    assert 300 < np.median(a.lengths) < 800
    u = synth.make_docs_uniform(64, 32, 128, 512, seed=0)
    assert u.lengths.min() >= 32 and u.lengths.max() <= 128 and u.offsets[-1] == u.lengths.sum()


def test_weights_shapes_and_pack_order():
    w = synth.make_weights(synth.TINY, 0)
    flat = synth.pack_weights(synth.TINY, w)
    assert flat.size == synth.TINY.numel()
    assert flat.dtype == np.float32
    np.testing.assert_array_equal(flat[:128], np.ones(128, np.float32))      # L0.attn_norm first
    assert abs(float(np.std(w["L0.wq"])) - 0.02) < 0.002
    w2 = synth.make_weights(synth.TINY, 0)
    np.testing.assert_array_equal(w["head"], w2["head"])


def test_scale_shape_constants():
    s = synth.SCALE
    assert s.kv_elems_per_token() == 32768
    assert abs(s.gemm_flops_per_token() / 1.51e9 - 1) < 0.01
    assert 880e6 < s.numel() < 890e6


def test_join_pairs_distinct_ordered():
    p = synth.join_pairs(100, 500, seed=1)
    assert p.shape == (500, 2)
    assert np.all(p[:, 0] != p[:, 1])
    assert len({tuple(x) for x in p.tolist()}) == 500


def test_mixed_batch_split():
    w = synth.mixed_batch(seed=0, n_docs=300, n_pairs=40)
    n_f, n_m = len(w.extra["filter_docs"]), len(w.extra["map_docs"])
    assert n_f + n_m + (300 - n_f - n_m) == 300 and abs(n_f - n_m) <= 1
    assert w.extra["join_pairs"].min() >= n_f + n_m
