"""Host logic without a GPU: the batching form's grouping of a collection into HBM-sized
groups, the topic-document generator, the choice of the stored oracle samples, the bound
derivation, and the stored full-size oracle values' own consistency."""
import os

import numpy as np
import pytest

from paper_2602_04430_amd import batching
from paper_2602_04430_amd import synth
from tests.golden import make_scale_golden as msg
from tests.golden import scale_bounds as sb


def test_plan_groups_is_the_smallest_count_that_fits():
    rng = np.random.default_rng(0)
    n = 300
    dbytes = rng.integers(1, 100, n)
    f, m = np.arange(0, 100), np.arange(100, 200)
    pairs = rng.integers(200, 300, (40, 2))
    for cap in (dbytes.sum() + 1, 6000, 3000, 1500):
        G = batching.plan_groups(dbytes, f, m, pairs, cap)

        def fits(g_count):
            return all(dbytes[batching.group_docs(*batching.group_parts(f, m, pairs, g_count, g))].sum() <= cap
                       for g in range(g_count))
        assert fits(G) and (G == 1 or not fits(G - 1))
        # every item lands in exactly one group
        parts = [batching.group_parts(f, m, pairs, G, g) for g in range(G)]
        assert np.array_equal(np.concatenate([p[0] for p in parts]), f)
        assert np.array_equal(np.concatenate([p[1] for p in parts]), m)
        assert np.array_equal(np.concatenate([p[2] for p in parts]), pairs)


def test_interleave_and_output_order():
    nf, nm, nj = 7, 5, 3
    op, lst = batching.interleave(nf, nm, nj, seed=4)
    assert sorted(zip(op.tolist(), lst.tolist())) == sorted(
        [(0, i) for i in range(nf)] + [(1, nf + i) for i in range(nm)] + [(2, nf + nm + 2 * i) for i in range(nj)])
    of, om_, oj = batching.output_order(op, lst, nf, nm)
    # output row r of an operator is its r-th item in the interleaved order
    assert list(of) == [l for o, l in zip(op, lst) if o == 0]
    assert list(om_) == [l - nf for o, l in zip(op, lst) if o == 1]
    assert list(oj) == [(l - nf - nm) // 2 for o, l in zip(op, lst) if o == 2]
    assert sorted(of) == list(range(nf)) and sorted(om_) == list(range(nm)) and sorted(oj) == list(range(nj))


def test_topic_docs():
    d0, t0 = synth.topic_docs(200, 16, 4, 32, 128, 512, seed=3, stream=0)
    d1, t1 = synth.topic_docs(100, 16, 4, 32, 128, 512, seed=3, stream=1)
    again, _ = synth.topic_docs(200, 16, 4, 32, 128, 512, seed=3, stream=0)
    assert np.array_equal(d0.tokens, again.tokens)
    assert d0.offsets[-1] == len(d0.tokens) and np.all((d0.lengths >= 32) & (d0.lengths <= 128))
    # documents of one topic draw from one set of 4 ids, shared across streams
    sets = {}
    for docs, topics in ((d0, t0), (d1, t1)):
        for i in range(len(docs.lengths)):
            sets.setdefault(int(topics[i]), set()).update(docs.doc(i).tolist())
    assert all(len(s) <= 4 for s in sets.values()) and len(sets) == 16


def test_stored_samples_are_the_documented_choice():
    wl = synth.scale_filter(0)
    s = msg.filter_sample(wl.docs.lengths)
    L = wl.docs.lengths
    assert len(s) == 64 and s == sorted(s) and len(set(s)) == 64
    assert L[s].min() == L.min() and L[s].max() == L.max()
    fs, ms, ps = msg.mixed_sample(synth.mixed_batch(0))
    mw = synth.mixed_batch(0)
    quarter = len(mw.extra["filter_docs"]) // 4
    assert set(fs) <= set(mw.extra["filter_docs"][:quarter].tolist()) and len(fs) == 8
    assert max(mw.docs.lengths[fs]) == 8192 and len(ms) == 8 and len(ps) == 4


def test_bound_derivation_on_constructed_values():
    ref = {}
    for d, r, base in ((1, 1.0, 0.0), (2, 0.5, 1.0)):
        o = np.array([base, -base])
        ref[(d, r, "fp64")] = o
        ref[(d, r, "bf16w")] = o + 0.01
        ref[(d, r, "bf16form")] = o + 0.01 + np.array([0.02, -0.03])
        ref[(d, r, "fp8fmt")] = o + 0.1
        ref[(d, r, "fp8w")] = o + 0.11
        ref[(d, r, "bf16fp8")] = o + 0.11 + np.array([0.05, 0.0])
    rows, b = sb.derive(ref)
    # N = |emulation - BF16 weights| = 0.03, F = |emulation - oracle| = |(0.03, -0.02)| = 0.03
    assert b["max_N"] == pytest.approx(0.03) and b["max_F"] == pytest.approx(0.03)
    assert b["E_bf16_form"] == pytest.approx(0.06) and b["E_bf16"] == pytest.approx(0.09)
    # N8 = 0.05; the FP8 form sits (0.06, 0.01) from the format oracle, (0.16, 0.11) from the oracle
    assert b["max_fp8_format_effect"] == pytest.approx(0.1) and b["max_N8"] == pytest.approx(0.05)
    assert b["E_fp8_form"] == pytest.approx(0.1) and b["E_fp8_format"] == pytest.approx(0.16)
    assert b["E_fp8"] == pytest.approx(0.26)


def test_stored_mixed_oracle_is_self_consistent():
    """Every stored greedy id is the first arg-max of its stored step's slice logits, the file
    holds exactly the documented items, and the logits are finite."""
    from tests.test_gpu_mixed_scale import load_mixed_oracle
    f, m, j = load_mixed_oracle()
    fs, ms, ps = msg.mixed_sample(synth.mixed_batch(0))
    assert sorted(f) == sorted(fs) and sorted(m) == sorted(ms) and sorted(j) == sorted(ps)
    lo, nl = synth.MAP_SLICE
    for d, ref in m.items():
        assert ref.step_logits.shape == (synth.MAP_TOKENS, nl) and np.all(np.isfinite(ref.step_logits))
        assert np.array_equal(ref.tokens, lo + np.argmax(ref.step_logits, axis=1))
    assert all(np.all(np.isfinite(v)) for v in list(f.values()) + list(j.values()))


@pytest.mark.skipif(not all(os.path.exists(f) for f in [msg.FILTER_FILE] + sb.FP8_VARIANT_FILES),
                    reason="stored filter oracle values not written yet")
def test_stored_filter_oracle_covers_the_sample_and_its_bounds():
    ref, lengths = sb.load_filter_oracle()
    wl = synth.scale_filter(0)
    s = msg.filter_sample(wl.docs.lengths)
    assert sorted(lengths) == s
    for d in s:
        for r in wl.r_grid:
            for v in msg.VARIANTS + msg.FP8_VARIANTS:
                assert np.all(np.isfinite(ref[(d, float(r), v)]))
    b = sb.load_bounds()
    _, again = sb.derive(ref)
    for k, v in again.items():
        assert b[k] == pytest.approx(v, abs=1e-5)
