"""Pins of the cascade oracle (oracle/cascade.py): its outcome equals Eqs. 1-3 evaluated on the
full table of per-stage decisions (every stage answering every tuple), the processed counts
equal Eq. 4's sums of unsure tuples, and the special cases reduce to plain filters: one stage
is the filter itself; stages that never decide (thresholds +inf / -inf) pass every tuple to
the last stage, whose equal thresholds leave no tuple unsure."""
import numpy as np
import pytest

from oracle import cascade as oca
from oracle import model as om
from paper_2602_04430_amd import synth

MICRO = synth.ModelShape(n_layers=2, d_model=32, n_heads=4, n_kv_heads=2, head_dim=8, d_ffn=64, vocab=64)


@pytest.fixture(scope="module")
def setup():
    m = om.Model(MICRO, synth.make_weights(MICRO, 8, gain_jitter=0.1))
    docs = synth.make_docs_uniform(24, 5, 40, MICRO.vocab, seed=8)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(24)]
    suffix = synth.suffix_tokens(6, MICRO.vocab, seed=8)
    lists = {r: synth.retained_lists(docs.lengths, r, seed=8) for r in (0.1, 0.25, 0.5, 1.0)}
    per = {r: [idx[offs[i]:offs[i + 1]] for i in range(24)] for r, (idx, offs) in lists.items()}
    return m, docs, caches, suffix, per


def _lo(m, caches, lists, suffix):
    return np.array([om.filter_eval(m, c, R, suffix, synth.YES_ID, synth.NO_ID).log_odds
                     for c, R in zip(caches, lists)])


def test_cascade_equals_the_recurrence_on_the_full_decision_table(setup):
    m, docs, caches, suffix, per = setup
    rs = (0.1, 0.25, 0.5, 1.0)
    # thresholds at the 60% quantile of |log-odds| of each early stage, 0 for the last
    th = tuple(float(np.quantile(np.abs(_lo(m, caches, per[r], suffix)), 0.6)) for r in rs[:-1]) + (0.0,)
    stages = [oca.Stage(per[r], t, -t) for r, t in zip(rs, th)]
    res = oca.cascade_filter(m, caches, stages, suffix, synth.YES_ID, synth.NO_ID)
    table = np.stack([[om.decide(lo, t, -t) for lo in _lo(m, caches, per[r], suffix)] for r, t in zip(rs, th)])
    acc, rej, uns, processed = oca.recurrence(table)
    np.testing.assert_array_equal(res.decision == 1, acc == 1)
    np.testing.assert_array_equal(res.decision == 0, rej == 1)
    np.testing.assert_array_equal(res.decision == -1, uns == 1)
    np.testing.assert_array_equal(res.processed, processed)
    assert uns.sum() == 0                       # the last stage's equal thresholds decide everything
    # each tuple's stage is the first whose table entry decides it
    first = np.array([np.flatnonzero(table[:, t] != -1)[0] for t in range(table.shape[1])])
    np.testing.assert_array_equal(res.stage, first)
    assert 0 < processed[-1] < len(caches)      # the ladder really forwards a subset


def test_one_stage_is_the_filter(setup):
    m, docs, caches, suffix, per = setup
    res = oca.cascade_filter(m, caches, [oca.Stage(per[0.25], 0.0, 0.0)], suffix, synth.YES_ID, synth.NO_ID)
    for t, c in enumerate(caches):
        ref = om.filter_eval(m, c, per[0.25][t], suffix, synth.YES_ID, synth.NO_ID)
        assert res.decision[t] == ref.decision
        np.testing.assert_array_equal(res.logits[t], ref.logits)


def test_undeciding_stages_pass_everything_to_the_last(setup):
    m, docs, caches, suffix, per = setup
    stages = [oca.Stage(per[0.1], np.inf, -np.inf), oca.Stage(per[0.5], np.inf, -np.inf), oca.Stage(per[1.0], 0, 0)]
    res = oca.cascade_filter(m, caches, stages, suffix, synth.YES_ID, synth.NO_ID)
    np.testing.assert_array_equal(res.processed, [24, 24, 24])
    np.testing.assert_array_equal(res.stage, np.full(24, 2))
    lo = _lo(m, caches, per[1.0], suffix)
    np.testing.assert_array_equal(res.decision, np.where(lo > 0, 1, np.where(lo < 0, 0, -1)))
