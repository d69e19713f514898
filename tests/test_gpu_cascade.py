"""The cascade executor (kvop_cascade_eval) over the retention ladder r = 0.1, 0.25, 0.5, 1.

Two properties, each against its own reference:
  * self-consistency with the GPU's own operator: every stage's op_eval over ALL items gives a
    table of decisions; by Eqs. 1-3 an item's outcome is that of the first stage of the table
    that decides it (else the last stage's), and stage i processes the items no earlier stage
    decided (Eq. 4).  The executor must reproduce exactly that, with the logits of the item's
    own stage (bit-exact: the same kernels see the same item).
  * parity with the FP64 oracle's cascade (oracle/cascade.py) on seeded lists: logits within
    the precision's bound at each item's stage, and stage and decision equal wherever no stage
    the item reached has an oracle log-odds within 2E of that stage's thresholds (there a
    result within E cannot flip).
Thresholds are quantiles of |log-odds| per early stage and 0 for the last, so every stage
forwards a real, shrinking subset."""
import numpy as np
import pytest
import torch

from oracle import cascade as oca
from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, say

pytestmark = pytest.mark.gpu

SHAPE = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
RS = (0.1, 0.25, 0.5, 1.0)


def _lists(lengths, seed):
    return {r: synth.retained_lists(lengths, r, seed=seed) for r in RS}


def _thresholds(lo_by_stage, q=0.6):
    # float32-representable, the precision the thresholds have on the GPU
    return [float(np.float32(np.quantile(np.abs(lo), q))) for lo in lo_by_stage[:-1]] + [0.0]


def _cascade(eng, kind, handles, suffix, stages):
    n = len(handles) // (2 if kind == K.KVOP_JOIN else 1)
    op = K.make_op(kind, suffix, synth.YES_ID, synth.NO_ID)
    lg = torch.full((max(n, 1), 2), float("nan"), dtype=torch.float32, device="cuda")
    dec = torch.full((max(n, 1),), 7, dtype=torch.int8, device="cuda")
    stg = torch.full((max(n, 1),), 99, dtype=torch.int8, device="cuda")
    dev = [(r, tp, tn, torch.from_numpy(np.asarray(idx, np.int32)).cuda(), offs) for r, tp, tn, idx, offs in stages]
    proc = K.kvop_cascade_eval(eng.pool, op, dev, handles, lg, dec, stg)
    torch.cuda.synchronize()
    return (lg.cpu().numpy()[:n].astype(np.float64), dec.cpu().numpy()[:n], stg.cpu().numpy()[:n], proc)


def _first_deciding(table):
    """Per item: index of the first stage whose decision is not unsure, else the last stage."""
    n_st, n = table.shape
    out = np.full(n, n_st - 1)
    for t in range(n):
        d = np.flatnonzero(table[:, t] != -1)
        if len(d):
            out[t] = d[0]
    return out


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
def test_executor_is_the_recurrence_over_its_own_stages(device, compute, kv):
    w = synth.make_weights(SHAPE, 41, gain_jitter=0.1)
    docs = synth.make_docs_lognormal(400, 90, 1, 700, SHAPE.vocab, seed=41)
    suffix = synth.suffix_tokens(12, SHAPE.vocab, seed=41)
    eng = Engine(SHAPE, w, compute, kv)
    h = eng.build(docs)
    lists = _lists(docs.lengths, 41)
    say("cascade self-consistency", compute, kv)
    lo = [lg[:, 0] - lg[:, 1] for lg, _ in (eng.filter(h, *lists[r], suffix, r=r) for r in RS)]
    th = _thresholds(lo)
    # the table's decisions are op_eval's own, taken with each stage's thresholds
    full = [eng.filter(h, *lists[r], suffix, r=r, theta=(t, -t)) for r, t in zip(RS, th)]
    table = np.stack([d.astype(np.int64) for _, d in full])
    lg, dec, stg, proc = _cascade(eng, K.KVOP_FILTER, h, suffix,
                                  [(r, t, -t, *lists[r]) for r, t in zip(RS, th)])
    first = _first_deciding(table)
    np.testing.assert_array_equal(stg, first)
    np.testing.assert_array_equal(dec, table[first, np.arange(len(first))])
    want_logits = np.stack([full[s][0][t] for t, s in enumerate(first)])
    np.testing.assert_array_equal(lg, want_logits)
    np.testing.assert_array_equal(proc, [int(np.sum(first >= i)) for i in range(len(RS))])
    assert proc[0] == len(docs.lengths) and 0 < proc[-1] < proc[1] < proc[0], proc
    assert np.all(dec != -1)                           # the last stage's equal thresholds decide
    say("processed per stage", proc.tolist())
    eng.close()


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16")])
def test_filter_cascade_matches_oracle(device, compute, kv):
    w = synth.make_weights(SHAPE, 42, gain_jitter=0.1)
    docs = synth.make_docs_uniform(48, 1, 300, SHAPE.vocab, seed=42)
    suffix = synth.suffix_tokens(10, SHAPE.vocab, seed=42)
    lists = _lists(docs.lengths, 42)
    per = {r: [idx[offs[i]:offs[i + 1]] for i in range(len(docs.lengths))] for r, (idx, offs) in lists.items()}
    m = om.Model(SHAPE, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(docs.lengths))]
    lo_ref = np.array([[om.filter_eval(m, c, R, suffix, synth.YES_ID, synth.NO_ID).log_odds
                        for c, R in zip(caches, per[r])] for r in RS])
    th = _thresholds(list(lo_ref))
    ref = oca.cascade_filter(m, caches, [oca.Stage(per[r], t, -t) for r, t in zip(RS, th)], suffix,
                             synth.YES_ID, synth.NO_ID)
    eng = Engine(SHAPE, w, compute, kv)
    h = eng.build(docs)
    say("cascade vs oracle", compute, kv)
    lg, dec, stg, proc = _cascade(eng, K.KVOP_FILTER, h, suffix, [(r, t, -t, *lists[r]) for r, t in zip(RS, th)])
    eng.close()
    E = BOUND[(compute, kv)]
    # an item is "clear" when no stage it reaches in the oracle's run is within 2E of a threshold
    clear = np.ones(len(caches), bool)
    for t in range(len(caches)):
        for i in range(ref.stage[t] + 1):
            if min(abs(lo_ref[i, t] - th[i]), abs(lo_ref[i, t] + th[i])) < 2 * E:
                clear[t] = False
    np.testing.assert_array_equal(stg[clear], ref.stage[clear])
    np.testing.assert_array_equal(dec[clear], ref.decision[clear])
    same = stg == ref.stage
    err = float(np.max(np.abs(lg[same] - ref.logits[same])))
    assert err <= E, err
    assert np.all(np.abs(proc - ref.processed) <= np.sum(~clear)), (proc, ref.processed)
    if compute == "f32":
        assert clear.mean() > 0.8 and np.array_equal(proc, ref.processed), (clear.mean(), proc, ref.processed)
    say(f"max logit error {err:.3g} (bound {E}); clear items {clear.mean():.2f}; processed {proc.tolist()}")


def test_join_cascade_matches_oracle(device):
    """A join cascade over pairs: the stage lists of A and B as in kvop_op_eval's join form."""
    w = synth.make_weights(SHAPE, 43, gain_jitter=0.1)
    docs = synth.make_docs_uniform(12, 1, 120, SHAPE.vocab, seed=43)
    suffix = synth.suffix_tokens(9, SHAPE.vocab, seed=43)
    pairs = synth.join_pairs(12, 30, seed=43)
    lists = _lists(docs.lengths, 43)
    per = {r: [idx[offs[i]:offs[i + 1]] for i in range(len(docs.lengths))] for r, (idx, offs) in lists.items()}
    m = om.Model(SHAPE, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(docs.lengths))]

    def join_lists(r):
        idx, offs = [], [0]
        for a, b in pairs:
            for x in (a, b):
                idx.append(per[r][x])
                offs.append(offs[-1] + len(per[r][x]))
        return np.concatenate(idx), np.array(offs, np.int64)

    lo_ref = np.array([[om.join_eval(m, caches[a], per[r][a], caches[b], per[r][b], suffix, synth.YES_ID,
                                     synth.NO_ID).log_odds for a, b in pairs] for r in RS])
    th = _thresholds(list(lo_ref))
    eng = Engine(SHAPE, w, "f32", "f32")
    h = eng.build(docs)
    hs = np.array([h[x] for ab in pairs for x in ab], np.uint64)
    say("join cascade vs oracle")
    lg, dec, stg, proc = _cascade(eng, K.KVOP_JOIN, hs, suffix, [(r, t, -t, *join_lists(r)) for r, t in zip(RS, th)])
    eng.close()
    E = BOUND[("f32", "f32")]
    table = np.stack([np.where(l > t, 1, np.where(l < -t, 0, -1)) for l, t in zip(lo_ref, th)])
    assert np.min(np.abs(np.abs(lo_ref) - np.array(th)[:, None])) >= 2 * E   # no item in the band
    first = _first_deciding(table)
    np.testing.assert_array_equal(stg, first)
    np.testing.assert_array_equal(dec, table[first, np.arange(len(pairs))])
    np.testing.assert_array_equal(proc, [int(np.sum(first >= i)) for i in range(len(RS))])
    for t, (a, b) in enumerate(pairs):
        r = RS[first[t]]
        res = om.join_eval(m, caches[a], per[r][a], caches[b], per[r][b], suffix, synth.YES_ID, synth.NO_ID)
        assert np.max(np.abs(lg[t] - res.logits)) <= E


def test_degenerate_cascades(device):
    """One stage is op_eval itself; stages that never decide forward every item to the last;
    no items is a no-op; a map or an empty ladder is rejected."""
    w = synth.make_weights(SHAPE, 44, gain_jitter=0.1)
    docs = synth.make_docs_uniform(40, 1, 200, SHAPE.vocab, seed=44)
    suffix = synth.suffix_tokens(8, SHAPE.vocab, seed=44)
    lists = _lists(docs.lengths, 44)
    eng = Engine(SHAPE, w, "bf16", "bf16")
    h = eng.build(docs)
    say("cascade degenerate cases")
    lg0, dec0 = eng.filter(h, *lists[0.5], suffix, r=0.5, theta=(0.3, -0.3))
    lg, dec, stg, proc = _cascade(eng, K.KVOP_FILTER, h, suffix, [(0.5, 0.3, -0.3, *lists[0.5])])
    np.testing.assert_array_equal(lg, lg0)
    np.testing.assert_array_equal(dec, dec0)
    np.testing.assert_array_equal(stg, 0)
    np.testing.assert_array_equal(proc, [40])
    inf = float("inf")
    lg1, dec1 = eng.filter(h, *lists[1.0], suffix, r=1.0)
    lg, dec, stg, proc = _cascade(eng, K.KVOP_FILTER, h, suffix,
                                  [(0.1, inf, -inf, *lists[0.1]), (0.25, inf, -inf, *lists[0.25]),
                                   (1.0, 0.0, 0.0, *lists[1.0])])
    np.testing.assert_array_equal(proc, [40, 40, 40])
    np.testing.assert_array_equal(stg, 2)
    np.testing.assert_array_equal(lg, lg1)
    np.testing.assert_array_equal(dec, dec1)
    _, _, _, proc = _cascade(eng, K.KVOP_FILTER, np.zeros(0, np.uint64), suffix,
                             [(0.1, 1.0, -1.0, np.zeros(0, np.int32), [0])])
    np.testing.assert_array_equal(proc, [0])
    with pytest.raises(K.KvopError):
        _cascade(eng, K.KVOP_FILTER, h, suffix, [])
    with pytest.raises(K.KvopError):
        _cascade(eng, K.KVOP_FILTER, h, suffix, [(0.5, float("nan"), 0.0, *lists[0.5])])
    # a bad list in a later stage (unsorted rows) is found before any stage runs: outputs untouched
    bad_idx = lists[1.0][0].copy()
    i3 = int(np.flatnonzero(np.diff(lists[1.0][1]) >= 2)[0])
    o0 = int(lists[1.0][1][i3])
    bad_idx[o0], bad_idx[o0 + 1] = bad_idx[o0 + 1], bad_idx[o0]
    op = K.make_op(K.KVOP_FILTER, suffix, synth.YES_ID, synth.NO_ID)
    lg = torch.full((40, 2), 123.0, device="cuda")
    dec = torch.full((40,), 7, dtype=torch.int8, device="cuda")
    stg = torch.full((40,), 9, dtype=torch.int8, device="cuda")
    with pytest.raises(K.KvopError):
        K.kvop_cascade_eval(eng.pool, op, [(0.25, 0.5, -0.5, torch.from_numpy(lists[0.25][0]).cuda(), lists[0.25][1]),
                                           (1.0, 0.0, 0.0, torch.from_numpy(bad_idx).cuda(), lists[1.0][1])],
                            h, lg, dec, stg)
    torch.cuda.synchronize()
    assert bool((lg == 123.0).all()) and bool((dec == 7).all()) and bool((stg == 9).all())
    op = K.make_op(K.KVOP_MAP, suffix, label_lo=0, label_n=4, n_gen=1)
    buf = torch.zeros(40, 2, device="cuda")
    with pytest.raises(K.KvopError):
        K.kvop_cascade_eval(eng.pool, op, [(1.0, 0.0, 0.0, torch.from_numpy(lists[1.0][0]).cuda(), lists[1.0][1])], h,
                            buf, buf, buf)
    eng.close()
