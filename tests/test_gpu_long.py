"""Maximum lengths of the workloads: documents of 8192 rows (the longest of the mixed
workload), filtered at r = 1 and r = 0.1, and joined pairwise at r = 0.25 (the suffix then
sits at positions 16384 + j), against the FP64 oracle, next to a one-row document in the same
call (the shortest)."""
import numpy as np
import pytest

from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

SHAPE = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
LENGTHS = np.array([8192, 1, 8192], np.int64)


@pytest.fixture(scope="module")
def long_setup():
    w = synth.make_weights(SHAPE, 71, gain_jitter=0.1)
    tokens = np.random.default_rng(71).integers(0, SHAPE.vocab, int(LENGTHS.sum())).astype(np.int32)
    docs = synth.Docs(LENGTHS, tokens, np.concatenate([[0], np.cumsum(LENGTHS)]))
    m = om.Model(SHAPE, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(LENGTHS))]
    suffix = synth.suffix_tokens(12, SHAPE.vocab, seed=71)
    return w, docs, m, caches, suffix


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16")])
def test_longest_documents_and_pairs(device, long_setup, compute, kv):
    w, docs, m, caches, suffix = long_setup
    E = BOUND[(compute, kv)]
    eng = Engine(SHAPE, w, compute, kv)
    h = eng.build(docs)
    say("longest documents", compute, kv)
    for r in (1.0, 0.1):
        idx, offs = synth.retained_lists(docs.lengths, r, seed=71)
        lg, dec = eng.filter(h, idx, offs, suffix, r=r)
        ref = [om.filter_eval(m, caches[i], idx[offs[i]:offs[i + 1]], suffix, synth.YES_ID, synth.NO_ID)
               for i in range(len(LENGTHS))]
        err = float(np.max(np.abs(lg - np.stack([x.logits for x in ref]))))
        say(f"r={r}: max-abs logit error {err:.3g} (bound {E})")
        assert err <= E
        assert decisions_agree_outside_band([x.log_odds for x in ref], dec, E)[0] == 0
    idx, offs = synth.retained_lists(docs.lengths, 0.25, seed=72)
    lists = [idx[offs[i]:offs[i + 1]] for i in range(len(LENGTHS))]
    pairs = [(0, 2), (2, 0), (0, 1)]
    jidx = np.concatenate([lists[x] for ab in pairs for x in ab])
    joff = np.concatenate([[0], np.cumsum([len(lists[x]) for ab in pairs for x in ab])])
    hs = np.array([h[x] for ab in pairs for x in ab], np.uint64)
    lg, dec = eng.filter(hs, jidx, joff, suffix, r=0.25, kind=K.KVOP_JOIN)
    ref = [om.join_eval(m, caches[a], lists[a], caches[b], lists[b], suffix, synth.YES_ID, synth.NO_ID)
           for a, b in pairs]
    err = float(np.max(np.abs(lg - np.stack([x.logits for x in ref]))))
    say(f"joins of 8192-row documents at r = 0.25: max-abs logit error {err:.3g} (bound {E})")
    assert err <= E
    assert decisions_agree_outside_band([x.log_odds for x in ref], dec, E)[0] == 0
    eng.close()
