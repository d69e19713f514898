"""Expected-attention compression on the GPU against the FP64 oracle (oracle/compress.py):
the per-row scores written by kvop_kv_build_scored (FP32 path against the plain oracle; BF16
path against the oracle's emulation of the BF16 form, which rounds at the same points), the
retained lists of kvop_ea_select (bit-exact against the oracle's top-k applied to the same
scores, including ties and documents longer than 4096 rows), that scoring leaves the caches
exactly as kvop_kv_build makes them, and the op_eval of a compressed profile.

Tolerances: FP32 scores rtol 1e-3 (the scores are exponentials of D^2-term FP32 sums of
O(10) magnitude: ~1e-4 relative, plus the FP32 forward's own drift); BF16 scores against the
BF16-form emulation rtol 3e-2 (the GPU's FP32 residual stream sends a value near a BF16
rounding midpoint to the other side now and then; one such flip moves an element by 2^-8)."""
import numpy as np
import pytest
import torch

from oracle import codecs
from oracle import compress as oc
from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

SHAPE128 = synth.ModelShape(n_layers=2, d_model=512, n_heads=4, n_kv_heads=2, head_dim=128, d_ffn=1024, vocab=512)
SHAPE64 = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
# lengths: one row, ragged, and beyond 1024 rows (the log-weight pass splits a document's keys
# into 1024-row segments that each recompute the document's statistics)
LENGTHS = np.array([1, 2, 5, 16, 63, 64, 65, 130, 300, 1500, 2100], np.int64)


def _docs(shape, seed, lengths=LENGTHS):
    tokens = np.random.default_rng(seed).integers(0, shape.vocab, int(lengths.sum())).astype(np.int32)
    return synth.Docs(lengths, tokens, np.concatenate([[0], np.cumsum(lengths)]))


def _scored(eng, docs, n_future):
    scores = torch.full((int(docs.lengths.sum()),), float("nan"), dtype=torch.float32, device="cuda")
    h = K.kvop_kv_build_scored(eng.pool, torch.from_numpy(docs.tokens).cuda(), docs.offsets, n_future, scores)
    torch.cuda.synchronize()
    return h, scores


@pytest.mark.parametrize("compute", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [SHAPE128, SHAPE64], ids=["d128", "d64"])
@pytest.mark.parametrize("n_future", [1, 32])
def test_scores_match_oracle(device, compute, shape, n_future):
    w = synth.make_weights(shape, 31, gain_jitter=0.1)
    docs = _docs(shape, 31)
    eng = Engine(shape, w, compute, compute)
    say("ea scores", compute, shape.head_dim, n_future)
    _, scores = _scored(eng, docs, n_future)
    got = scores.cpu().numpy().astype(np.float64)
    eng.close()
    if compute == "f32":
        m, rtol = om.Model(shape, w), 1e-3
    else:
        wb = {k: codecs.bf16_round(v) if v.ndim == 2 else v for k, v in w.items()}
        m, rtol = om.Model(shape, wb, act=codecs.bf16_round), 3e-2
    worst = 0.0
    for i, L in enumerate(docs.lengths):
        ref = oc.ea_scores(m, docs.doc(i), n_future)
        g = got[docs.offsets[i]:docs.offsets[i + 1]]
        err = float(np.max(np.abs(g - ref) / np.maximum(np.abs(ref), 1e-30)))
        worst = max(worst, err)
        np.testing.assert_allclose(g, ref, rtol=rtol, atol=1e-6, err_msg=f"document {i} L {L}")
        np.testing.assert_allclose(g.sum(), shape.n_layers * shape.n_kv_heads, rtol=1e-4)
    say(f"max relative score error {worst:.3g} (bound {rtol})")


def test_select_is_the_exact_top_k_with_ties_and_long_documents(device):
    """Scores from the host (many equal values, zeros, documents up to 9000 rows): the GPU
    lists equal the oracle's top-k of the same float32 values at every r."""
    lengths = np.array([1, 2, 3, 4, 5, 17, 100, 256, 257, 4097, 9000], np.int64)
    rng = np.random.default_rng(5)
    sc = rng.integers(0, 40, int(lengths.sum())).astype(np.float32) * np.float32(0.125)
    sc[:: 7] = 0.0
    offs = np.concatenate([[0], np.cumsum(lengths)])
    eng = Engine(SHAPE64, synth.make_weights(SHAPE64, 1), "f32", "f32", pool_bytes=1 << 24)
    dsc = torch.from_numpy(sc).cuda()
    for r in (1.0, 0.8, 0.5, 0.25, 0.1, 0.0):
        total = sum(K.kvop_retained_count(r, int(L)) for L in lengths)
        idx = torch.full((max(total, 1),), -1, dtype=torch.int32, device="cuda")
        io = K.kvop_ea_select(eng.pool, dsc, offs, r, idx)
        torch.cuda.synchronize()
        got = idx.cpu().numpy()
        for i, L in enumerate(lengths):
            k = synth.retained_count(r, int(L))
            assert io[i + 1] - io[i] == k
            want = oc.ea_select(sc[offs[i]:offs[i + 1]].astype(np.float64), k)
            np.testing.assert_array_equal(got[io[i]:io[i + 1]], want, err_msg=f"r {r} document {i}")
    eng.close()


def test_scored_build_keeps_the_caches_and_drives_compressed_profiles(device):
    """kvop_kv_build_scored builds the same caches as kvop_kv_build (identical op_eval
    logits); its lists at r < 1 are the oracle's top-k of the GPU scores, nested across r; a
    filter over them matches the oracle's filter over the same lists."""
    shape = SHAPE128
    w = synth.make_weights(shape, 32, gain_jitter=0.1)
    docs = _docs(shape, 32)
    suffix = synth.suffix_tokens(16, shape.vocab, seed=32)
    eng = Engine(shape, w, "bf16", "bf16")
    h_plain = eng.build(docs)
    h_sc, scores = _scored(eng, docs, len(suffix))
    full, fo = synth.full_lists(docs.lengths)
    lg_plain, _ = eng.filter(h_plain, full, fo, suffix)
    lg_sc, _ = eng.filter(h_sc, full, fo, suffix)
    np.testing.assert_array_equal(lg_plain, lg_sc)
    sc = scores.cpu().numpy()
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(docs.lengths))]
    prev = None
    for r in (0.5, 0.25, 0.1):
        total = sum(K.kvop_retained_count(r, int(L)) for L in docs.lengths)
        idx = torch.empty(total, dtype=torch.int32, device="cuda")
        io = K.kvop_ea_select(eng.pool, scores, docs.offsets, r, idx)
        torch.cuda.synchronize()
        lists = [idx.cpu().numpy()[io[i]:io[i + 1]] for i in range(len(docs.lengths))]
        for i, L in enumerate(docs.lengths):
            want = oc.ea_select(sc[docs.offsets[i]:docs.offsets[i + 1]].astype(np.float64),
                                synth.retained_count(r, int(L)))
            np.testing.assert_array_equal(lists[i], want)
            if prev is not None:
                assert set(lists[i]) <= set(prev[i])
        prev = lists
        lg, dec = eng.filter(h_sc, np.concatenate(lists), io, suffix, r=r)
        ref = [om.filter_eval(m, caches[i], lists[i], suffix, synth.YES_ID, synth.NO_ID)
               for i in range(len(docs.lengths))]
        E = BOUND[("bf16", "bf16")]
        assert float(np.max(np.abs(lg - np.stack([x.logits for x in ref])))) <= E
        assert decisions_agree_outside_band([x.log_odds for x in ref], dec, E)[0] == 0
    with pytest.raises(K.KvopError):
        _scored(eng, docs, 0)
    eng.close()
