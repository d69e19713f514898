"""The direct-to-LDS attention kernels (every variant) against the FP64 oracle and against the
register-staged kernel: prefill inside kv_build, filter over retained rows at several r
(ragged tiles, documents shorter than one 16-key block, several tiles per document), joins
and map decoding, with a BF16 and an FP8 cache, head_dim 128 and 64."""
import numpy as np
import pytest
import torch

from oracle import codecs
from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

SHAPE128 = synth.ModelShape(n_layers=2, d_model=512, n_heads=4, n_kv_heads=2, head_dim=128, d_ffn=1024, vocab=512)
SHAPE64 = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)


@pytest.fixture
def attention_kernel():
    """Sets the process-wide attention kernel for one test and restores the one before."""
    before = K.kvop_get_attention_kernel()
    yield K.kvop_set_attention_kernel
    K.kvop_set_attention_kernel(before)


def _run_filter(shape, w, docs, suffix, kv, variant, set_kernel, rs):
    set_kernel(variant)
    eng = Engine(shape, w, "bf16", kv)
    handles = eng.build(docs)
    out = {}
    for r in rs:
        idx, offs = synth.retained_lists(docs.lengths, r, seed=21)
        out[r] = eng.filter(handles, idx, offs, suffix, r=r)
    eng.close()
    return out


@pytest.mark.parametrize("kv", ["bf16", "fp8"])
@pytest.mark.parametrize("shape", [SHAPE128, SHAPE64], ids=["d128", "d64"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_dma_attention_filter_matches_oracle_and_register_kernel(device, attention_kernel, variant, shape, kv):
    w = synth.make_weights(shape, 21, gain_jitter=0.1)
    # lengths: shorter than a 16-key block, ragged, and several 64-key tiles
    lengths = np.array([1, 5, 15, 16, 33, 64, 65, 97, 128, 200, 257, 300], np.int64)
    rng = np.random.default_rng(21)
    tokens = rng.integers(0, shape.vocab, int(lengths.sum())).astype(np.int32)
    docs = synth.Docs(lengths, tokens, np.concatenate([[0], np.cumsum(lengths)]))
    suffix = synth.suffix_tokens(16, shape.vocab, seed=21)
    rs = (1.0, 0.5, 0.1)
    say("dma attention", variant, shape.head_dim, kv)
    got = _run_filter(shape, w, docs, suffix, kv, variant, attention_kernel, rs)
    ref_kernel = _run_filter(shape, w, docs, suffix, kv, -1, attention_kernel, rs)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(lengths))]
    E = BOUND[("bf16", kv)]
    exact = kv == "bf16" and (variant in (0, 1) or shape.head_dim == 64)
    for r in rs:
        lg, dec = got[r]
        idx, offs = synth.retained_lists(docs.lengths, r, seed=21)
        ref = [om.filter_eval(m, caches[i], idx[offs[i]:offs[i + 1]], suffix, synth.YES_ID, synth.NO_ID)
               for i in range(len(lengths))]
        err = float(np.max(np.abs(lg - np.stack([x.logits for x in ref]))))
        diff = float(np.max(np.abs(lg - ref_kernel[r][0])))
        say(f"r={r}: error vs oracle {err:.3g} (bound {E}), vs register-staged kernel {diff:.3g}")
        assert err <= E
        assert decisions_agree_outside_band([x.log_odds for x in ref], dec, E)[0] == 0
        if exact:          # same tiles, same arithmetic: the same bits
            assert diff == 0.0
        else:
            assert diff <= E


@pytest.mark.parametrize("kv", ["bf16", "fp8"])
@pytest.mark.parametrize("variant", [1, 2])
def test_dma_attention_join_and_map_match_oracle(device, attention_kernel, variant, kv):
    shape = SHAPE128
    w = synth.make_weights(shape, 22, gain_jitter=0.1)
    docs = synth.make_docs_uniform(8, 1, 150, shape.vocab, seed=22)
    attention_kernel(variant)
    eng = Engine(shape, w, "bf16", kv)
    handles = eng.build(docs)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(8)]
    E = BOUND[("bf16", kv)]
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=22)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(8)]
    # join
    suffix = synth.suffix_tokens(17, shape.vocab, seed=22)
    pairs = synth.join_pairs(8, 10, seed=22)
    idx, offs, hs = [], [0], []
    for a, b in pairs:
        for x in (a, b):
            idx.append(lists[x])
            offs.append(offs[-1] + len(lists[x]))
            hs.append(handles[x])
    say("dma join", variant, kv)
    lg, dec = eng.filter(np.array(hs, np.uint64), np.concatenate(idx), np.array(offs), suffix, r=r, kind=K.KVOP_JOIN)
    lo_ref = []
    for p, (a, b) in enumerate(pairs):
        res = om.join_eval(m, caches[a], lists[a], caches[b], lists[b], suffix, synth.YES_ID, synth.NO_ID)
        assert np.max(np.abs(lg[p] - res.logits)) <= E, p
        lo_ref.append(res.log_odds)
    assert decisions_agree_outside_band(lo_ref, dec, E)[0] == 0
    # map: every step's logits until the texts diverge inside the band
    msuf = synth.suffix_tokens(12, shape.vocab, seed=23)
    lo, nsl, n_gen = 256, 256, 6
    say("dma map", variant, kv)
    mlg, tk = eng.map(handles, idx1, offs1, msuf, lo, nsl, n_gen, r=r)
    for i in range(8):
        res = om.map_eval(m, caches[i], lists[i], msuf, lo, nsl, n_gen)
        srt = np.sort(res.step_logits, axis=1)
        margins = srt[:, -1] - srt[:, -2]
        for t in range(n_gen):
            if not np.array_equal(tk[i, :t], res.tokens[:t]):
                break
            assert np.max(np.abs(mlg[i, t] - res.step_logits[t])) <= E, (i, t)
        if np.all(margins >= 2 * E):
            np.testing.assert_array_equal(tk[i], res.tokens)
    eng.close()


def test_fp8_widening_is_exact_for_every_code(device):
    """The hardware E4M3 -> BF16 conversion of the direct-load kernels, all 256 codes, bit for
    bit against the format's definition (every E4M3 value is a BF16 value; NaN stays NaN)."""
    codes = torch.arange(256, dtype=torch.uint8, device=device)
    out = torch.empty(256, dtype=torch.int16, device=device)
    K.kvop_debug_fp8_to_bf16(codes, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint16)
    ref = codecs.e4m3_decode_table()
    ref_bits = (codecs.bf16_round(ref.astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16)
    finite = np.isfinite(ref)
    np.testing.assert_array_equal(got[finite], ref_bits[finite])
    as_f = (got.astype(np.uint32) << 16).view(np.float32)
    assert np.all(np.isnan(as_f[~finite]))
