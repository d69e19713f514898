"""Padded batching (KVOP_FLAG_PADDED): every item's attention iterates over the largest key
count of its wave, loading, multiplying and masking the keys past its own.  Masked keys add
exactly nothing to the online softmax, so every output must equal the unpadded call's
bit for bit: filters, joins, maps and the cascade executor, BF16 and FP8 caches, every
direct-load attention variant.  Combinations without the direct-load kernels are refused."""
import numpy as np
import pytest
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import Engine, say

pytestmark = pytest.mark.gpu

SHAPE128 = synth.ModelShape(n_layers=2, d_model=512, n_heads=4, n_kv_heads=2, head_dim=128, d_ffn=1024, vocab=512)
SHAPE64 = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)


@pytest.fixture
def attention_variant():
    prev = K.kvop_get_attention_kernel()
    yield K.kvop_set_attention_kernel
    K.kvop_set_attention_kernel(prev)


@pytest.mark.parametrize("kv", ["bf16", "fp8"])
@pytest.mark.parametrize("shape", [SHAPE128, SHAPE64], ids=["d128", "d64"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_padded_filter_and_join_equal_unpadded(device, attention_variant, kv, shape, variant):
    attention_variant(variant)
    w = synth.make_weights(shape, 51, gain_jitter=0.1)
    docs = synth.make_docs_lognormal(60, 60, 1, 700, shape.vocab, seed=51)
    suffix = synth.suffix_tokens(11, shape.vocab, seed=51)
    eng = Engine(shape, w, "bf16", kv)
    h = eng.build(docs)
    say("padded filter/join", kv, shape.head_dim, variant)
    for r in (1.0, 0.25):
        idx, offs = synth.retained_lists(docs.lengths, r, seed=51)
        lg0, d0 = eng.filter(h, idx, offs, suffix, r=r, theta=(0.2, -0.2))
        lg1, d1 = eng.filter(h, idx, offs, suffix, r=r, theta=(0.2, -0.2), flags=K.KVOP_FLAG_PADDED)
        np.testing.assert_array_equal(lg1, lg0)
        np.testing.assert_array_equal(d1, d0)
    pairs = synth.join_pairs(60, 40, seed=51)
    lists = [idx[offs[i]:offs[i + 1]] for i in range(60)]
    jidx = np.concatenate([lists[x] for ab in pairs for x in ab])
    joff = np.concatenate([[0], np.cumsum([len(lists[x]) for ab in pairs for x in ab])])
    hs = np.array([h[x] for ab in pairs for x in ab], np.uint64)
    lg0, d0 = eng.filter(hs, jidx, joff, suffix, r=0.25, kind=K.KVOP_JOIN)
    lg1, d1 = eng.filter(hs, jidx, joff, suffix, r=0.25, kind=K.KVOP_JOIN, flags=K.KVOP_FLAG_PADDED)
    np.testing.assert_array_equal(lg1, lg0)
    np.testing.assert_array_equal(d1, d0)
    eng.close()


@pytest.mark.parametrize("kv", ["bf16", "fp8"])
def test_padded_map_and_cascade_equal_unpadded(device, kv):
    shape = SHAPE128
    w = synth.make_weights(shape, 52, gain_jitter=0.1)
    docs = synth.make_docs_uniform(50, 1, 400, shape.vocab, seed=52)
    suffix = synth.suffix_tokens(9, shape.vocab, seed=52)
    eng = Engine(shape, w, "bf16", kv)
    h = eng.build(docs)
    say("padded map/cascade", kv)
    idx, offs = synth.retained_lists(docs.lengths, 0.5, seed=52)
    m = len(h)
    outs = []
    for flags in (0, K.KVOP_FLAG_PADDED):
        op = K.make_op(K.KVOP_MAP, suffix, label_lo=256, label_n=256, n_gen=5, flags=flags)
        lg = torch.full((m, 5, 256), float("nan"), dtype=torch.float32, device="cuda")
        tk = torch.full((m, 5), -1, dtype=torch.int32, device="cuda")
        K.kvop_op_eval(eng.pool, op, 0.5, torch.from_numpy(idx).cuda(), offs, h, lg, None, tk)
        torch.cuda.synchronize()
        outs.append((lg.cpu().numpy(), tk.cpu().numpy()))
    np.testing.assert_array_equal(outs[1][0], outs[0][0])
    np.testing.assert_array_equal(outs[1][1], outs[0][1])
    lists = {r: synth.retained_lists(docs.lengths, r, seed=52) for r in (0.1, 0.5, 1.0)}
    res = []
    for flags in (0, K.KVOP_FLAG_PADDED):
        op = K.make_op(K.KVOP_FILTER, suffix, synth.YES_ID, synth.NO_ID, flags=flags)
        stages = [(r, t, -t, torch.from_numpy(lists[r][0]).cuda(), lists[r][1]) for r, t in
                  ((0.1, 0.8), (0.5, 0.5), (1.0, 0.0))]
        lg = torch.empty(m, 2, device="cuda")
        dec = torch.empty(m, dtype=torch.int8, device="cuda")
        stg = torch.empty(m, dtype=torch.int8, device="cuda")
        proc = K.kvop_cascade_eval(eng.pool, op, stages, h, lg, dec, stg)
        torch.cuda.synchronize()
        res.append((lg.cpu().numpy(), dec.cpu().numpy(), stg.cpu().numpy(), proc))
    for a, b in zip(res[0], res[1]):
        np.testing.assert_array_equal(b, a)
    eng.close()


def test_padded_refused_without_direct_load_kernels(device, attention_variant):
    shape = SHAPE64
    w = synth.make_weights(shape, 53)
    docs = synth.make_docs_uniform(4, 1, 50, shape.vocab, seed=53)
    suffix = synth.suffix_tokens(4, shape.vocab, seed=53)
    full, fo = synth.full_lists(docs.lengths)
    eng = Engine(shape, w, "f32", "f32")
    h = eng.build(docs)
    with pytest.raises(K.KvopError):
        eng.filter(h, full, fo, suffix, flags=K.KVOP_FLAG_PADDED)
    eng.close()
    eng = Engine(shape, w, "bf16", "bf16")
    h = eng.build(docs)
    attention_variant(-1)
    with pytest.raises(K.KvopError):
        eng.filter(h, full, fo, suffix, flags=K.KVOP_FLAG_PADDED)
    eng.close()
