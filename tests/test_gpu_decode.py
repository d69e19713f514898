"""The decoding-step attention kernel (one query position per item, keys and values streamed
from HBM into registers) for every query-head grouping it serves (G = 1, 2, 4 query heads per
kv head), head dims 64 and 128, BF16 and FP8 caches.  A map's greedy decode is checked
against the FP64 oracle (slice logits within E while the texts agree, ids pinned while the
oracle's margins stay outside the band) at r = 1 and 0.5, over documents from 1 row to past
several rounds of the kernel's key batches.  The same map with padded batching must equal
the unpadded call bit for bit."""
import numpy as np
import pytest
import torch

from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, check_map, say

pytestmark = pytest.mark.gpu

# (G, D) -> shape with G = n_heads / n_kv_heads
SHAPES = {
    (1, 128): synth.ModelShape(n_layers=2, d_model=256, n_heads=2, n_kv_heads=2, head_dim=128, d_ffn=512, vocab=512),
    (2, 64): synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512),
    (4, 64): synth.ModelShape(n_layers=2, d_model=512, n_heads=8, n_kv_heads=2, head_dim=64, d_ffn=1024, vocab=512),
    (4, 128): synth.ModelShape(n_layers=2, d_model=1024, n_heads=8, n_kv_heads=2, head_dim=128, d_ffn=1024,
                               vocab=512),
}
LENGTHS = np.array([1, 3, 17, 40, 100, 300], np.int64)
LO, NSL, N_GEN = 256, 256, 5


@pytest.mark.parametrize("kv", ["bf16", "fp8"])
@pytest.mark.parametrize("gd", list(SHAPES), ids=[f"g{g}_d{d}" for g, d in SHAPES])
def test_decode_kernel_map_matches_oracle_and_padded(device, gd, kv):
    shape = SHAPES[gd]
    w = synth.make_weights(shape, 61, gain_jitter=0.1)
    rng = np.random.default_rng(61)
    tokens = rng.integers(0, shape.vocab, int(LENGTHS.sum())).astype(np.int32)
    docs = synth.Docs(LENGTHS, tokens, np.concatenate([[0], np.cumsum(LENGTHS)]))
    suffix = synth.suffix_tokens(7, shape.vocab, seed=61)
    E = BOUND[("bf16", kv)]
    say("decode kernel", gd, kv)
    eng = Engine(shape, w, "bf16", kv)
    h = eng.build(docs)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(len(LENGTHS))]
    n = len(LENGTHS)
    for r in (1.0, 0.5):
        idx, offs = synth.retained_lists(docs.lengths, r, seed=61)
        lg, tk = eng.map(h, idx, offs, suffix, LO, NSL, N_GEN, r=r)
        refs = [om.map_eval(m, caches[i], idx[offs[i]:offs[i + 1]], suffix, LO, NSL, N_GEN) for i in range(n)]
        checked, whole, err, fails = check_map(tk, lg, refs, E)
        say(f"r={r}: max-abs slice-logit error {err:.3g} (bound {E}), ids outside the band checked {checked} of "
            f"{n * N_GEN}")
        assert not fails, fails
        # padded batching: every item iterates over the call's largest list, the extra keys
        # masked; the result must not change in any bit
        outs = []
        for flags in (0, K.KVOP_FLAG_PADDED):
            op = K.make_op(K.KVOP_MAP, suffix, label_lo=LO, label_n=NSL, n_gen=N_GEN, flags=flags)
            plg = torch.full((n, N_GEN, NSL), float("nan"), dtype=torch.float32, device="cuda")
            ptk = torch.full((n, N_GEN), -1, dtype=torch.int32, device="cuda")
            K.kvop_op_eval(eng.pool, op, r, torch.from_numpy(idx).cuda(), offs, h, plg, None, ptk)
            torch.cuda.synchronize()
            outs.append((plg.cpu().numpy(), ptk.cpu().numpy()))
        np.testing.assert_array_equal(outs[1][0], outs[0][0])
        np.testing.assert_array_equal(outs[1][1], outs[0][1])
        np.testing.assert_array_equal(outs[0][1], tk)
    eng.close()
