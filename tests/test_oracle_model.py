"""Pins of the FP64 oracle against things other than itself.

* closed forms (RMSNorm of a constant row, uniform attention when queries are zero),
* rotary embedding against its complex-number form and its relative-position property,
* an independent decoder implementation (HF transformers' Llama in float64 with its SDPA
  attention, additive 4-D masks and explicit positions; its rotary table and RMSNorm, which
  it evaluates in float32, are given float64 arithmetic) for the recompute route,
* invariants tying the cached route to the recompute route: retention 1 equals full
  recompute, retention r < 1 equals a masked recompute, a join equals a block-diagonal
  recompute, every map decode step equals a recompute over the generated text,
* causality and the decision rule.
"""
import numpy as np
import pytest
import torch

from oracle import model as om
from paper_2602_04430_amd import synth

MICRO = synth.ModelShape(n_layers=2, d_model=32, n_heads=4, n_kv_heads=2, head_dim=8, d_ffn=64, vocab=64)


def micro_model(seed=0, jitter=0.1, shape=MICRO):
    return om.Model(shape, synth.make_weights(shape, seed, gain_jitter=jitter))


def rel_err(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


# ----------------------------------------------------------------------------- primitives

def test_rmsnorm_constant_row_closed_form():
    eps = 1e-5
    for c in (0.0, 0.3, -2.5, 7.0):
        g = np.linspace(0.5, 1.5, 16)
        y = om.rmsnorm(np.full(16, c), g, eps)
        np.testing.assert_allclose(y, g * c / np.sqrt(c * c + eps), rtol=1e-14, atol=0)


def test_rmsnorm_unit_rms_and_scale_invariance():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 64)) * 3
    y = om.rmsnorm(x, np.ones(64), 0.0)
    np.testing.assert_allclose(np.sqrt(np.mean(y * y, axis=1)), 1.0, rtol=1e-14)
    np.testing.assert_allclose(om.rmsnorm(7.0 * x, np.ones(64), 0.0), y, rtol=1e-13)


def test_rope_matches_complex_rotation():
    rng = np.random.default_rng(2)
    D, n = 16, 9
    x = rng.standard_normal((3, n, D))
    pos = rng.integers(0, 5000, n).astype(np.float64)
    got = om.rope(x, pos, 10000.0)
    h = D // 2
    freq = 10000.0 ** (-np.arange(0, D, 2) / D)
    z = (x[..., :h] + 1j * x[..., h:]) * np.exp(1j * pos[:, None] * freq[None, :])
    np.testing.assert_allclose(got, np.concatenate([z.real, z.imag], axis=-1), rtol=0, atol=1e-12)


def test_rope_identity_norm_and_relative_position():
    rng = np.random.default_rng(3)
    q, k = rng.standard_normal((1, 1, 32)), rng.standard_normal((1, 1, 32))
    np.testing.assert_array_equal(om.rope(q, np.zeros(1), 1e4), q)
    for p in (1.0, 17.0, 4095.0):
        np.testing.assert_allclose(np.linalg.norm(om.rope(q, np.array([p]), 1e4)), np.linalg.norm(q), rtol=1e-14)
    def dot(p1, p2):
        return float(np.sum(om.rope(q, np.array([p1]), 1e4) * om.rope(k, np.array([p2]), 1e4)))
    for shift in (5.0, 300.0, 8000.0):
        assert abs(dot(40.0, 12.0) - dot(40.0 + shift, 12.0 + shift)) < 1e-12
    # composing rotations adds positions (used by the join geometry)
    a = om.rope(om.rope(k, np.array([12.0]), 1e4), np.array([30.0]), 1e4)
    np.testing.assert_allclose(a, om.rope(k, np.array([42.0]), 1e4), atol=1e-13)


def test_attention_rows_sum_to_one_and_zero_query_is_mean_of_visible_values():
    rng = np.random.default_rng(4)
    H, Hkv, n, m, D = 4, 2, 5, 11, 8
    K = rng.standard_normal((Hkv, m, D))
    V = rng.standard_normal((Hkv, m, D))
    vis = rng.random((n, m)) < 0.6
    vis[:, 0] = True
    # zero queries: every visible score is 0, so the output is the plain mean of the visible rows
    out = om.attention(np.zeros((H, n, D)), K, V, vis)
    for h in range(H):
        for i in range(n):
            np.testing.assert_allclose(out[h, i], V[h // 2][vis[i]].mean(axis=0), rtol=1e-13, atol=1e-15)
    # with one-hot value rows (head_dim = m) the outputs are the attention weights themselves:
    # every row sums to 1 and hidden columns get exactly 0
    q = rng.standard_normal((H, n, m)) * 3
    Kw = rng.standard_normal((Hkv, m, m))
    Vid = np.broadcast_to(np.eye(m), (Hkv, m, m)).copy()
    p = om.attention(q, Kw, Vid, vis)
    np.testing.assert_allclose(p.sum(axis=-1), 1.0, atol=1e-12)
    assert np.all(p[:, ~vis] == 0.0)


def test_attention_matches_scalar_loops():
    rng = np.random.default_rng(5)
    H, Hkv, n, m, D = 4, 2, 3, 6, 4
    q = rng.standard_normal((H, n, D))
    K = rng.standard_normal((Hkv, m, D))
    V = rng.standard_normal((Hkv, m, D))
    vis = np.tril(np.ones((n, m), bool), k=m - n)
    out = om.attention(q, K, V, vis)
    for h in range(H):
        kh = h // (H // Hkv)
        for i in range(n):
            scores = []
            for j in range(m):
                if vis[i, j]:
                    scores.append((j, sum(q[h, i, d] * K[kh, j, d] for d in range(D)) / D ** 0.5))
            mx = max(s for _, s in scores)
            w = [(j, np.exp(s - mx)) for j, s in scores]
            z = sum(e for _, e in w)
            for d in range(D):
                ref = sum(e * V[kh, j, d] for j, e in w) / z
                assert abs(out[h, i, d] - ref) < 1e-13


def test_decision_rule():
    assert om.decide(0.5, 0.0, 0.0) == 1
    assert om.decide(-0.5, 0.0, 0.0) == 0
    assert om.decide(0.0, 0.0, 0.0) == -1          # exactly at the threshold: not accepted
    assert om.decide(0.2, 0.5, -0.5) == -1
    assert om.decide(0.6, 0.5, -0.5) == 1
    assert om.decide(-0.6, 0.5, -0.5) == 0


# ----------------------------------------------------------------------------- independent decoder

def hf_llama(shape, weights):
    from transformers import LlamaConfig, LlamaForCausalLM
    cfg = LlamaConfig(vocab_size=shape.vocab, hidden_size=shape.d_model, intermediate_size=shape.d_ffn,
                      num_hidden_layers=shape.n_layers, num_attention_heads=shape.n_heads,
                      num_key_value_heads=shape.n_kv_heads, head_dim=shape.head_dim,
                      max_position_embeddings=4096, rms_norm_eps=shape.rms_eps, rope_theta=shape.rope_theta,
                      tie_word_embeddings=False, attention_bias=False, mlp_bias=False,
                      attn_implementation="sdpa")
    m = LlamaForCausalLM(cfg).double().eval()
    # HF evaluates the rotary angles in float32; give it a float64 table of the standard
    # rotate-half rotary embedding so the comparison can be held at 1e-12.
    D = shape.head_dim
    inv64 = 1.0 / (shape.rope_theta ** (torch.arange(0, D, 2, dtype=torch.float64) / D))

    def rotary64(x, position_ids):
        freqs = position_ids[..., None].to(torch.float64) * inv64
        emb = torch.cat((freqs, freqs), dim=-1)
        return emb.cos().to(x.dtype), emb.sin().to(x.dtype)

    m.model.rotary_emb.forward = rotary64

    # HF's RMSNorm also upcasts to float32 only; evaluate it in the model's float64
    def norm64(mod):
        def fwd(h):
            return mod.weight * (h * torch.rsqrt(h.pow(2).mean(-1, keepdim=True) + mod.variance_epsilon))
        return fwd

    for mod in m.modules():
        if type(mod).__name__ == "LlamaRMSNorm":
            mod.forward = norm64(mod)
    t = lambda a: torch.tensor(np.asarray(a, np.float64))
    with torch.no_grad():
        m.model.embed_tokens.weight.copy_(t(weights["embed"]))
        m.model.norm.weight.copy_(t(weights["final_norm"]))
        m.lm_head.weight.copy_(t(weights["head"]))
        for i, layer in enumerate(m.model.layers):
            layer.input_layernorm.weight.copy_(t(weights[f"L{i}.attn_norm"]))
            layer.post_attention_layernorm.weight.copy_(t(weights[f"L{i}.ffn_norm"]))
            layer.self_attn.q_proj.weight.copy_(t(weights[f"L{i}.wq"]))
            layer.self_attn.k_proj.weight.copy_(t(weights[f"L{i}.wk"]))
            layer.self_attn.v_proj.weight.copy_(t(weights[f"L{i}.wv"]))
            layer.self_attn.o_proj.weight.copy_(t(weights[f"L{i}.wo"]))
            layer.mlp.gate_proj.weight.copy_(t(weights[f"L{i}.w_gate"]))
            layer.mlp.up_proj.weight.copy_(t(weights[f"L{i}.w_up"]))
            layer.mlp.down_proj.weight.copy_(t(weights[f"L{i}.w_down"]))
    return m


def hf_logits(hf, tokens, positions, visible):
    n = len(tokens)
    mask = torch.zeros(1, 1, n, n, dtype=torch.float64)
    mask[0, 0][~torch.tensor(visible)] = float("-inf")
    with torch.no_grad():
        out = hf(torch.tensor(np.asarray(tokens, np.int64))[None], attention_mask=mask,
                 position_ids=torch.tensor(np.asarray(positions, np.int64))[None])
    return out.logits[0].numpy()


@pytest.mark.parametrize("shape", [MICRO, synth.TINY], ids=["micro_gqa", "tiny"])
def test_recompute_route_matches_hf_llama_causal(shape):
    w = synth.make_weights(shape, 7, gain_jitter=0.2)
    m = om.Model(shape, w)
    hf = hf_llama(shape, w)
    toks = np.random.default_rng(8).integers(0, shape.vocab, 40)
    n = len(toks)
    vis = np.tril(np.ones((n, n), bool))
    x = om.forward_masked(m, toks, np.arange(n), vis)
    ours = m.final(x) @ m.w["head"].T
    ref = hf_logits(hf, toks, np.arange(n), vis)
    assert rel_err(ours, ref) < 1e-12


def test_masked_recompute_matches_hf_llama_with_join_mask_and_shifted_positions():
    w = synth.make_weights(MICRO, 9, gain_jitter=0.2)
    m = om.Model(MICRO, w)
    hf = hf_llama(MICRO, w)
    rng = np.random.default_rng(10)
    la, lb, S = 9, 7, 4
    toks = rng.integers(0, MICRO.vocab, la + lb + S)
    ra = [0, 1, 2, 3, 6]
    rb = [0, 1, 2, 3, 5]
    vis = om.recompute_join_mask(la, lb, S, ra, rb)
    pos = np.arange(la + lb + S)
    x = om.forward_masked(m, toks, pos, vis)
    ours = m.final(x) @ m.w["head"].T
    assert rel_err(ours, hf_logits(hf, toks, pos, vis)) < 1e-12


# ----------------------------------------------------------------------------- cached vs recompute

def _doc(m, L, seed):
    return np.random.default_rng(seed).integers(0, m.s.vocab, L)


@pytest.mark.parametrize("L", [1, 3, 4, 5, 23])
def test_cached_full_retention_equals_recompute(L):
    m = micro_model()
    doc, suffix = _doc(m, L, 11), _doc(m, 5, 12)
    cache = om.kv_build(m, doc)
    r = om.filter_eval(m, cache, np.arange(L), suffix, 1, 0)
    ref = om.filter_recompute(m, doc, np.arange(L), suffix, 1, 0)
    np.testing.assert_allclose(r.logits, ref, rtol=1e-12, atol=1e-14)
    assert r.log_odds == pytest.approx(ref[0] - ref[1], abs=1e-13)


def test_cached_partial_retention_equals_masked_recompute_all_subsets():
    """Every retained subset of a 6-row document that keeps the first 4 rows."""
    m = micro_model(seed=1)
    doc, suffix = _doc(m, 6, 13), _doc(m, 3, 14)
    cache = om.kv_build(m, doc)
    for extra in ([], [4], [5], [4, 5]):
        R = [0, 1, 2, 3] + extra
        got = om.filter_eval(m, cache, R, suffix, 1, 0).logits
        np.testing.assert_allclose(got, om.filter_recompute(m, doc, R, suffix, 1, 0), rtol=1e-12, atol=1e-14)


def test_cached_random_retention_equals_masked_recompute():
    m = micro_model(seed=2)
    L = 40
    doc, suffix = _doc(m, L, 15), _doc(m, 6, 16)
    cache = om.kv_build(m, doc)
    for r in (1.0, 0.5, 0.25, 0.1):
        idx, offs = synth.retained_lists([L], r, seed=3)
        got = om.filter_eval(m, cache, idx, suffix, 1, 0).logits
        np.testing.assert_allclose(got, om.filter_recompute(m, doc, idx, suffix, 1, 0), rtol=1e-12, atol=1e-14)


def test_join_equals_block_diagonal_recompute():
    m = micro_model(seed=3)
    la, lb, S = 13, 9, 4
    da, db, suffix = _doc(m, la, 17), _doc(m, lb, 18), _doc(m, S, 19)
    ca, cb = om.kv_build(m, da), om.kv_build(m, db)
    ra = [0, 1, 2, 3, 5, 8, 12]
    rb = [0, 1, 2, 3, 7]
    got = om.join_eval(m, ca, ra, cb, rb, suffix, 1, 0)
    toks = np.concatenate([da, db, suffix])
    x = om.forward_masked(m, toks, np.arange(la + lb + S), om.recompute_join_mask(la, lb, S, ra, rb))
    ref = m.logits_rows(m.final(x[-1]), [1, 0])
    np.testing.assert_allclose(got.logits, ref, rtol=1e-12, atol=1e-14)


def test_map_every_step_equals_recompute():
    m = micro_model(seed=4)
    L, S, n_gen = 17, 4, 5
    doc, suffix = _doc(m, L, 20), _doc(m, S, 21)
    cache = om.kv_build(m, doc)
    R = [0, 1, 2, 3, 4, 9, 10, 16]
    lo, nsl = 8, 32
    res = om.map_eval(m, cache, R, suffix, lo, nsl, n_gen)
    for t in range(n_gen):
        toks = np.concatenate([doc, suffix, res.tokens[:t]])
        n = len(toks)
        vis = np.zeros((n, n), bool)
        vis[:L, :L] = np.tril(np.ones((L, L), bool))
        vis[L:, R] = True
        vis[L:, L:] = np.tril(np.ones((n - L, n - L), bool))
        x = om.forward_masked(m, toks, np.arange(n), vis)
        z = m.logits_rows(m.final(x[-1]), np.arange(lo, lo + nsl))
        np.testing.assert_allclose(res.step_logits[t], z, rtol=1e-11, atol=1e-13)
        assert res.tokens[t] == lo + int(np.argmax(z))


def test_causality_of_prefill_and_suffix():
    m = micro_model(seed=5)
    doc = _doc(m, 12, 22)
    c0 = om.kv_build(m, doc)
    doc2 = doc.copy()
    doc2[7] = (doc2[7] + 1) % m.s.vocab
    c1 = om.kv_build(m, doc2)
    np.testing.assert_array_equal(c0.K[:, :, :7], c1.K[:, :, :7])
    np.testing.assert_array_equal(c0.V[:, :, :7], c1.V[:, :, :7])
    assert np.max(np.abs(c0.K[:, :, 7:] - c1.K[:, :, 7:])) > 0
    # a suffix row never sees later suffix rows: changing the last token leaves row S-2 unchanged
    s = _doc(m, 5, 23)
    s2 = s.copy()
    s2[-1] = (s2[-1] + 3) % m.s.vocab
    R = np.arange(12)
    x0, _, _ = om._suffix_pass(m, [c0.K[i] for i in range(2)], [c0.V[i] for i in range(2)], 12, s, 12)
    x1, _, _ = om._suffix_pass(m, [c0.K[i] for i in range(2)], [c0.V[i] for i in range(2)], 12, s2, 12)
    np.testing.assert_array_equal(x0[:-1], x1[:-1])
    del R


def test_retention_changes_result_and_unretained_rows_do_not_matter():
    """Rows outside the retained list cannot influence the suffix: overwrite them with noise."""
    m = micro_model(seed=6)
    L = 20
    doc, suffix = _doc(m, L, 24), _doc(m, 4, 25)
    c = om.kv_build(m, doc)
    R = [0, 1, 2, 3, 10, 15]
    base = om.filter_eval(m, c, R, suffix, 1, 0).logits
    noisy = om.Cache(c.K.copy(), c.V.copy(), c.pooled)
    drop = np.setdiff1d(np.arange(L), R)
    noisy.K[:, :, drop] = 99.0
    noisy.V[:, :, drop] = -99.0
    np.testing.assert_array_equal(om.filter_eval(m, noisy, R, suffix, 1, 0).logits, base)
    assert np.max(np.abs(om.filter_eval(m, c, np.arange(L), suffix, 1, 0).logits - base)) > 0


def test_pooled_is_mean_of_final_normed_rows():
    m = micro_model(seed=7)
    doc = _doc(m, 9, 26)
    c = om.kv_build(m, doc)
    x = om.forward_masked(m, doc, np.arange(9), np.tril(np.ones((9, 9), bool)))
    np.testing.assert_allclose(c.pooled, m.final(x).mean(axis=0), rtol=1e-13, atol=1e-15)


def test_oracle_reproduces_stored_tiny_filter_values():
    """Regression pin: the stored values were written by tests/golden/make_golden.py."""
    import os
    from tests.golden.make_golden import tiny_filter_rows
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny_filter_fp64.txt")
    ref = np.loadtxt(path, comments="#")
    got = np.array(tiny_filter_rows(), np.float64)
    np.testing.assert_array_equal(got[:, 0], ref[:, 0])
    np.testing.assert_allclose(got[:, 1:], ref[:, 1:], rtol=0, atol=1e-13)


# ----------------------------------------------------------------------------- cache number formats

def test_kv_build_store_hook_identity_and_zero():
    """With an identity format the cache is unchanged; with a format that stores zeros the
    prefill's own attention reads those zeros, so every layer's attention adds nothing:
    the result equals a model whose output projections are zero."""
    m = micro_model(seed=4)
    doc = _doc(m, 21, 13)
    plain = om.kv_build(m, doc)
    ident = om.kv_build(m, doc, store=lambda a: a)
    np.testing.assert_array_equal(ident.K, plain.K)
    np.testing.assert_array_equal(ident.pooled, plain.pooled)
    zero = om.kv_build(m, doc, store=np.zeros_like)
    w0 = dict(m.w)
    for i in range(m.s.n_layers):
        w0[f"L{i}.wo"] = np.zeros_like(m.w[f"L{i}.wo"])
    no_attn = om.kv_build(om.Model(MICRO, w0), doc)
    np.testing.assert_array_equal(zero.pooled, no_attn.pooled)
    assert np.all(zero.K == 0) and np.all(zero.V == 0)


def test_fp8_format_cache_stays_close_and_is_what_later_layers_see():
    """The FP8 format moves the cache by at most the format's rounding in layer 0 (its
    input does not depend on the cache), and later layers differ from the unquantised
    cache by more than their own rounding because their inputs already saw FP8 values."""
    from oracle import codecs
    m = micro_model(seed=5)
    doc = _doc(m, 40, 14)
    plain = om.kv_build(m, doc)
    q = om.kv_build(m, doc, store=codecs.fp8_cache_roundtrip)
    np.testing.assert_array_equal(q.K[0], codecs.fp8_cache_roundtrip(plain.K[0]))
    np.testing.assert_array_equal(q.V[0], codecs.fp8_cache_roundtrip(plain.V[0]))
    assert not np.array_equal(q.K[1], codecs.fp8_cache_roundtrip(plain.K[1]))
    assert rel_err(q.K, plain.K) < 0.1


def test_reduced_precision_form_hooks():
    """The activation-format hook of the oracle (used to emulate the BF16 form): an identity
    format reproduces the plain oracle up to FP64 reordering; the format is applied at the
    documented points, 8 per layer plus the probabilities of every query head; and the
    layer-0 keys of a BF16 emulation are exactly the BF16 rounding of the rotated BF16-rounded
    projection (RNE at every point, as the kernels round)."""
    from oracle import codecs
    m = micro_model(seed=6)
    doc = _doc(m, 30, 15)
    plain = om.kv_build(m, doc)
    ident = om.kv_build(om.Model(MICRO, m.w, act=lambda t: t), doc)
    np.testing.assert_allclose(ident.K, plain.K, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ident.pooled, plain.pooled, rtol=0, atol=1e-12)
    calls = []

    def spy(t):
        calls.append(t.shape)
        return t

    ms = om.Model(MICRO, m.w, act=spy)
    x = m.w["embed"][np.asarray(doc)]
    pos = np.arange(len(doc), dtype=np.float64)
    causal = np.tril(np.ones((len(doc), len(doc)), bool))
    ms.layer(0, x, pos, ms.empty_ctx(), ms.empty_ctx(), causal)
    assert len(calls) == 8 + MICRO.n_heads
    mb = om.Model(MICRO, m.w, act=codecs.bf16_round)
    cb = om.kv_build(mb, doc, store=codecs.bf16_round)
    h = codecs.bf16_round(om.rmsnorm(x, m.L(0, "attn_norm"), MICRO.rms_eps))
    k = codecs.bf16_round(h @ m.L(0, "wk").T).reshape(len(doc), MICRO.n_kv_heads, MICRO.head_dim).transpose(1, 0, 2)
    np.testing.assert_array_equal(cb.K[0], codecs.bf16_round(om.rope(k, pos, MICRO.rope_theta)))
    assert not np.array_equal(cb.K[1], plain.K[1])
