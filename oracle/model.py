"""FP64 CPU oracle of the KV-cache-backed semantic operators.

TEST INFRASTRUCTURE ONLY.  This package is imported by the tests, by the
package smoke check and by the benchmark's CPU-baseline leg, and by nothing
else: the GPU library and its Python binding never import, call or link it.

What it computes (paper Section 5, "KV cache-enabled Operators"):
  * Offline cache creation: every document is fed once through the decoder
    and its per-layer keys and values are kept (Section 5, "Offline").
  * Online execution: an operator-specific query (the instruction suffix) is
    appended to a document's cached keys/values and one forward pass yields the
    output (Section 5, "Online").  A filter reads the logits of the tokens '1'
    and '0', takes their log-odds and accepts, rejects or marks the tuple
    unsure against two thresholds (Section 5; Section 4.1, soft decisions on
    log-odds, Eq. 14 in its zero-temperature limit).  A map decodes a longer
    output (Section 5).  A join is a filter over pairs drawn from the cartesian
    product (Section 4.2, "Semantic joins").
  * Query-agnostic compression keeps a subset of each document's rows
    (Section 2.3 and Section 5); here that subset is an input list.

The decoder is a Llama-style pre-norm transformer written out plainly:
RMSNorm, rotary position embedding on queries and keys (rotate-half pairing,
base 10000), grouped-query softmax attention with scale 1/sqrt(head_dim),
SwiGLU feed-forward, final RMSNorm and an untied output head, all in float64.
Readings where the paper is silent are listed with the design notes of the
repository (architecture constants, positions after compression, join
geometry, answer token ids, the decision rule at the threshold).

Two routes are provided and kept deliberately different:
  * the cached route (kv_build, then filter_eval / map_eval / join_eval),
  * the recompute route (forward_masked) over the concatenated text with one
    explicit boolean visibility mask; it exists to pin the cached route.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np


# ----------------------------------------------------------------------------- primitives

def rmsnorm(x: np.ndarray, g: np.ndarray, eps: float) -> np.ndarray:
    """Root-mean-square normalisation over the last axis, times the gain."""
    return x / np.sqrt(np.mean(x * x, axis=-1, keepdims=True) + eps) * g


def rope(x: np.ndarray, pos: np.ndarray, theta: float) -> np.ndarray:
    """Rotary embedding: pair (i, i + D/2) rotated by angle pos * theta^(-2i/D).

    x has shape [..., n, D]; pos has n entries (any real positions)."""
    D = x.shape[-1]
    h = D // 2
    inv = theta ** (-(2.0 * np.arange(h, dtype=np.float64)) / D)
    ang = np.asarray(pos, np.float64)[:, None] * inv[None, :]
    c, s = np.cos(ang), np.sin(ang)
    x1, x2 = x[..., :h], x[..., h:]
    return np.concatenate([x1 * c - x2 * s, x2 * c + x1 * s], axis=-1)


def softmax(s: np.ndarray, axis: int = -1) -> np.ndarray:
    m = np.max(s, axis=axis, keepdims=True)
    e = np.exp(s - m)
    return e / np.sum(e, axis=axis, keepdims=True)


def silu(x: np.ndarray) -> np.ndarray:
    return x / (1.0 + np.exp(-x))


def attention(q: np.ndarray, K: np.ndarray, V: np.ndarray, visible: np.ndarray, pround=None) -> np.ndarray:
    """Grouped-query attention.  q [H, n, D]; K, V [Hkv, m, D]; visible [n, m] bool.

    Query head h uses key/value head floor(h * Hkv / H).  pround, when given, is a number
    format applied to the unnormalised probabilities exp(s - max) before they multiply V
    (the normaliser keeps the exact ones); it serves the emulation of a reduced-precision
    form and is off in the plain oracle."""
    H, n, D = q.shape
    Hkv = K.shape[0]
    out = np.empty_like(q)
    for h in range(H):
        kh = (h * Hkv) // H
        s = (q[h] @ K[kh].T) / np.sqrt(D)
        s = np.where(visible, s, -np.inf)
        if pround is None:
            out[h] = softmax(s, axis=-1) @ V[kh]
        else:
            e = np.exp(s - np.max(s, axis=-1, keepdims=True))
            out[h] = (pround(e) @ V[kh]) / np.sum(e, axis=-1, keepdims=True)
    return out


# ----------------------------------------------------------------------------- model

@dataclass
class Shape:
    n_layers: int
    d_model: int
    n_heads: int
    n_kv_heads: int
    head_dim: int
    d_ffn: int
    vocab: int
    rms_eps: float = 1e-5
    rope_theta: float = 10000.0


class Model:
    """Decoder weights promoted to float64.

    Weight keys: 'L{i}.attn_norm', 'L{i}.wq' [H*D, d], 'L{i}.wk' [Hkv*D, d],
    'L{i}.wv', 'L{i}.wo' [d, H*D], 'L{i}.ffn_norm', 'L{i}.w_gate' [F, d],
    'L{i}.w_up' [F, d], 'L{i}.w_down' [d, F], 'final_norm', 'embed' [V, d],
    'head' [V, d].  Linear maps apply as x @ W.T."""

    def __init__(self, shape, weights: Dict[str, np.ndarray], act=None):
        """act (optional): a number format (array -> array of the same shape) applied where
        a reduced-precision implementation rounds the activations: every projection's input
        and output, the rotated queries, the unnormalised attention probabilities and the
        attention output.  None (the oracle proper) keeps float64 throughout."""
        self.s = Shape(shape.n_layers, shape.d_model, shape.n_heads, shape.n_kv_heads,
                       shape.head_dim, shape.d_ffn, shape.vocab, shape.rms_eps, shape.rope_theta)
        self.w = {k: np.asarray(v, np.float64) for k, v in weights.items()}
        self.act = act

    def L(self, i: int, name: str) -> np.ndarray:
        return self.w[f"L{i}.{name}"]

    # one decoder layer over new rows x [n, d] at positions pos, with prior context keys
    # ctxK/ctxV [Hkv, m, D] (already rotated) and visibility [n, m + n] over (context, new rows).
    # store, when given, maps the new rows' keys/values [Hkv, n, D] to what a cache of that
    # number format holds; the attention then reads the stored values, and they are returned.
    def layer(self, i, x, pos, ctxK, ctxV, visible, store=None):
        s = self.s
        n = x.shape[0]
        r = self.act if self.act is not None else (lambda t: t)
        h = r(rmsnorm(x, self.L(i, "attn_norm"), s.rms_eps))
        q = r(h @ self.L(i, "wq").T).reshape(n, s.n_heads, s.head_dim).transpose(1, 0, 2)
        k = r(h @ self.L(i, "wk").T).reshape(n, s.n_kv_heads, s.head_dim).transpose(1, 0, 2)
        v = r(h @ self.L(i, "wv").T).reshape(n, s.n_kv_heads, s.head_dim).transpose(1, 0, 2)
        q = r(rope(q, pos, s.rope_theta))
        k = rope(k, pos, s.rope_theta)
        if store is not None:
            k, v = store(k), store(v)
        K = np.concatenate([ctxK, k], axis=1)
        V = np.concatenate([ctxV, v], axis=1)
        a = r(attention(q, K, V, visible, self.act))
        x = x + a.transpose(1, 0, 2).reshape(n, s.n_heads * s.head_dim) @ self.L(i, "wo").T
        h2 = r(rmsnorm(x, self.L(i, "ffn_norm"), s.rms_eps))
        f = r(silu(h2 @ self.L(i, "w_gate").T) * (h2 @ self.L(i, "w_up").T))
        x = x + f @ self.L(i, "w_down").T
        return x, k, v

    def empty_ctx(self):
        return np.zeros((self.s.n_kv_heads, 0, self.s.head_dim))

    def final(self, x: np.ndarray) -> np.ndarray:
        return rmsnorm(x, self.w["final_norm"], self.s.rms_eps)

    def logits_rows(self, y: np.ndarray, ids: Sequence[int]) -> np.ndarray:
        return y @ self.w["head"][np.asarray(ids)].T


# ----------------------------------------------------------------------------- cached route

@dataclass
class Cache:
    """One document's cache: post-rotation keys and values of every layer."""
    K: np.ndarray        # [layers, Hkv, L, D]
    V: np.ndarray        # [layers, Hkv, L, D]
    pooled: np.ndarray   # [d]: mean over the document's rows of the final-normed hidden state

    @property
    def length(self) -> int:
        return self.K.shape[2]


def kv_build(m: Model, tokens: Sequence[int], store=None) -> Cache:
    """Prefill one document causally at positions 0..L-1 and keep every layer's K and V
    (Section 5, "Offline: KV Cache Creation").

    store (optional) is the cache's number format as a round trip [Hkv, L, D] -> same
    shape (e.g. FP8 blocks, codecs.fp8_cache_roundtrip): every layer keeps the stored
    values, and the document's own causal attention already reads them, as it does when
    the prefill attends over the cache it is writing."""
    toks = np.asarray(tokens)
    L = len(toks)
    x = m.w["embed"][toks]
    pos = np.arange(L)
    causal = np.tril(np.ones((L, L), bool))
    Ks, Vs = [], []
    for i in range(m.s.n_layers):
        x, k, v = m.layer(i, x, pos, m.empty_ctx(), m.empty_ctx(), causal, store)
        Ks.append(k)
        Vs.append(v)
    pooled = m.final(x).mean(axis=0)
    return Cache(np.stack(Ks), np.stack(Vs), pooled)


def decide(lo: float, theta_pos: float, theta_neg: float) -> int:
    """Accept (1) iff log-odds > theta+, reject (0) iff log-odds < theta-, else unsure (-1)."""
    if lo > theta_pos:
        return 1
    if lo < theta_neg:
        return 0
    return -1


@dataclass
class FilterResult:
    logits: np.ndarray   # [2]: logit of the yes token, logit of the no token
    log_odds: float
    decision: int


def _suffix_pass(m: Model, ctxK, ctxV, n_ctx: int, suffix, pos0: int):
    """Run the suffix rows at positions pos0 + j against n_ctx context rows (all visible)
    plus causal suffix rows.  Returns the last hidden row and the suffix K/V per layer."""
    S = len(suffix)
    x = m.w["embed"][np.asarray(suffix)]
    pos = pos0 + np.arange(S)
    vis = np.concatenate([np.ones((S, n_ctx), bool), np.tril(np.ones((S, S), bool))], axis=1)
    sk, sv = [], []
    for i in range(m.s.n_layers):
        x, k, v = m.layer(i, x, pos, ctxK[i], ctxV[i], vis)
        sk.append(k)
        sv.append(v)
    return x, sk, sv


def filter_eval(m: Model, cache: Cache, retained: Sequence[int], suffix: Sequence[int],
                yes_id: int, no_id: int, theta_pos: float = 0.0, theta_neg: float = 0.0) -> FilterResult:
    """Filter over a cached document: the suffix sits after the document's original length
    (positions L + j) and sees the retained cached rows plus the earlier suffix rows."""
    R = np.asarray(retained, np.int64)
    ctxK = [cache.K[i][:, R] for i in range(m.s.n_layers)]
    ctxV = [cache.V[i][:, R] for i in range(m.s.n_layers)]
    x, _, _ = _suffix_pass(m, ctxK, ctxV, len(R), suffix, cache.length)
    y = m.final(x[-1])
    lg = m.logits_rows(y, [yes_id, no_id])
    lo = float(lg[0] - lg[1])
    return FilterResult(lg, lo, decide(lo, theta_pos, theta_neg))


def join_context(m: Model, a: Cache, ra, b: Cache, rb):
    """Context rows of a pair: A's retained rows, then B's retained rows moved to positions
    L_A + p.  B's cached keys carry rotation p; a further rotation by L_A puts them at L_A + p."""
    ra = np.asarray(ra, np.int64)
    rb = np.asarray(rb, np.int64)
    shift = np.full(len(rb), float(a.length))
    ctxK = [np.concatenate([a.K[i][:, ra], rope(b.K[i][:, rb], shift, m.s.rope_theta)], axis=1)
            for i in range(m.s.n_layers)]
    ctxV = [np.concatenate([a.V[i][:, ra], b.V[i][:, rb]], axis=1) for i in range(m.s.n_layers)]
    return ctxK, ctxV, len(ra) + len(rb)


def join_eval(m: Model, a: Cache, ra, b: Cache, rb, suffix, yes_id: int, no_id: int,
              theta_pos: float = 0.0, theta_neg: float = 0.0) -> FilterResult:
    """Join = filter over the pair (A, B): suffix at positions L_A + L_B + j."""
    ctxK, ctxV, n = join_context(m, a, ra, b, rb)
    x, _, _ = _suffix_pass(m, ctxK, ctxV, n, suffix, a.length + b.length)
    y = m.final(x[-1])
    lg = m.logits_rows(y, [yes_id, no_id])
    lo = float(lg[0] - lg[1])
    return FilterResult(lg, lo, decide(lo, theta_pos, theta_neg))


@dataclass
class MapResult:
    tokens: np.ndarray        # [n_gen] decoded ids
    step_logits: np.ndarray   # [n_gen, slice_n] logits over the label slice at every step


def map_eval(m: Model, cache: Cache, retained, suffix, slice_lo: int, slice_n: int,
             n_gen: int) -> MapResult:
    """Map: greedy decode of n_gen ids restricted to the label slice [slice_lo, slice_lo+n).

    Step 1 reads the suffix's last row; each further step feeds the previous id at the next
    position and attends to the retained rows, the suffix and the ids generated so far.
    Ties go to the lowest id."""
    R = np.asarray(retained, np.int64)
    nl = m.s.n_layers
    ctxK = [cache.K[i][:, R] for i in range(nl)]
    ctxV = [cache.V[i][:, R] for i in range(nl)]
    x, sk, sv = _suffix_pass(m, ctxK, ctxV, len(R), suffix, cache.length)
    ctxK = [np.concatenate([ctxK[i], sk[i]], axis=1) for i in range(nl)]
    ctxV = [np.concatenate([ctxV[i], sv[i]], axis=1) for i in range(nl)]
    ids = np.arange(slice_lo, slice_lo + slice_n)
    toks, steps = [], []
    pos = cache.length + len(suffix)
    for t in range(n_gen):
        z = m.logits_rows(m.final(x[-1]), ids)
        g = int(slice_lo + int(np.argmax(z)))
        toks.append(g)
        steps.append(z)
        if t == n_gen - 1:
            break
        x = m.w["embed"][[g]]
        n_ctx = ctxK[0].shape[1]
        vis = np.ones((1, n_ctx + 1), bool)
        for i in range(nl):
            x, k, v = m.layer(i, x, np.array([pos]), ctxK[i], ctxV[i], vis)
            ctxK[i] = np.concatenate([ctxK[i], k], axis=1)
            ctxV[i] = np.concatenate([ctxV[i], v], axis=1)
        pos += 1
    return MapResult(np.asarray(toks, np.int64), np.stack(steps))


# ----------------------------------------------------------------------------- recompute route

def forward_masked(m: Model, tokens, positions, visible) -> np.ndarray:
    """Plain forward over a whole sequence with one explicit visibility mask [n, n]
    (row i may attend to row j iff visible[i, j]) and explicit positions.  Returns the final
    hidden states before the last norm [n, d]."""
    toks = np.asarray(tokens)
    x = m.w["embed"][toks]
    pos = np.asarray(positions)
    for i in range(m.s.n_layers):
        x, _, _ = m.layer(i, x, pos, m.empty_ctx(), m.empty_ctx(), np.asarray(visible, bool))
    return x


def recompute_filter_mask(L: int, S: int, retained) -> np.ndarray:
    """Mask over [document; suffix]: document rows causal over the document; suffix rows see
    the retained document rows and the earlier suffix rows."""
    n = L + S
    vis = np.zeros((n, n), bool)
    vis[:L, :L] = np.tril(np.ones((L, L), bool))
    vis[L:, np.asarray(retained, np.int64)] = True
    vis[L:, L:] = np.tril(np.ones((S, S), bool))
    return vis


def recompute_join_mask(la: int, lb: int, S: int, ra, rb) -> np.ndarray:
    """Mask over [A; B; suffix]: A causal over A, B causal over B only (block-diagonal, as each
    cache is built alone), suffix rows see retained rows of both and earlier suffix rows."""
    n = la + lb + S
    vis = np.zeros((n, n), bool)
    vis[:la, :la] = np.tril(np.ones((la, la), bool))
    vis[la:la + lb, la:la + lb] = np.tril(np.ones((lb, lb), bool))
    s0 = la + lb
    vis[s0:, np.asarray(ra, np.int64)] = True
    vis[s0:, la + np.asarray(rb, np.int64)] = True
    vis[s0:, s0:] = np.tril(np.ones((S, S), bool))
    return vis


def filter_recompute(m: Model, doc, retained, suffix, yes_id, no_id) -> np.ndarray:
    L, S = len(doc), len(suffix)
    toks = np.concatenate([np.asarray(doc), np.asarray(suffix)])
    x = forward_masked(m, toks, np.arange(L + S), recompute_filter_mask(L, S, retained))
    return m.logits_rows(m.final(x[-1]), [yes_id, no_id])
