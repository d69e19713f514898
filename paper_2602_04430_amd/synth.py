"""Seeded synthetic inputs for the KV-cached semantic operator.

This module only draws random inputs: model weights, document token ids,
instruction suffixes, document lengths and retained-row index lists. It holds
none of the operator's arithmetic, so both the GPU library's callers and the
CPU oracle can take their inputs from it without sharing any computation.

Shapes and distributions follow the workloads the operator is evaluated on:
a small decoder (2 layers, d_model 128) over 64 short documents, and a
16-layer, d_model 2048 GQA decoder over thousands of documents with
log-normally distributed lengths.  The paper evaluates on document
collections of roughly a thousand items each (Section 6, datasets); those
collections are not available, and these seeded synthetic documents stand in
for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

WEIGHT_STD = 0.02

# Stream ids for SeedSequence spawn keys: each kind of input draws from its
# own independent stream, so adding one input never shifts another.
_S_WEIGHTS, _S_LENGTHS, _S_TOKENS, _S_SUFFIX, _S_RETAIN, _S_PROXY, _S_PAIRS, _S_TOPICS = range(8)


@dataclass(frozen=True)
class ModelShape:
    """Llama-style pre-norm decoder shape (no biases, untied head)."""
    n_layers: int
    d_model: int
    n_heads: int
    n_kv_heads: int
    head_dim: int
    d_ffn: int
    vocab: int
    rms_eps: float = 1e-5
    rope_theta: float = 10000.0

    @property
    def group(self) -> int:
        return self.n_heads // self.n_kv_heads

    def layer_shapes(self) -> List[Tuple[str, Tuple[int, ...]]]:
        d, hd = self.d_model, self.head_dim
        return [
            ("attn_norm", (d,)),
            ("wq", (self.n_heads * hd, d)),
            ("wk", (self.n_kv_heads * hd, d)),
            ("wv", (self.n_kv_heads * hd, d)),
            ("wo", (d, self.n_heads * hd)),
            ("ffn_norm", (d,)),
            ("w_gate", (self.d_ffn, d)),
            ("w_up", (self.d_ffn, d)),
            ("w_down", (d, self.d_ffn)),
        ]

    def tail_shapes(self) -> List[Tuple[str, Tuple[int, ...]]]:
        d = self.d_model
        return [("final_norm", (d,)), ("embed", (self.vocab, d)), ("head", (self.vocab, d))]

    def numel(self) -> int:
        n = sum(int(np.prod(s)) for _, s in self.layer_shapes()) * self.n_layers
        return n + sum(int(np.prod(s)) for _, s in self.tail_shapes())

    def kv_elems_per_token(self) -> int:
        return 2 * self.n_layers * self.n_kv_heads * self.head_dim

    def gemm_flops_per_token(self) -> int:
        """2 x (weight elements of all layers' projections)."""
        d, hd, f = self.d_model, self.head_dim, self.d_ffn
        per_layer = d * (self.n_heads + 2 * self.n_kv_heads) * hd + self.n_heads * hd * d + 3 * d * f
        return 2 * per_layer * self.n_layers


# 2 layers, d_model 128, 4 heads of 32, SwiGLU 512, vocab 512 (multi-head).
TINY = ModelShape(n_layers=2, d_model=128, n_heads=4, n_kv_heads=4, head_dim=32, d_ffn=512, vocab=512)
# 16 layers, d_model 2048, 16 query / 8 KV heads of 128, SwiGLU 5632, vocab 32000.
SCALE = ModelShape(n_layers=16, d_model=2048, n_heads=16, n_kv_heads=8, head_dim=128, d_ffn=5632,
                   vocab=32000)

YES_ID = 1
NO_ID = 0
MAP_SLICE = (256, 256)   # (first id, count) of the label vocabulary a map decodes over
MAP_TOKENS = 8


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=tuple(key)))


def make_weights(shape: ModelShape, seed: int = 0, gain_jitter: float = 0.0) -> Dict[str, np.ndarray]:
    """FP32 master weights: matrices ~ N(0, 0.02^2); RMSNorm gains 1 (+ optional jitter).

    Keys: 'L{i}.{name}' for layer tensors, plus 'final_norm', 'embed', 'head'.
    Every tensor has its own seeded stream, keyed by (layer, tensor index).
    """
    out: Dict[str, np.ndarray] = {}
    names = shape.layer_shapes()
    for li in range(shape.n_layers):
        for ti, (name, shp) in enumerate(names):
            out[f"L{li}.{name}"] = _draw(shape, seed, li, ti, name, shp, gain_jitter)
    for ti, (name, shp) in enumerate(shape.tail_shapes()):
        out[name] = _draw(shape, seed, shape.n_layers, ti, name, shp, gain_jitter)
    return out


def _draw(shape, seed, li, ti, name, shp, gain_jitter):
    rng = _rng(seed, _S_WEIGHTS, li, ti)
    if name.endswith("norm"):
        g = np.ones(shp, np.float32)
        if gain_jitter:
            g += np.float32(gain_jitter) * rng.standard_normal(shp, dtype=np.float32)
        return g
    return rng.standard_normal(shp, dtype=np.float32) * np.float32(WEIGHT_STD)


def weight_order(shape: ModelShape) -> List[Tuple[str, Tuple[int, ...]]]:
    """The flat packing order the library's model-create call expects."""
    order = []
    for li in range(shape.n_layers):
        order += [(f"L{li}.{n}", s) for n, s in shape.layer_shapes()]
    return order + list(shape.tail_shapes())


def pack_weights(shape: ModelShape, w: Dict[str, np.ndarray]) -> np.ndarray:
    parts = []
    for name, shp in weight_order(shape):
        a = np.asarray(w[name], np.float32)
        assert a.shape == shp, (name, a.shape, shp)
        parts.append(a.reshape(-1))
    return np.concatenate(parts)


# ----------------------------------------------------------------------------- documents

def lengths_uniform(n: int, lo: int, hi: int, seed: int, stream: int = 0) -> np.ndarray:
    """Document lengths uniform over the integers [lo, hi]."""
    return _rng(seed, _S_LENGTHS, stream).integers(lo, hi + 1, size=n).astype(np.int64)


def lengths_lognormal(n: int, median: float, lo: int, hi: int, seed: int, sigma: float = 1.0,
                      stream: int = 0) -> np.ndarray:
    """L = clip(rint(exp(ln(median) + sigma*z)), lo, hi), z ~ N(0, 1)."""
    z = _rng(seed, _S_LENGTHS, stream).standard_normal(n)
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


def doc_tokens(lengths: Sequence[int], vocab: int, seed: int, stream: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Flat int32 token ids (uniform over the vocabulary) and int64 offsets (n+1)."""
    lengths = np.asarray(lengths, np.int64)
    offsets = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=offsets[1:])
    toks = _rng(seed, _S_TOKENS, stream).integers(0, vocab, size=int(offsets[-1])).astype(np.int32)
    return toks, offsets


def topic_docs(n: int, n_topics: int, topic_size: int, lo: int, hi: int, vocab: int, seed: int,
               stream: int = 0) -> Tuple["Docs", np.ndarray]:
    """Documents about topics: n_topics token sets of topic_size ids each (drawn once per
    seed, shared by every stream); each document picks a topic uniformly and draws its
    tokens uniformly from that topic's set, with a length uniform in [lo, hi].  Returns the
    documents and each document's topic.  Collections of documents on a few subjects are
    what a semantic filter sorts; the topics give the documents the structure a cheap
    model of the pooled document state can learn."""
    trng = _rng(seed, _S_TOPICS, 0)
    topics = np.stack([trng.choice(vocab, topic_size, replace=False) for _ in range(n_topics)])
    rng = _rng(seed, _S_TOPICS, 1 + stream)
    which = rng.integers(0, n_topics, size=n)
    L = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(L, out=offsets[1:])
    toks = np.concatenate([topics[t][rng.integers(0, topic_size, size=int(l))] for t, l in zip(which, L)])
    return Docs(L, toks.astype(np.int32), offsets), which


def suffix_tokens(length: int, vocab: int, seed: int, which: int = 0) -> np.ndarray:
    """An operator's instruction suffix: token ids uniform over the vocabulary."""
    return _rng(seed, _S_SUFFIX, which).integers(0, vocab, size=length).astype(np.int32)


# ----------------------------------------------------------------------------- retained rows

def retained_count(r: float, L: int) -> int:
    """k(r, L): rows kept at retention r; integer arithmetic so 0.1*L has no float ties.

    k = clamp(floor((round(1000 r) * L + 500) / 1000), min(4, L), L).
    """
    rm = int(round(1000.0 * float(r)))
    k = (rm * int(L) + 500) // 1000
    return int(min(max(k, min(4, int(L))), int(L)))


def retained_lists(lengths: Sequence[int], r: float, seed: int, stream: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Seeded retained-row lists: first min(4, L) rows always, the rest uniform without
    replacement from [4, L), sorted ascending.  One permutation per document is drawn from
    the same stream for every r, so the lists are nested: a smaller r keeps a subset.
    Returns flat int32 indices and int64 offsets (n+1).
    """
    lengths = np.asarray(lengths, np.int64)
    rng = _rng(seed, _S_RETAIN, stream)
    out, offs = [], [0]
    for L in lengths:
        L = int(L)
        perm = rng.permutation(max(L - 4, 0)) + 4
        k = retained_count(r, L)
        head = np.arange(min(4, L))
        sel = np.sort(np.concatenate([head, perm[: k - len(head)]])).astype(np.int32)
        out.append(sel)
        offs.append(offs[-1] + len(sel))
    return np.concatenate(out) if out else np.zeros(0, np.int32), np.asarray(offs, np.int64)


def full_lists(lengths: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Explicit identity lists 0..L-1 (retention 1)."""
    lengths = np.asarray(lengths, np.int64)
    offs = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=offs[1:])
    return np.concatenate([np.arange(L, dtype=np.int32) for L in lengths]), offs


def join_pairs(n_docs: int, n_pairs: int, seed: int) -> np.ndarray:
    """Ordered pairs (a, b), a != b, sampled without repeating a pair. int32 [n_pairs, 2]."""
    rng = _rng(seed, _S_PAIRS)
    seen, out = set(), []
    while len(out) < n_pairs:
        a, b = (int(v) for v in rng.integers(0, n_docs, size=2))
        if a != b and (a, b) not in seen:
            seen.add((a, b))
            out.append((a, b))
    return np.asarray(out, np.int32).reshape(-1, 2)


def proxy_init(d_in: int, d_hidden: int, n_out: int, seed: int) -> Dict[str, np.ndarray]:
    """Proxy MLP initial parameters: matrices ~ N(0, 0.02^2), biases 0 (FP32)."""
    rng = _rng(seed, _S_PROXY, 0)
    return {
        "w1": rng.standard_normal((d_hidden, d_in), dtype=np.float32) * np.float32(WEIGHT_STD),
        "b1": np.zeros(d_hidden, np.float32),
        "w2": rng.standard_normal((n_out, d_hidden), dtype=np.float32) * np.float32(WEIGHT_STD),
        "b2": np.zeros(n_out, np.float32),
    }


def proxy_order(n: int, epoch: int, seed: int) -> np.ndarray:
    """Seeded minibatch order for one training epoch."""
    return _rng(seed, _S_PROXY, 1 + epoch).permutation(n).astype(np.int32)


# ----------------------------------------------------------------------------- workloads

@dataclass
class Docs:
    lengths: np.ndarray      # int64 [n]
    tokens: np.ndarray       # int32 [sum L]
    offsets: np.ndarray      # int64 [n+1]

    def doc(self, i: int) -> np.ndarray:
        return self.tokens[self.offsets[i]: self.offsets[i + 1]]

    def subset(self, idx: Sequence[int]) -> "Docs":
        idx = list(idx)
        L = self.lengths[idx]
        offs = np.zeros(len(idx) + 1, np.int64)
        np.cumsum(L, out=offs[1:])
        toks = np.concatenate([self.doc(i) for i in idx]) if idx else np.zeros(0, np.int32)
        return Docs(L.copy(), toks, offs)


@dataclass
class Workload:
    name: str
    shape: ModelShape
    docs: Docs
    suffix: np.ndarray
    r_grid: Tuple[float, ...] = (1.0,)
    extra: dict = field(default_factory=dict)


def make_docs_uniform(n, lo, hi, vocab, seed, stream=0) -> Docs:
    L = lengths_uniform(n, lo, hi, seed, stream)
    t, o = doc_tokens(L, vocab, seed, stream)
    return Docs(L, t, o)


def make_docs_lognormal(n, median, lo, hi, vocab, seed, stream=0, sigma=1.0) -> Docs:
    L = lengths_lognormal(n, median, lo, hi, seed, sigma, stream)
    t, o = doc_tokens(L, vocab, seed, stream)
    return Docs(L, t, o)


def tiny_filter(seed: int = 0) -> Workload:
    """64 documents, lengths uniform in [32, 128], one shared 16-token suffix, r = 1."""
    docs = make_docs_uniform(64, 32, 128, TINY.vocab, seed)
    return Workload("tiny_filter_fp32", TINY, docs, suffix_tokens(16, TINY.vocab, seed), (1.0,))


def scale_filter(seed: int = 0, n: int = 4096) -> Workload:
    """4096 documents, lengths lognormal (median 512, sigma 1) clipped to [64, 4096],
    one shared 32-token suffix, retention r in {1, 0.5, 0.25, 0.1}."""
    docs = make_docs_lognormal(4096, 512, 64, 4096, SCALE.vocab, seed)
    if n != 4096:
        docs = docs.subset(range(n))
    return Workload("scale_filter", SCALE, docs, suffix_tokens(32, SCALE.vocab, seed),
                    (1.0, 0.5, 0.25, 0.1))


def proxy_split(seed: int = 0, n_train: int = 50000, n_eval: int = 20000) -> Tuple[Docs, Docs]:
    """Training and fresh evaluation documents for the proxy, from separate streams,
    with the same length law as the scale workload."""
    tr = make_docs_lognormal(n_train, 512, 64, 4096, SCALE.vocab, seed, stream=101)
    ev = make_docs_lognormal(n_eval, 512, 64, 4096, SCALE.vocab, seed, stream=102)
    return tr, ev


def mixed_batch(seed: int = 0, n_docs: int = 16384, n_pairs: int = 2048) -> Workload:
    """Mixed operators: 16384 documents (lognormal median 384 clipped to [16, 8192]); one
    third filter, one third map, one third join-side documents paired into n_pairs pairs."""
    docs = make_docs_lognormal(n_docs, 384, 16, 8192, SCALE.vocab, seed, stream=201)
    n_f = (n_docs + 2) // 3
    n_m = (n_docs - n_f + 1) // 2
    join_side = np.arange(n_f + n_m, n_docs)
    pairs = join_pairs(len(join_side), n_pairs, seed)
    extra = {
        "filter_docs": np.arange(0, n_f),
        "map_docs": np.arange(n_f, n_f + n_m),
        "join_pairs": join_side[pairs],
        "suffix_map": suffix_tokens(32, SCALE.vocab, seed, which=1),
        "suffix_join": suffix_tokens(32, SCALE.vocab, seed, which=2),
    }
    return Workload("mixed_bf16", SCALE, docs, suffix_tokens(32, SCALE.vocab, seed, which=0), (1.0,),
                    extra)
