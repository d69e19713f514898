"""FP64 oracle of query-agnostic cache compression by expected attention.

TEST INFRASTRUCTURE ONLY.  Imported by the tests and nothing else; the GPU library never
imports, calls or links it.

The paper keeps, offline and without knowing any future query, the rows of each document's
cache with the largest expected contribution to attention over possible future queries, by
the Expected Attention method it cites (Section 2.3; Section 5, "Offline" and the choice of
tokens for the compressed profiles).  The method's steps, as read here (each reading is
listed with the repository's design notes):

  1. The queries a future operator will issue at layer l, query head h are modelled as a
     Gaussian whose mean and covariance are those of the document's own pre-rotation
     queries at that layer and head (population covariance over its L rows).
  2. Those queries sit at the n positions right after the document, L .. L+n-1.  The rotary
     embedding is averaged over these positions: per rotated pair j the 2x2 rotation
     becomes [[c, -s], [s, c]] with c, s the means of cos and sin of p * theta_j.  The
     Gaussian is mapped through the averaged rotation R: mean R mu, covariance R Sigma R^T.
  3. For a (rotated) key k the expected un-normalised attention is the Gaussian's moment
     generating function at k / sqrt(D): exp(mu_r . k / sqrt(D) + k^T Sigma_r k / (2 D)).
     Normalised over the document's keys it is the key's expected attention weight.
  4. The key's expected contribution to the attention output is its weight times the norm
     of its value.  The query heads sharing a kv head are averaged.
  5. Every (layer, kv head) is normalised to total 1 and a row's score is the sum over
     layers and kv heads.  A document keeps its k highest-scoring rows (equal scores: the
     lower row first), listed in ascending order; the lists of smaller k are prefixes of
     the same ranking, so the retention ladder is nested.
"""
from __future__ import annotations

import numpy as np

from . import model as om


def averaged_rotation(L: int, n: int, D: int, theta: float):
    """Means over positions p = L .. L+n-1 of cos(p w_j) and sin(p w_j), w_j = theta^(-2j/D)."""
    h = D // 2
    inv = theta ** (-(2.0 * np.arange(h, dtype=np.float64)) / D)
    p = np.arange(L, L + n, dtype=np.float64)
    ang = p[:, None] * inv[None, :]
    return np.cos(ang).mean(axis=0), np.sin(ang).mean(axis=0)


def apply_averaged_rotation(x: np.ndarray, c: np.ndarray, s: np.ndarray) -> np.ndarray:
    """The averaged rotation applied along the last axis (rotate-half pairing (j, j + D/2))."""
    h = x.shape[-1] // 2
    x1, x2 = x[..., :h], x[..., h:]
    return np.concatenate([x1 * c - x2 * s, x2 * c + x1 * s], axis=-1)


def expected_log_weight(mu_r: np.ndarray, sig_r: np.ndarray, K: np.ndarray) -> np.ndarray:
    """log E[exp(q . k / sqrt(D))] for q ~ N(mu_r, sig_r), one value per row k of K [m, D]."""
    D = K.shape[-1]
    lin = K @ mu_r / np.sqrt(D)
    quad = np.einsum("ia,ab,ib->i", K, sig_r, K) / (2.0 * D)
    return lin + quad


def layer_contributions(qt: np.ndarray, k: np.ndarray, v: np.ndarray, L_pos: int, n_future: int,
                        theta: float) -> np.ndarray:
    """Normalised expected contributions of one layer.

    qt [H, L, D]: pre-rotation queries; k [Hkv, L, D]: rotated keys; v [Hkv, L, D].
    Returns [Hkv, L], every row summing to 1."""
    H, L, D = qt.shape
    Hkv = k.shape[0]
    c, s = averaged_rotation(L_pos, n_future, D, theta)
    vnorm = np.sqrt(np.sum(v * v, axis=-1))               # [Hkv, L]
    contrib = np.zeros((Hkv, L))
    for h in range(H):
        g = (h * Hkv) // H
        mu = qt[h].mean(axis=0)
        dev = qt[h] - mu
        sig = dev.T @ dev / L
        mu_r = apply_averaged_rotation(mu, c, s)
        sig_r = apply_averaged_rotation(apply_averaged_rotation(sig, c, s).T, c, s).T
        e = expected_log_weight(mu_r, sig_r, k[g])
        w = np.exp(e - e.max())
        w /= w.sum()
        contrib[g] += w * vnorm[g] / (H // Hkv)
    tot = contrib.sum(axis=1, keepdims=True)
    return np.where(tot > 0, contrib / np.where(tot > 0, tot, 1.0), 1.0 / L)


def ea_scores(m: om.Model, tokens, n_future: int) -> np.ndarray:
    """Per-row expected-attention scores of one document ([L] float64), summed over layers
    and kv heads.  The document is run through the decoder exactly as its cache is built."""
    s = m.s
    toks = np.asarray(tokens)
    L = len(toks)
    x = m.w["embed"][toks]
    pos = np.arange(L, dtype=np.float64)
    causal = np.tril(np.ones((L, L), dtype=bool))
    score = np.zeros(L)
    r = m.act if m.act is not None else (lambda t: t)   # the model's activation format, as in its layers
    for i in range(s.n_layers):
        h = r(om.rmsnorm(x, m.L(i, "attn_norm"), s.rms_eps))
        qt = r(h @ m.L(i, "wq").T).reshape(L, s.n_heads, s.head_dim).transpose(1, 0, 2)
        x, k, v = m.layer(i, x, pos, m.empty_ctx(), m.empty_ctx(), causal)
        score += layer_contributions(qt, k, v, L, n_future, s.rope_theta).sum(axis=0)
    return score


def ea_select(scores: np.ndarray, k: int) -> np.ndarray:
    """Rows kept: the k highest scores, equal scores taken lower row first; ascending."""
    order = np.argsort(-np.asarray(scores, np.float64), kind="stable")
    return np.sort(order[:k]).astype(np.int32)
