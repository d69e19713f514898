"""FP64 reference of the learned proxy (test infrastructure only).

The proxy is the cheap first stage of a two-stage cascade: it accepts or
rejects a tuple only when it is confident and otherwise passes the tuple on
as unsure to the full KV-cached operator (cascade semantics: paper
Section 4.1, Eqs. 1-3; only unsure tuples reach the next, more expensive
operator).  Its input is the document's pooled cached hidden state; its
labels are the full operator's own decisions.

Network: z = W2 gelu(W1 f + b1) + b2, p = softmax(z); class 1 means "accept".
Loss: mean cross-entropy.  Optimiser: Adam (Kingma and Ba, 2015) with bias
correction, the same optimiser the paper uses for its planner (Section 4.1).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(x: np.ndarray) -> np.ndarray:
    """Exact GELU: x * Phi(x), Phi the standard normal CDF."""
    return 0.5 * x * (1.0 + _erf(np.asarray(x, np.float64) / _SQRT2))


def gelu_grad(x: np.ndarray) -> np.ndarray:
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    x = np.asarray(x, np.float64)
    return 0.5 * (1.0 + _erf(x / _SQRT2)) + x * _INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(p: Dict[str, np.ndarray], f: np.ndarray):
    """Returns (h1, a, z, probs) for features f [n, d_in]."""
    f = np.asarray(f, np.float64)
    h1 = f @ np.asarray(p["w1"], np.float64).T + np.asarray(p["b1"], np.float64)
    a = gelu(h1)
    z = a @ np.asarray(p["w2"], np.float64).T + np.asarray(p["b2"], np.float64)
    zm = z - z.max(axis=1, keepdims=True)
    e = np.exp(zm)
    return h1, a, z, e / e.sum(axis=1, keepdims=True)


def loss_and_grads(p: Dict[str, np.ndarray], f: np.ndarray, y: np.ndarray) -> Tuple[float, Dict[str, np.ndarray]]:
    """Mean cross-entropy over the batch and its analytic gradients."""
    f = np.asarray(f, np.float64)
    y = np.asarray(y, np.int64)
    n = f.shape[0]
    h1, a, z, probs = forward(p, f)
    loss = float(-np.mean(np.log(probs[np.arange(n), y])))
    dz = probs.copy()
    dz[np.arange(n), y] -= 1.0
    dz /= n
    w2 = np.asarray(p["w2"], np.float64)
    g = {"w2": dz.T @ a, "b2": dz.sum(axis=0)}
    dh1 = (dz @ w2) * gelu_grad(h1)
    g["w1"] = dh1.T @ f
    g["b1"] = dh1.sum(axis=0)
    return loss, g


def adam_step(param: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One bias-corrected Adam update at step t (1-based).  Returns (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(p: Dict[str, np.ndarray], f: np.ndarray, tau: float):
    """(class, confidence, answered): answered iff the larger class probability > tau."""
    _, _, _, probs = forward(p, f)
    cls = np.argmax(probs, axis=1)
    conf = probs.max(axis=1)
    return cls, conf, conf > tau
