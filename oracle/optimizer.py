"""FP64 oracle of the plan optimizer over profiled log-odds.

TEST INFRASTRUCTURE ONLY.  Imported by the tests and nothing else; the GPU library never
imports, calls or links it.

What it computes, in the paper's order (Sections 4.1 and 4.2):

  * A query has m logical filters; filter j is a cascade of candidate physical operators
    o_1 .. o_n (here: the same filter over cache profiles of increasing cost), each with a
    per-tuple cost c_i and, on a profiling sample S, its log-odds per tuple.  The gold plan
    runs only the most expensive operator of every filter; a tuple is in the gold result iff
    every filter's gold operator accepts it.
  * Relaxation (Section 4.1, "Continuous Relaxation" and "Optimizing Tunable Parameters"):
    the indicator "o_i is selected" becomes the pick factor sigma_i = sigmoid(s_i / tau);
    the operator's accept / reject / unsure becomes softmax([LO - theta+, theta- - LO, 0] /
    tau).  Eqs. 1-3 then carry soft accept / reject / unsure values down the cascade, and a
    tuple's cost is sum_i unsure_(i-1) * sigma_i * c_i (Eq. 4 with the selection factor
    the relaxation puts on every operator's contribution).
  * Several filters (Section 4.2, "Multiple Semantic Filters"): the plan accepts a tuple
    iff every filter does; relaxed, the product of the filters' soft accepts.  TP, FP, FN
    (Eqs. 5-7) compare that with the gold result.
  * Bounds (Eqs. 8-9): with a Beta(1, 1) prior the recall posterior is Beta(1 + TP, 1 + FN)
    and its lower bound at credible level alpha is the l with P(Recall >= l) = alpha, i.e.
    the (1 - alpha) quantile; precision likewise with Beta(1 + TP, 1 + FP).
  * Loss (Eqs. 10-13): normalised cost + beta * ReLU(T_P - l_P) + beta * ReLU(T_R - l_R),
    minimised by Adam over (s, theta+, theta-) while tau falls exponentially; at the end
    tau = 0: an operator is selected iff s > 0 and decides by its hard thresholds.
  * Ordering (Section 4.2, "Operator Ordering", Algorithm 1): a subset dynamic programme
    over the selected physical operators with their inter- and intra-operator
    selectivities, keeping the cheapest way to have executed each subset.

The gradient here is the central difference of the loss (the definition, not a derivation).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
from scipy.special import betaincinv, expit


# ----------------------------------------------------------------------------- bounds (Eqs. 8-9)

def beta_lower_bound(a: float, b: float, alpha: float) -> float:
    """l such that P(X >= l) = alpha for X ~ Beta(a, b)."""
    return float(betaincinv(a, b, 1.0 - alpha))


# ----------------------------------------------------------------------------- problem

@dataclass
class Problem:
    log_odds: List[np.ndarray]   # per filter: [n_j, S] profiled log-odds of its operators
    cost: List[np.ndarray]       # per filter: [n_j] per-tuple costs
    gold: List[np.ndarray]       # per filter: [S] 1 iff its gold operator accepts
    target_recall: float
    target_precision: float
    alpha: float


@dataclass
class Options:
    steps: int = 300
    lr: float = 0.05
    beta: float = 10.0          # constraint weight: a violation of 0.1 outweighs the whole cost range
    tau0: float = 1.0
    tau_end: float = 0.02
    theta0: float = 1.0


def n_params(pb: Problem) -> int:
    return 3 * sum(len(c) for c in pb.cost)


def split(pb: Problem, params: np.ndarray):
    """params = per filter, per operator: (s, theta+, theta-), filters in order."""
    out, k = [], 0
    for c in pb.cost:
        n = len(c)
        p = params[k:k + 3 * n].reshape(n, 3)
        out.append((p[:, 0], p[:, 1], p[:, 2]))
        k += 3 * n
    return out


def initial_params(pb: Problem, opts: Options) -> np.ndarray:
    p = []
    for c in pb.cost:
        for _ in range(len(c)):
            p += [0.0, opts.theta0, -opts.theta0]
    return np.array(p, np.float64)


# ----------------------------------------------------------------------------- relaxed cascade

def sigmoid(x):
    return expit(x)


def soft_decisions(lo, theta_pos, theta_neg, tau):
    """softmax([LO - theta+, theta- - LO, 0] / tau) -> (accept, reject, unsure)."""
    z = np.stack([lo - theta_pos, theta_neg - lo, np.zeros_like(lo)]) / tau
    z = z - z.max(axis=0)
    e = np.exp(z)
    e /= e.sum(axis=0)
    return e[0], e[1], e[2]


def relaxed_filter(lo: np.ndarray, cost: np.ndarray, s, theta_pos, theta_neg, tau):
    """Eqs. 1-3 and 4 with pick factors and soft decisions; returns (accept, reject, unsure,
    cost) per tuple after the last operator."""
    S = lo.shape[1]
    acc, rej, uns, c = np.zeros(S), np.zeros(S), np.ones(S), np.zeros(S)
    for i in range(lo.shape[0]):
        sig = sigmoid(s[i] / tau)
        pa, pr, _ = soft_decisions(lo[i], theta_pos[i], theta_neg[i], tau)
        c = c + uns * sig * cost[i]
        acc = acc + uns * sig * pa
        rej = rej + uns * sig * pr
        uns = 1.0 - acc - rej
    return acc, rej, uns, c


def counts(accept: np.ndarray, gold: np.ndarray):
    """Eqs. 5-7: (TP, FP, FN) of the (soft) plan output against the gold result."""
    return float(np.sum(accept * gold)), float(np.sum(accept * (1 - gold))), float(np.sum((1 - accept) * gold))


def loss(pb: Problem, params: np.ndarray, tau: float, beta: float) -> float:
    """Eqs. 10-13."""
    S = len(pb.gold[0])
    A = np.ones(S)
    total = np.zeros(S)
    for (s, tp, tn), lo, c in zip(split(pb, params), pb.log_odds, pb.cost):
        acc, _, _, ct = relaxed_filter(lo, c, s, tp, tn, tau)
        A = A * acc
        total = total + ct
    G = np.prod(np.stack(pb.gold), axis=0).astype(np.float64)
    TP, FP, FN = counts(A, G)
    l_cost = total.sum() / (S * sum(float(np.sum(c)) for c in pb.cost))
    l_r = beta_lower_bound(1 + TP, 1 + FN, pb.alpha)
    l_p = beta_lower_bound(1 + TP, 1 + FP, pb.alpha)
    return l_cost + beta * max(pb.target_precision - l_p, 0.0) + beta * max(pb.target_recall - l_r, 0.0)


def grad_fd(pb: Problem, params: np.ndarray, tau: float, beta: float, h: float = 1e-6) -> np.ndarray:
    g = np.zeros_like(params)
    for k in range(len(params)):
        e = np.zeros_like(params)
        e[k] = h
        g[k] = (loss(pb, params + e, tau, beta) - loss(pb, params - e, tau, beta)) / (2 * h)
    return g


def temperature(k: int, opts: Options) -> float:
    """Exponential schedule from tau0 (step 0) to tau_end (last step)."""
    if opts.steps <= 1:
        return opts.tau0
    return opts.tau0 * (opts.tau_end / opts.tau0) ** (k / (opts.steps - 1))


def optimize(pb: Problem, opts: Options, b1=0.9, b2=0.999, eps=1e-8):
    """Adam over the relaxed loss; returns (final params, loss at each step before its update)."""
    p = initial_params(pb, opts)
    m, v = np.zeros_like(p), np.zeros_like(p)
    trace = []
    for k in range(opts.steps):
        tau = temperature(k, opts)
        trace.append(loss(pb, p, tau, opts.beta))
        g = grad_fd(pb, p, tau, opts.beta)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** (k + 1))
        vh = v / (1 - b2 ** (k + 1))
        p = p - opts.lr * mh / (np.sqrt(vh) + eps)
    return p, np.array(trace)


# ----------------------------------------------------------------------------- the plan at tau = 0

@dataclass
class Plan:
    selected: List[np.ndarray]    # per filter: [n_j] bool
    theta_pos: List[np.ndarray]
    theta_neg: List[np.ndarray]


def extract(pb: Problem, params: np.ndarray) -> Plan:
    """tau -> 0: selected iff s > 0; the soft decision becomes the arg-max of [LO - theta+,
    theta- - LO, 0], which is the threshold rule once theta+ >= theta- (if not, both become
    their midpoint, where the arg-max decides every tuple the same way)."""
    sel, tps, tns = [], [], []
    for s, tp, tn in split(pb, params):
        mid = 0.5 * (tp + tn)
        sel.append(s > 0)
        tps.append(np.where(tp >= tn, tp, mid).astype(np.float32))
        tns.append(np.where(tp >= tn, tn, mid).astype(np.float32))
    return Plan(sel, tps, tns)


def hard_decisions(lo, theta_pos, theta_neg):
    """Accept iff LO > theta+, reject iff LO < theta-, else unsure (1 / 0 / -1)."""
    return np.where(lo > theta_pos, 1, np.where(lo < theta_neg, 0, -1))


def evaluate(pb: Problem, plan: Plan):
    """The discrete plan on the sample: per-filter cascades over the selected operators; a
    tuple still unsure after a filter's last selected operator is not accepted.  Returns a
    dict with TP, FP, FN, both bounds, the normalised cost, the per-operator selectivities
    (inter: not rejected, intra: unsure; over the whole sample) and the tuples each
    operator processes in the cascade."""
    S = len(pb.gold[0])
    A = np.ones(S, np.int64)
    total = 0.0
    inter, intra, processed = [], [], []
    for lo, c, sel, tp, tn in zip(pb.log_odds, pb.cost, plan.selected, plan.theta_pos, plan.theta_neg):
        uns = np.ones(S, np.int64)
        acc = np.zeros(S, np.int64)
        for i in range(lo.shape[0]):
            d = hard_decisions(lo[i].astype(np.float32), tp[i], tn[i])
            inter.append(float(np.mean(d != 0)))
            intra.append(float(np.mean(d == -1)))
            if not sel[i]:
                processed.append(0)
                continue
            processed.append(int(uns.sum()))
            total += float(uns.sum()) * float(c[i])
            acc = acc + uns * (d == 1)
            uns = uns * (d == -1)
        A = A * acc
    G = np.prod(np.stack(pb.gold), axis=0)
    TP, FP, FN = counts(A.astype(np.float64), G.astype(np.float64))
    return {"tp": TP, "fp": FP, "fn": FN,
            "recall_lb": beta_lower_bound(1 + TP, 1 + FN, pb.alpha),
            "precision_lb": beta_lower_bound(1 + TP, 1 + FP, pb.alpha),
            "cost_frac": total / (S * sum(float(np.sum(c)) for c in pb.cost)),
            "accept": A, "sel_inter": np.array(inter), "sel_intra": np.array(intra),
            "processed": np.array(processed)}


# ----------------------------------------------------------------------------- ordering (Algorithm 1)

def order_cost(order: Sequence[int], impl, cost, sel_inter, sel_intra, N: float) -> float:
    """Cost of running the physical operators in `order` under the selectivity model: an
    operator processes the tuples still pending for its own logical operator; afterwards its
    own logical operator keeps the intra fraction, every other one the inter fraction."""
    n_log = max(impl) + 1 if len(impl) else 0
    rem = np.full(n_log, float(N))
    c = 0.0
    for o in order:
        j = impl[o]
        c += cost[o] * rem[j]
        f = np.full(n_log, sel_inter[o])
        f[j] = sel_intra[o]
        rem = rem * f
    return c


def dp_reorder(impl, cost, sel_inter, sel_intra, N: float):
    """Subset dynamic programme: for every subset, the cheapest cost of having executed
    exactly it and the pending tuples per logical operator; returns (order, cost)."""
    m = len(impl)
    n_log = max(impl) + 1 if m else 0
    best = {0: (0.0, np.full(n_log, float(N)))}
    parent = {0: None}
    for size in range(m):
        for subset in [x for x in best if bin(x).count("1") == size]:
            c0, rem = best[subset]
            for o in range(m):
                if subset >> o & 1:
                    continue
                nxt = subset | (1 << o)
                j = impl[o]
                c = c0 + cost[o] * rem[j]
                if nxt not in best or c < best[nxt][0]:
                    f = np.full(n_log, sel_inter[o])
                    f[j] = sel_intra[o]
                    best[nxt] = (c, rem * f)
                    parent[nxt] = (subset, o)
    full = (1 << m) - 1
    order, x = [], full
    while parent[x] is not None:
        x, o = parent[x]
        order.append(o)
    return order[::-1], best[full][0]


def brute_force_order(impl, cost, sel_inter, sel_intra, N: float):
    """Minimum of order_cost over every permutation."""
    best = None
    for perm in itertools.permutations(range(len(impl))):
        c = order_cost(perm, impl, cost, sel_inter, sel_intra, N)
        if best is None or c < best[1]:
            best = (list(perm), c)
    return best
