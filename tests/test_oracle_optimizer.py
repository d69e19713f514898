"""Pins of the plan-optimizer oracle (oracle/optimizer.py) against what the paper and the
mathematics fix: the Beta lower bound's closed forms (a = 1 or b = 1) and its defining
integral by quadrature; the paper's worked soft-pick example; the relaxed cascade at low
temperature against the hard recurrence of oracle/cascade.py; the cost term's closed form;
Algorithm 1 against brute force over all orders; and the optimizer's behaviour on problems
whose answer is known (a perfect cheap operator is used, a useless one is not)."""
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import gammaln

from oracle import cascade as oca
from oracle import optimizer as oo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "soft_pick_example.txt")


def test_beta_bound_closed_forms():
    for alpha in (0.5, 0.9, 0.95, 0.99):
        for b in (1.0, 2.0, 7.5, 300.0):
            # Beta(1, b): P(X >= l) = (1 - l)^b
            assert oo.beta_lower_bound(1.0, b, alpha) == pytest.approx(1 - alpha ** (1 / b), rel=1e-12, abs=1e-15)
        for a in (1.0, 3.0, 42.0, 1000.0):
            # Beta(a, 1): P(X >= l) = 1 - l^a
            assert oo.beta_lower_bound(a, 1.0, alpha) == pytest.approx((1 - alpha) ** (1 / a), rel=1e-12)


def test_beta_bound_is_the_defining_integral():
    rng = np.random.default_rng(3)
    for _ in range(12):
        a, b = rng.uniform(1, 400, 2)
        alpha = rng.uniform(0.5, 0.99)
        l = oo.beta_lower_bound(a, b, alpha)
        lnB = gammaln(a) + gammaln(b) - gammaln(a + b)
        dens = lambda x: np.exp((a - 1) * np.log(x) + (b - 1) * np.log1p(-x) - lnB)
        mode = (a - 1) / (a + b - 2)
        upper = integrate.quad(dens, l, 1.0, points=[mode] if l < mode else None, limit=200, epsabs=1e-13)[0]
        assert upper == pytest.approx(alpha, abs=1e-8)


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[f[0]] = f[1:]
    return out


def test_paper_soft_pick_example():
    g = _golden()
    tau = 0.01
    s1 = tau * np.log(float(g["sigma1"][0]) / (1 - float(g["sigma1"][0])))
    s2 = 50.0
    lo = np.array([[-40.0], [40.0]])              # o1 rejects, o2 accepts, far from the thresholds
    acc, rej, uns, cost = oo.relaxed_filter(lo, np.array([1.0, 0.0]), np.array([s1, s2]), np.array([1.0, 0.0]),
                                            np.array([-1.0, 0.0]), tau)
    assert acc[0] == pytest.approx(float(g["accept"][0]), abs=1e-12)
    assert rej[0] == pytest.approx(float(g["reject"][0]), abs=1e-12)
    assert uns[0] == pytest.approx(float(g["unsure"][0]), abs=1e-12)
    assert cost[0] == pytest.approx(float(g["cost_share_op1"][0]), abs=1e-12)   # o1 has unit cost, o2 none
    for key, label in (("label1", 1.0), ("label0", 0.0)):
        tp, fp, fn = oo.counts(acc, np.array([label]))
        f = g[key]
        want = {f[0]: float(f[1]), f[2]: float(f[3]), f[4]: float(f[5])}
        assert (tp, fp, fn) == pytest.approx((want["tp"], want["fp"], want["fn"]), abs=1e-12)


@pytest.mark.parametrize("selected", [(1, 1, 1, 1), (0, 1, 0, 1), (1, 0, 1, 0)])
def test_relaxed_at_low_temperature_is_the_hard_recurrence(selected):
    rng = np.random.default_rng(sum(selected) + 10 * selected[0])
    n, S = 4, 300
    lo = rng.normal(0, 3, (n, S))
    tp, tn = rng.uniform(0.5, 2, n), -rng.uniform(0.5, 2, n)
    # keep tuples away from the thresholds so tau -> 0 has settled
    near = np.any((np.abs(lo - tp[:, None]) < 0.05) | (np.abs(lo - tn[:, None]) < 0.05), axis=0)
    lo = lo[:, ~near]
    cost = rng.uniform(1, 5, n)
    s = np.where(np.array(selected) == 1, 1.0, -1.0)
    tau = 1e-3
    acc, rej, uns, c = oo.relaxed_filter(lo, cost, s, tp, tn, tau)
    rows = [i for i in range(n) if selected[i]]
    table = np.stack([oo.hard_decisions(lo[i], tp[i], tn[i]) for i in rows])
    a, r, u, processed = oca.recurrence(table)
    np.testing.assert_allclose(acc, a, atol=1e-12)
    np.testing.assert_allclose(rej, r, atol=1e-12)
    np.testing.assert_allclose(uns, u, atol=1e-12)
    np.testing.assert_allclose(c.sum(), sum(p * cost[i] for p, i in zip(processed, rows)), rtol=1e-12)


def test_cost_term_closed_form():
    """One filter, one operator, targets 0 (bounds inactive): the loss is the pick factor
    sigmoid(s / tau) itself, and its derivative sigma (1 - sigma) / tau."""
    lo = np.random.default_rng(1).normal(0, 2, (1, 50))
    pb = oo.Problem([lo], [np.array([3.0])], [(lo[0] > 0).astype(np.int8)], 0.0, 0.0, 0.95)
    for s, tau in ((0.3, 1.0), (-0.2, 0.5), (0.05, 0.1)):
        p = np.array([s, 1.0, -1.0])
        sig = 1 / (1 + np.exp(-s / tau))
        assert oo.loss(pb, p, tau, 1.0) == pytest.approx(sig, rel=1e-12)
        g = oo.grad_fd(pb, p, tau, 1.0)
        assert g[0] == pytest.approx(sig * (1 - sig) / tau, rel=1e-6)
        assert abs(g[1]) < 1e-9 and abs(g[2]) < 1e-9      # thresholds do not change the cost of one stage


def test_evaluate_counts_the_cascade():
    rng = np.random.default_rng(7)
    S = 200
    gold_lo = rng.normal(0, 2, S)
    lo = np.stack([gold_lo + rng.normal(0, 1, S), gold_lo + rng.normal(0, 0.5, S), gold_lo])
    pb = oo.Problem([lo], [np.array([1.0, 2.0, 10.0])], [(gold_lo > 0).astype(np.int8)], 0.9, 0.9, 0.95)
    plan = oo.Plan([np.array([True, False, True])], [np.array([1.5, 1.0, 0.0], np.float32)],
                   [np.array([-1.5, -1.0, 0.0], np.float32)])
    ev = oo.evaluate(pb, plan)
    table = np.stack([oo.hard_decisions(lo[i].astype(np.float32), plan.theta_pos[0][i], plan.theta_neg[0][i])
                      for i in (0, 2)])
    a, _, _, processed = oca.recurrence(table)
    np.testing.assert_array_equal(ev["accept"], a)
    np.testing.assert_array_equal(ev["processed"], [processed[0], 0, processed[1]])
    assert ev["cost_frac"] == pytest.approx((processed[0] * 1 + processed[1] * 10) / (S * 13.0))
    G = (gold_lo > 0).astype(np.int64)
    assert ev["tp"] == np.sum(a * G) and ev["fp"] == np.sum(a * (1 - G)) and ev["fn"] == np.sum((1 - a) * G)


def test_dp_reorder_equals_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(40):
        m = int(rng.integers(1, 7))
        n_log = int(rng.integers(1, min(m, 3) + 1))
        impl = list(rng.integers(0, n_log, m))
        cost = rng.uniform(0.1, 10, m)
        sel_intra = rng.uniform(0, 1, m)
        sel_inter = np.maximum(sel_intra, rng.uniform(0, 1, m))   # not rejected >= unsure
        order, c = oo.dp_reorder(impl, cost, sel_inter, sel_intra, 1000.0)
        _, cb = oo.brute_force_order(impl, cost, sel_inter, sel_intra, 1000.0)
        assert sorted(order) == list(range(m))
        assert c == pytest.approx(cb, rel=1e-12)
        assert oo.order_cost(order, impl, cost, sel_inter, sel_intra, 1000.0) == pytest.approx(c, rel=1e-12)


def test_dp_reorder_single_filter_textbook_rule():
    """One logical filter of binary operators (sel_inter = sel_intra = pass fraction): the
    best order sorts by cost / (1 - pass fraction), the classic rule the paper starts from."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        m = 5
        cost = rng.uniform(0.1, 10, m)
        sel = rng.uniform(0.05, 0.95, m)
        order, c = oo.dp_reorder([0] * m, cost, sel, sel, 100.0)
        rank = list(np.argsort(cost / (1 - sel), kind="stable"))
        assert c == pytest.approx(oo.order_cost(rank, [0] * m, cost, sel, sel, 100.0), rel=1e-12)


def _two_op_problem(cheap_noise, S=400, seed=5):
    rng = np.random.default_rng(seed)
    gold_lo = rng.normal(0, 3, S)
    cheap = gold_lo + cheap_noise * rng.normal(0, 1, S) if cheap_noise < 1e6 else rng.normal(0, 3, S)
    lo = np.stack([cheap, gold_lo])
    return oo.Problem([lo], [np.array([1.0, 10.0])], [(gold_lo > 0).astype(np.int8)], 0.9, 0.9, 0.95)


def test_optimizer_uses_a_perfect_cheap_operator():
    pb = _two_op_problem(0.0)
    p, trace = oo.optimize(pb, oo.Options(steps=200))
    ev = oo.evaluate(pb, oo.extract(pb, p))
    assert ev["recall_lb"] >= 0.9 and ev["precision_lb"] >= 0.9
    assert ev["cost_frac"] < 0.25, ev["cost_frac"]          # the cheap operator decides most tuples
    assert trace[-1] < trace[0]


def test_optimizer_ignores_a_useless_cheap_operator():
    pb = _two_op_problem(1e9)
    p, _ = oo.optimize(pb, oo.Options(steps=200))
    plan = oo.extract(pb, p)
    ev = oo.evaluate(pb, plan)
    assert ev["recall_lb"] >= 0.9 and ev["precision_lb"] >= 0.9
    assert plan.selected[0][1]                              # the gold operator stays in the plan
    assert ev["processed"][1] >= 0.8 * 400                  # and sees most tuples


def test_two_filters_gold_plan_is_exact():
    """Two logical filters, each running only its gold operator at thresholds 0: the plan is
    the gold plan (no FP, no FN), its cost is the two gold operators on every tuple, and the
    relaxed loss at low temperature has the same counts (the global result is the AND)."""
    rng = np.random.default_rng(21)
    S = 300
    g1, g2 = rng.normal(0, 2, S), rng.normal(0.5, 2, S)
    g1, g2 = np.where(np.abs(g1) < 0.05, 0.1, g1), np.where(np.abs(g2) < 0.05, 0.1, g2)   # settled at low tau
    lo1 = np.stack([g1 + rng.normal(0, 1, S), g1])
    lo2 = np.stack([g2 + rng.normal(0, 1, S), g2])
    gold = [(g1 > 0).astype(np.int8), (g2 > 0).astype(np.int8)]
    pb = oo.Problem([lo1, lo2], [np.array([1.0, 4.0]), np.array([2.0, 8.0])], gold, 0.9, 0.9, 0.95)
    plan = oo.Plan([np.array([False, True])] * 2, [np.zeros(2, np.float32)] * 2, [np.zeros(2, np.float32)] * 2)
    ev = oo.evaluate(pb, plan)
    G = gold[0] * gold[1]
    assert ev["fp"] == 0 and ev["fn"] == 0 and ev["tp"] == G.sum()
    assert ev["cost_frac"] == pytest.approx((4.0 + 8.0) / 15.0)
    p = np.array([-1, 0, 0, 1, 0, 0, -1, 0, 0, 1, 0, 0], np.float64)
    tau = 1e-3
    L = oo.loss(pb, p, tau, 10.0)
    lr = oo.beta_lower_bound(1 + G.sum(), 1, 0.95)
    assert L == pytest.approx(12.0 / 15.0 + 10 * max(0.9 - lr, 0) * 2, abs=1e-9)
