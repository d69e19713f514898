"""The library's plan optimizer (kvop_plan_*, host code) against the FP64 oracle
(oracle/optimizer.py): the Beta bound, the relaxed loss and its gradient (the library's
reverse mode against the oracle's central differences of the loss), whole Adam runs with
their temperature schedule (loss at every step, final parameters, the plan read at tau = 0),
the discrete plan's evaluation, and Algorithm 1's ordering.  Host logic: no GPU involved.

Tolerances: the bound to 1e-12 relative (both solve I_l(a, b) = 1 - alpha to double
resolution); loss 1e-12 relative; gradient 1e-6 relative + 1e-8 absolute (the oracle's
central difference with h = 1e-6 has O(h^2) truncation and eps |L| / h ~ 1e-9 rounding for
losses up to ~10); an Adam run to 1e-6 (Adam's normalised steps keep those differences at
the same size); the discrete plan and everything evaluated from it exactly."""
import numpy as np
import pytest

from oracle import optimizer as oo
from paper_2602_04430_amd import kvop as K


def _problem(n_filters=1, n_ops=3, S=200, seed=0, noise=(1.0, 0.5), targets=(0.9, 0.9), alpha=0.95):
    rng = np.random.default_rng(seed)
    los, costs, golds = [], [], []
    for j in range(n_filters):
        g = rng.normal(0.3 * j, 2, S)
        rows = [g + rng.normal(0, noise[i % len(noise)], S) for i in range(n_ops - 1)] + [g]
        los.append(np.stack(rows).astype(np.float32).astype(np.float64))   # profiled log-odds are FP32
        costs.append(np.cumsum(rng.uniform(1, 4, n_ops)))
        golds.append((g.astype(np.float32) > 0).astype(np.int8))
    pb = oo.Problem(los, costs, golds, targets[0], targets[1], alpha)
    return pb, K.PlanProblem(los, costs, golds, targets[0], targets[1], alpha)


def test_beta_lower_bound():
    rng = np.random.default_rng(1)
    cases = [(1, 1, 0.95), (1, 9, 0.5), (7, 1, 0.99), (3000, 12, 0.95), (12, 3000, 0.95), (2000, 2000, 0.9)]
    cases += [tuple(rng.uniform(1, 600, 2)) + (rng.uniform(0.05, 0.995),) for _ in range(30)]
    for a, b, al in cases:
        assert K.kvop_beta_lower_bound(a, b, al) == pytest.approx(oo.beta_lower_bound(a, b, al), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("n_filters,n_ops,targets", [(1, 2, (0.9, 0.9)), (1, 4, (0.97, 0.95)), (2, 3, (0.9, 0.8)),
                                                      (3, 2, (0.0, 0.0))])
def test_loss_and_gradient(n_filters, n_ops, targets):
    pb, P = _problem(n_filters, n_ops, seed=n_filters * 10 + n_ops, targets=targets)
    rng = np.random.default_rng(n_ops)
    for tau in (1.0, 0.3, 0.05):
        params = rng.normal(0, 1, oo.n_params(pb))
        loss, grad = K.kvop_plan_loss(P, params, tau, 10.0)
        assert loss == pytest.approx(oo.loss(pb, params, tau, 10.0), rel=1e-12)
        np.testing.assert_allclose(grad, oo.grad_fd(pb, params, tau, 10.0), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("case", ["perfect_cheap", "useful_cheap", "useless_cheap", "two_filters"])
def test_optimize_matches_oracle(case):
    if case == "two_filters":
        pb, P = _problem(2, 2, S=150, seed=3)
    else:
        noise = {"perfect_cheap": 0.0, "useful_cheap": 1.0, "useless_cheap": 30.0}[case]
        pb, P = _problem(1, 2, S=300, seed=4, noise=(noise,))
    opts = oo.Options(steps=150)
    p_ref, trace_ref = oo.optimize(pb, opts)
    got = K.kvop_plan_optimize(P, steps=opts.steps, lr=opts.lr, beta=opts.beta, tau0=opts.tau0,
                               tau_end=opts.tau_end, theta0=opts.theta0)
    np.testing.assert_allclose(got["trace"], trace_ref, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(got["params"], p_ref, rtol=1e-6, atol=1e-6)
    plan = oo.extract(pb, p_ref)
    np.testing.assert_array_equal(got["selected"], np.concatenate(plan.selected).astype(np.int8))
    np.testing.assert_allclose(got["theta_pos"], np.concatenate(plan.theta_pos), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(got["theta_neg"], np.concatenate(plan.theta_neg), rtol=1e-6, atol=1e-6)
    cuts = np.cumsum([len(c) for c in pb.cost])[:-1]
    ev = oo.evaluate(pb, oo.Plan(plan.selected, np.split(got["theta_pos"], cuts), np.split(got["theta_neg"], cuts)))
    rep = got["report"]
    assert (rep["tp"], rep["fp"], rep["fn"]) == (ev["tp"], ev["fp"], ev["fn"])
    assert rep["cost_frac"] == pytest.approx(ev["cost_frac"], rel=1e-12)
    assert rep["recall_lb"] == pytest.approx(ev["recall_lb"], rel=1e-12)
    assert rep["precision_lb"] == pytest.approx(ev["precision_lb"], rel=1e-12)
    if case != "two_filters":
        assert rep["recall_lb"] >= 0.9 and rep["precision_lb"] >= 0.9     # the constraints hold on the sample


def test_evaluate_matches_oracle():
    pb, P = _problem(2, 4, S=500, seed=9)
    rng = np.random.default_rng(9)
    for _ in range(5):
        sel = [rng.integers(0, 2, 4).astype(bool) for _ in range(2)]
        tp = [rng.uniform(-0.5, 2, 4).astype(np.float32) for _ in range(2)]
        tn = [(t - rng.uniform(0, 2, 4)).astype(np.float32) for t in tp]
        ev = oo.evaluate(pb, oo.Plan(sel, tp, tn))
        got = K.kvop_plan_evaluate(P, np.concatenate(sel), np.concatenate(tp), np.concatenate(tn))
        np.testing.assert_array_equal(got["accept"], ev["accept"])
        np.testing.assert_array_equal(got["processed"], ev["processed"])
        np.testing.assert_array_equal(got["sel_inter"], ev["sel_inter"])
        np.testing.assert_array_equal(got["sel_intra"], ev["sel_intra"])
        r = got["report"]
        assert (r["tp"], r["fp"], r["fn"]) == (ev["tp"], ev["fp"], ev["fn"])
        assert r["cost_frac"] == pytest.approx(ev["cost_frac"], rel=1e-12)


def test_reorder_matches_oracle_and_brute_force():
    rng = np.random.default_rng(13)
    for _ in range(30):
        m = int(rng.integers(1, 7))
        n_log = int(rng.integers(1, min(m, 4) + 1))
        impl = rng.integers(0, n_log, m)
        cost = rng.uniform(0.1, 10, m)
        intra = rng.uniform(0, 1, m)
        inter = np.maximum(intra, rng.uniform(0, 1, m))
        order, c = K.kvop_plan_reorder(impl, cost, inter, intra, 4096.0)
        _, c_dp = oo.dp_reorder(list(impl), cost, inter, intra, 4096.0)
        _, c_bf = oo.brute_force_order(list(impl), cost, inter, intra, 4096.0)
        assert sorted(order) == list(range(m))
        assert c == pytest.approx(c_dp, rel=1e-12) and c == pytest.approx(c_bf, rel=1e-12)
        assert oo.order_cost(order, list(impl), cost, inter, intra, 4096.0) == pytest.approx(c, rel=1e-12)
    # the largest instance the entry point takes
    m = 20
    impl, cost = rng.integers(0, 5, m), rng.uniform(0.1, 10, m)
    intra = rng.uniform(0, 1, m)
    inter = np.maximum(intra, rng.uniform(0, 1, m))
    order, c = K.kvop_plan_reorder(impl, cost, inter, intra, 1.0)
    assert sorted(order) == list(range(m))
    assert oo.order_cost(order, list(impl), cost, inter, intra, 1.0) == pytest.approx(c, rel=1e-12)


def test_planner_errors():
    pb, P = _problem(1, 2)
    for bad in (dict(steps=0), dict(lr=0.0), dict(tau0=0.01, tau_end=0.1), dict(tau_end=0.0)):
        with pytest.raises(K.KvopError):
            K.kvop_plan_optimize(P, **bad)
    with pytest.raises(K.KvopError):        # a cost that is not positive
        K.kvop_plan_loss(K.PlanProblem(pb.log_odds, [np.array([1.0, 0.0])], pb.gold, 0.9, 0.9, 0.95),
                         np.zeros(6), 1.0, 1.0)
    with pytest.raises(K.KvopError):
        K.kvop_plan_loss(K.PlanProblem(pb.log_odds, pb.cost, pb.gold, 0.9, 0.9, 1.0), np.zeros(6), 1.0, 1.0)
    bad_lo = [pb.log_odds[0].copy()]
    bad_lo[0][0, 3] = np.nan
    with pytest.raises(K.KvopError):
        K.kvop_plan_loss(K.PlanProblem(bad_lo, pb.cost, pb.gold, 0.9, 0.9, 0.95), np.zeros(6), 1.0, 1.0)
    with pytest.raises(K.KvopError):
        K.kvop_plan_reorder(np.zeros(21, np.int32), np.ones(21), np.ones(21), np.ones(21), 1.0)
    with pytest.raises(K.KvopError):
        K.kvop_plan_reorder([0, 1], [1.0, 1.0], [1.5, 0.5], [0.5, 0.5], 1.0)
    with pytest.raises(K.KvopError):
        K.kvop_beta_lower_bound(0.0, 1.0, 0.95)
