"""Pins of the expected-attention compression oracle (oracle/compress.py) to things other than
itself: the averaged rotation is the mean of the oracle's own rotations; the expected weight
is the Gaussian moment generating function (checked by Monte Carlo sampling); with no query
spread and one future position the method reduces to plain softmax attention of that query;
the per-(layer, head) normalisation, value-norm weighting and the nested top-k ladder."""
import numpy as np
import pytest

from oracle import compress as oc
from oracle import model as om
from paper_2602_04430_amd import synth

MICRO = synth.ModelShape(n_layers=2, d_model=32, n_heads=4, n_kv_heads=2, head_dim=8, d_ffn=64, vocab=64)


@pytest.mark.parametrize("L,n", [(0, 1), (5, 1), (17, 32), (1000, 7)])
def test_averaged_rotation_is_the_mean_of_rotations(L, n):
    D, theta = 16, 10000.0
    x = np.random.default_rng(L + n).standard_normal(D)
    mean = np.mean([om.rope(x[None, :], np.array([p], np.float64), theta)[0] for p in range(L, L + n)], axis=0)
    c, s = oc.averaged_rotation(L, n, D, theta)
    np.testing.assert_allclose(oc.apply_averaged_rotation(x, c, s), mean, rtol=0, atol=1e-13)


def test_expected_log_weight_is_the_gaussian_mgf():
    """log E[exp(q.k/sqrt(D))] against a Monte Carlo estimate over 400 000 Gaussian queries
    (standard error of the estimate well under the 0.01 tolerance at these spreads)."""
    rng = np.random.default_rng(7)
    D = 8
    mu = rng.standard_normal(D) * 0.5
    A = rng.standard_normal((D, D)) * 0.3
    sig = A @ A.T
    K = rng.standard_normal((5, D))
    q = rng.multivariate_normal(mu, sig, size=400_000)
    mc = np.log(np.mean(np.exp(q @ K.T / np.sqrt(D)), axis=0))
    np.testing.assert_allclose(oc.expected_log_weight(mu, sig, K), mc, rtol=0, atol=1e-2)
    # no spread: the linear term alone
    np.testing.assert_allclose(oc.expected_log_weight(mu, np.zeros((D, D)), K), K @ mu / np.sqrt(D), atol=1e-15)


def test_no_spread_and_one_future_position_is_softmax_attention():
    """All queries equal (covariance 0) and a single future position L: the expected weights
    are the softmax attention of that query, rotated at L, over the document's keys; with
    unit value norms they are the contributions."""
    rng = np.random.default_rng(3)
    H = Hkv = 2
    L, D, theta = 9, 8, 10000.0
    q0 = rng.standard_normal((H, 1, D))
    qt = np.repeat(q0, L, axis=1)
    k = rng.standard_normal((Hkv, L, D))
    v = rng.standard_normal((Hkv, L, D))
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    got = oc.layer_contributions(qt, k, v, L, 1, theta)
    for h in range(H):
        qr = om.rope(q0[h], np.array([L], np.float64), theta)[0]
        want = om.softmax(k[h] @ qr / np.sqrt(D))
        np.testing.assert_allclose(got[h], want, rtol=0, atol=1e-12)


def test_contribution_scales_with_the_value_norm():
    """Two keys with equal expected weight and value norms 1 and 3: contributions 1/4, 3/4."""
    D = 4
    qt = np.zeros((1, 2, D))
    k = np.zeros((1, 2, D))
    v = np.zeros((1, 2, D))
    v[0, 0, 0], v[0, 1, 1] = 1.0, 3.0
    np.testing.assert_allclose(oc.layer_contributions(qt, k, v, 2, 4, 10000.0), [[0.25, 0.75]], atol=1e-15)


def test_scores_total_and_the_nested_ladder():
    m = om.Model(MICRO, synth.make_weights(MICRO, 5, gain_jitter=0.1))
    L = 23
    doc = np.random.default_rng(9).integers(0, MICRO.vocab, L)
    sc = oc.ea_scores(m, doc, 32)
    assert sc.shape == (L,) and np.all(sc >= 0)
    np.testing.assert_allclose(sc.sum(), MICRO.n_layers * MICRO.n_kv_heads, rtol=1e-12)
    prev = np.zeros(0, np.int32)
    for kk in range(1, L + 1):
        sel = oc.ea_select(sc, kk)
        assert len(sel) == kk and np.all(np.diff(sel) > 0)
        assert set(prev) <= set(sel)
        assert sc[sel].min() >= np.delete(sc, sel).max(initial=-1.0)
        prev = sel
    np.testing.assert_array_equal(oc.ea_select(sc, L), np.arange(L))


def test_selection_ties_take_the_lower_row():
    np.testing.assert_array_equal(oc.ea_select(np.array([1.0, 2.0, 2.0, 0.0, 2.0]), 2), [1, 2])
    np.testing.assert_array_equal(oc.ea_select(np.array([5.0, 5.0, 5.0]), 2), [0, 1])
