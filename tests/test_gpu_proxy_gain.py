"""What the learned proxy gains over the method without it.

Method without the proxy: the full operator (the filter at r = 1, BF16 weights/activations and
BF16 cache) evaluates every tuple.  With it (Section 4.1, Eqs. 1-3: a cheap first stage that
accepts or rejects the tuples it is sure of and passes the rest on): the proxy answers the
tuples whose confidence exceeds tau and the full operator evaluates only the others.

The documents are about topics (synth.topic_docs: 16 topics of 4 token ids, lengths uniform
in [32, 128]) on the small 2-layer decoder, so that a tuple's answer depends on what its
document is about, as with a filter over a real collection.  Everything the proxy learns from
comes from the full operator: its decisions on 4096 training documents (threshold at the
median training log-odds, so the classes are balanced), and a tenth of them held out for
early stopping and for tau* (the smallest tau in {0.9, 0.95, 0.99} with at most 1% held-out
disagreement).  On 2048 fresh documents the test measures the proxy's coverage, the
cascade's disagreement with the full operator, the operator evaluations saved and the time
of both routes; it requires at most 1% disagreement, a coverage of at least 20%, and that an
untrained proxy (its initial parameters, the same standardiser) gains nothing at that bar."""
import time

import numpy as np
import pytest
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import Engine, say

pytestmark = pytest.mark.gpu

SHAPE = synth.TINY
N_TRAIN, N_FRESH = 4096, 2048
HIDDEN = 256
TAUS = (0.9, 0.95, 0.99)


def _pack(p):
    return np.concatenate([p["w1"].ravel(), p["b1"], p["w2"].ravel(), p["b2"]]).astype(np.float32)


def _infer(px, feats, tau, device):
    n = feats.shape[0]
    cls = torch.empty(n, dtype=torch.int8, device=device)
    conf = torch.empty(n, dtype=torch.float32, device=device)
    ans = torch.empty(n, dtype=torch.int8, device=device)
    K.kvop_proxy_infer(px, feats, tau, cls, conf, ans)
    torch.cuda.synchronize()
    return cls.cpu().numpy(), conf.cpu().numpy(), ans.cpu().numpy().astype(bool)


def test_trained_proxy_gains_over_the_full_operator_alone(device):
    seed = 3
    w = synth.make_weights(SHAPE, 0)
    suffix = synth.suffix_tokens(16, SHAPE.vocab, seed)
    tr_docs, _ = synth.topic_docs(N_TRAIN, 16, 4, 32, 128, SHAPE.vocab, seed, stream=0)
    ev_docs, _ = synth.topic_docs(N_FRESH, 16, 4, 32, 128, SHAPE.vocab, seed, stream=1)
    eng = Engine(SHAPE, w, "bf16", "bf16", pool_bytes=1 << 30)
    # ---- training data: pooled features and the full operator's log-odds
    htr, ftr = eng.build(tr_docs, pooled=True)
    idx, offs = synth.full_lists(tr_docs.lengths)
    lg, _ = eng.filter(htr, idx, offs, suffix)
    lo_tr = lg[:, 0] - lg[:, 1]
    K.kvop_kv_release(eng.pool, htr)
    n_fit = N_TRAIN - N_TRAIN // 10
    theta = float(np.float32(np.median(lo_tr[:n_fit])))
    labels_np = (lo_tr > theta).astype(np.int32)
    labels = torch.from_numpy(labels_np).to(device)
    p0 = synth.proxy_init(SHAPE.d_model, HIDDEN, 2, seed)
    px = K.kvop_proxy_create(SHAPE.d_model, HIDDEN, torch.from_numpy(_pack(p0)).to(device))
    K.kvop_proxy_fit_standardizer(px, ftr[:n_fit])
    best = torch.empty(SHAPE.d_model * HIDDEN + 3 * HIDDEN + 2, device=device)
    best_loss, best_ep, bs = np.inf, -1, 256
    for ep in range(20):
        order = torch.from_numpy(synth.proxy_order(n_fit, ep, seed)).to(device)
        for s0 in range(0, n_fit - bs + 1, bs):
            K.kvop_proxy_train_step(px, ftr, labels, order[s0:s0 + bs], bs, 1e-3)
        c, cf, _ = _infer(px, ftr[n_fit:], 0.5, device)
        p_true = np.where(c == labels_np[n_fit:], cf, 1.0 - cf).astype(np.float64)
        vl = float(-np.mean(np.log(np.maximum(p_true, 1e-12))))
        if vl < best_loss:
            best_loss, best_ep = vl, ep
            K.kvop_proxy_params(px, best)
    K.kvop_proxy_destroy(px)
    px = K.kvop_proxy_create(SHAPE.d_model, HIDDEN, best)
    K.kvop_proxy_fit_standardizer(px, ftr[:n_fit])
    tau_star = None
    for tau in TAUS:
        c, _, an = _infer(px, ftr[n_fit:], tau, device)
        if np.mean((c != labels_np[n_fit:]) & an) <= 0.01:
            tau_star = tau
            break
    say(f"proxy: best epoch {best_ep}, held-out loss {best_loss:.4f}, theta {theta:.4f}, tau* {tau_star}")
    assert tau_star is not None
    # ---- fresh documents: the full operator alone, and the cascade
    hev, fev = eng.build(ev_docs, pooled=True)
    idx, offs = synth.full_lists(ev_docs.lengths)
    idx_d = torch.from_numpy(idx).to(device)
    op = K.make_op(K.KVOP_FILTER, suffix, synth.YES_ID, synth.NO_ID, theta, theta)
    lg = torch.empty(N_FRESH, 2, dtype=torch.float32, device=device)
    dec = torch.empty(N_FRESH, dtype=torch.int8, device=device)
    cls = torch.empty(N_FRESH, dtype=torch.int8, device=device)
    conf = torch.empty(N_FRESH, dtype=torch.float32, device=device)
    ans = torch.empty(N_FRESH, dtype=torch.int8, device=device)

    def full():
        K.kvop_op_eval(eng.pool, op, 1.0, idx_d, offs, hev, lg, dec)
        torch.cuda.synchronize()

    def cascade():
        K.kvop_proxy_infer(px, fev, tau_star, cls, conf, ans)
        unsure = np.nonzero(ans.cpu().numpy() == 0)[0].astype(np.int32)    # the host routes them
        if len(unsure):
            K.kvop_op_eval_select(eng.pool, op, 1.0, idx_d, offs, hev, unsure, lg, dec)
        torch.cuda.synchronize()
        return unsure

    def timed(fn, reps=5):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        return (time.perf_counter() - t0) / reps * 1e3, out

    ms_full, _ = timed(full)
    full_dec = dec.cpu().numpy().copy()
    ms_cascade, unsure = timed(cascade)
    answered = ans.cpu().numpy().astype(bool)
    final = np.where(answered, cls.cpu().numpy(), dec.cpu().numpy())
    coverage = float(answered.mean())
    disagreement = float(np.mean(final != full_dec))
    # the method without training: the proxy's initial parameters, same standardiser
    p_un = K.kvop_proxy_create(SHAPE.d_model, HIDDEN, torch.from_numpy(_pack(p0)).to(device))
    K.kvop_proxy_fit_standardizer(p_un, ftr[:n_fit])
    uc, _, ua = _infer(p_un, fev, tau_star, device)
    un_cov = float(ua.mean())
    un_dis = float(np.mean((uc != full_dec) & ua))
    say(f"fresh tuples {N_FRESH}: trained proxy at tau {tau_star} answers {coverage:.1%} "
        f"(full-operator evaluations {len(unsure)} instead of {N_FRESH}), disagreement with the full operator "
        f"{disagreement:.2%}; time {ms_cascade:.2f} ms vs {ms_full:.2f} ms for the full operator alone "
        f"({1 - ms_cascade / ms_full:+.1%} saved); untrained proxy answers {un_cov:.1%} with disagreement "
        f"{un_dis:.2%}")
    assert len(unsure) == N_FRESH - int(answered.sum())
    assert disagreement <= 0.01
    assert coverage >= 0.2
    assert un_cov == 0.0 or un_dis > 0.01
    K.kvop_proxy_destroy(p_un)
    K.kvop_proxy_destroy(px)
    eng.close()
