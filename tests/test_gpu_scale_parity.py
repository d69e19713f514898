"""Full-size parity: the 16-layer d_model-2048 decoder (16 query / 8 kv heads of 128, FFN
5632, vocab 32000) over the 4096-document filter workload, evaluated in the launch
configuration the benchmark times (all 4096 documents in one op_eval per r), with sampled
documents checked one by one against the FP64 oracle for every (dtype, r).  Prints the
error table: max-abs logit error and decisions outside the margin band.  The BF16 build is
the scored one (kvop_kv_build_scored: identical caches), and the expected-attention scores of
sampled documents are checked against the oracle's emulation of the BF16 form.  On that build
two properties are checked over all 4096 documents, bit for bit: the cascade executor over
the expected-attention ladder equals Eqs. 1-3 applied to its stages' own evaluations, and
padded batching equals the unpadded evaluation.

Bounds at this shape:
  FP32                 E = 1e-4   (as at the small shapes)
  BF16, BF16 cache     E = E_BF16 against the FP64 oracle and E_BF16_FORM against the FP64
      emulation of the BF16 form (the oracle with BF16-rounded weights and its activation
      and cache formats set to BF16 rounding), both derived from the oracle alone by
      tests/golden/bf16_scale_bound.py (figures in bf16_scale_bound.txt beside it): the
      form's roundings other than the weights move these logits by up to N = 0.032; the GPU's
      own roundings are another realisation of them, so E_BF16_FORM = 2 N; the whole format
      effect F (weights included) is at most 0.052, so E_BF16 = F + E_BF16_FORM.
  BF16, FP8-E4M3 cache E = 0.35 against the FP64 oracle, and 0.15 against the FP64
      oracle of the same cache format (codecs.fp8_cache_roundtrip applied to every
      layer's stored keys/values).  The format alone moves the oracle's logits by up to
      0.17 on these documents (computed by the oracle, printed by the test); the GPU rounds
      its codes from BF16-computed keys/values, so where a value lies near a rounding
      midpoint it picks the neighbouring code, which an FP64 emulation with BF16 weights
      puts at up to 0.06 of logit, doubled here, plus the BF16 arithmetic error (0.03):
      0.15.  Against the FP64 oracle: 0.2 (format, rounded up) + 0.15.
"""
import numpy as np
import pytest
import torch

from oracle import codecs
from oracle import compress as oc
from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

# sampled documents: the first ones, the longest (L = 4096) and shortest (L = 64), and
# documents from the middle and the end of the batch
SAMPLE = [0, 1, 7, 19, 81, 100, 2047, 4095]
E_BF16_FORM = 0.065     # GPU BF16 path vs the FP64 emulation of the BF16 form
E_BF16 = 0.12          # GPU BF16 path vs the FP64 oracle
E_SCALE = {("f32", "f32"): 1e-4, ("bf16", "bf16"): E_BF16, ("bf16", "fp8"): 0.35}
E_FP8_FORMAT = 0.15      # GPU FP8 path vs the FP64 oracle of the FP8 cache format
E_EA = 3e-2              # expected-attention row scores (BF16) vs the emulation of the BF16 form, relative
EA_SAMPLE = [81, 100, 7]  # L = 64, 149, 123


def _refs(m, wl, lists, store=None, tag="fp64"):
    docs = wl.docs
    out = {}
    for i in SAMPLE:
        c = om.kv_build(m, docs.doc(i), store=store)
        for r in wl.r_grid:
            idx, offs = lists[r]
            out[(i, r)] = om.filter_eval(m, c, idx[offs[i]:offs[i + 1]], wl.suffix, synth.YES_ID, synth.NO_ID)
        say("oracle", tag, "document", i, "L", int(docs.lengths[i]))
    return out


@pytest.fixture(scope="module")
def scale_setup():
    shape = synth.SCALE
    wl = synth.scale_filter(0)
    w = synth.make_weights(shape, 0)
    m = om.Model(shape, w)
    lists = {r: synth.retained_lists(wl.docs.lengths, r, seed=0) for r in wl.r_grid}
    ref = _refs(m, wl, lists)
    flat = torch.from_numpy(synth.pack_weights(shape, w))
    return {"shape": shape, "wl": wl, "model": m, "flat": flat, "lists": lists, "ref": ref}


@pytest.fixture(scope="module")
def fp8_format_refs(scale_setup):
    s = scale_setup
    return _refs(s["model"], s["wl"], s["lists"], store=codecs.fp8_cache_roundtrip, tag="fp8-format")


@pytest.fixture(scope="module")
def bf16_form_model(scale_setup):
    w = synth.make_weights(scale_setup["shape"], 0)
    wb = {k: codecs.bf16_round(v) if v.ndim == 2 else v for k, v in w.items()}
    return om.Model(scale_setup["shape"], wb, act=codecs.bf16_round)


@pytest.fixture(scope="module")
def bf16_form_refs(scale_setup, bf16_form_model):
    s = scale_setup
    return _refs(bf16_form_model, s["wl"], s["lists"], store=codecs.bf16_round, tag="bf16-form")


@pytest.mark.parametrize("compute,kv", [("bf16", "bf16"), ("bf16", "fp8"), ("f32", "f32")])
def test_scale_filter_sampled_parity(device, scale_setup, request, compute, kv):
    S = scale_setup
    shape, wl, lists, ref = S["shape"], S["wl"], S["lists"], S["ref"]
    qref, qname, qbound = None, "", 0.0
    if kv == "fp8":
        qref, qname, qbound = request.getfixturevalue("fp8_format_refs"), "the FP8 format", E_FP8_FORMAT
    elif compute == "bf16":
        qref, qname, qbound = request.getfixturevalue("bf16_form_refs"), "the BF16 form", E_BF16_FORM
    docs = wl.docs
    flat = S["flat"].to(device)
    model = K.kvop_model_create(K.make_cfg(shape), flat, {"f32": K.KVOP_F32, "bf16": K.KVOP_BF16}[compute])
    del flat
    kvdt = {"f32": K.KVOP_KV_F32, "bf16": K.KVOP_KV_BF16, "fp8": K.KVOP_KV_FP8}[kv]
    # the FP32 caches of all 4096 documents (427 GB) exceed HBM: there the first 1024
    # documents and the sampled ones are evaluated
    sel = np.arange(4096) if compute == "bf16" else np.unique(np.concatenate([np.arange(1024), SAMPLE]))
    sub = docs.subset(sel)
    probe = K.kvop_pool_create(model, kvdt, 1 << 20)
    need = sum(K.kvop_doc_bytes(probe, int(L)) for L in sub.lengths)
    K.kvop_pool_destroy(probe)
    pool = K.kvop_pool_create(model, kvdt, need + (64 << 20))
    scored = compute == "bf16" and kv == "bf16"   # same caches, plus expected-attention scores
    if scored:
        scores = torch.empty(int(sub.lengths.sum()), dtype=torch.float32, device=device)
        handles = K.kvop_kv_build_scored(pool, torch.from_numpy(sub.tokens).to(device), sub.offsets,
                                         len(wl.suffix), scores)
    else:
        handles = K.kvop_kv_build(pool, torch.from_numpy(sub.tokens).to(device), sub.offsets)
    op = K.make_op(K.KVOP_FILTER, wl.suffix, synth.YES_ID, synth.NO_ID)
    E = E_SCALE[(compute, kv)]
    pos = {int(d): i for i, d in enumerate(sel)}
    failures = []
    outs = {}
    for r in wl.r_grid:
        idx, offs = lists[r]
        sidx = np.concatenate([idx[offs[d]:offs[d + 1]] for d in sel])
        soffs = np.concatenate([[0], np.cumsum([offs[d + 1] - offs[d] for d in sel])])
        lg = torch.empty(len(sel), 2, dtype=torch.float32, device=device)
        dec = torch.empty(len(sel), dtype=torch.int8, device=device)
        K.kvop_op_eval(pool, op, r, torch.from_numpy(sidx).to(device), soffs, handles, lg, dec)
        torch.cuda.synchronize()
        lg, dec = lg.cpu().numpy().astype(np.float64), dec.cpu().numpy()
        outs[r] = (lg, dec)
        got = np.stack([lg[pos[i]] for i in SAMPLE])
        exp = np.stack([ref[(i, r)].logits for i in SAMPLE])
        err = float(np.max(np.abs(got - exp)))
        bad, band = decisions_agree_outside_band([ref[(i, r)].log_odds for i in SAMPLE],
                                                 np.array([dec[pos[i]] for i in SAMPLE]), E)
        line = (f"error table {compute}/{kv} r={r}: max-abs logit error vs FP64 oracle {err:.3g} (bound {E}), "
                f"decisions outside the band that disagree: {bad}, in-band fraction {band:.2f}")
        if err > E or bad:
            failures.append(line)
        if qref is not None:
            qexp = np.stack([qref[(i, r)].logits for i in SAMPLE])
            qerr = float(np.max(np.abs(got - qexp)))
            fmt = float(np.max(np.abs(qexp - exp)))
            line += f"; vs the oracle of {qname} {qerr:.3g} (bound {qbound}); format alone {fmt:.3g}"
            if qerr > qbound:
                failures.append(line)
        say(line)
    if scored:
        # expected-attention scores of sampled documents from the same 4096-document build
        me = request.getfixturevalue("bf16_form_model")
        sc = scores.cpu().numpy().astype(np.float64)
        for i in EA_SAMPLE:
            ref = oc.ea_scores(me, docs.doc(i), len(wl.suffix))
            got = sc[sub.offsets[pos[i]]:sub.offsets[pos[i] + 1]]
            err = float(np.max(np.abs(got - ref) / np.abs(ref)))
            line = f"expected-attention scores, document {i} (L {len(ref)}): max relative error {err:.3g} (bound {E_EA})"
            say(line)
            if err > E_EA:
                failures.append(line)
        failures += _cascade_and_padding_at_scale(pool, op, handles, scores, sub, lists, outs, device)
    K.kvop_pool_destroy(pool)
    K.kvop_model_destroy(model)
    assert not failures, failures


def _cascade_and_padding_at_scale(pool, op, handles, scores, sub, lists, outs, device):
    """At the benchmark's size (all 4096 documents in one call), properties that need no
    oracle: the cascade over the expected-attention profiles r = 0.1 -> 0.25 -> 0.5 and the
    full r = 1 list equals Eqs. 1-3 applied to each stage's own full evaluation (stage,
    decision and logits bit for bit, Eq. 4's counts), and padded batching reproduces the
    unpadded r = 0.25 evaluation bit for bit."""
    failures = []
    n = len(sub.lengths)
    stage_lists = {}
    for r in (0.1, 0.25, 0.5):
        total = sum(K.kvop_retained_count(r, int(L)) for L in sub.lengths)
        idx_r = torch.empty(total, dtype=torch.int32, device=device)
        stage_lists[r] = (idx_r, K.kvop_ea_select(pool, scores, sub.offsets, r, idx_r))
    stage_lists[1.0] = (torch.from_numpy(lists[1.0][0]).to(device), lists[1.0][1])
    rs = (0.1, 0.25, 0.5, 1.0)

    def evaluate(r, theta, flags=0):
        o = K.make_op(K.KVOP_FILTER, op._keep, synth.YES_ID, synth.NO_ID, theta, -theta, flags=flags)
        lg = torch.empty(n, 2, dtype=torch.float32, device=device)
        dec = torch.empty(n, dtype=torch.int8, device=device)
        K.kvop_op_eval(pool, o, r, stage_lists[r][0], stage_lists[r][1], handles, lg, dec)
        torch.cuda.synchronize()
        return lg.cpu().numpy(), dec.cpu().numpy()

    th = []
    for r in rs[:-1]:
        lg, _ = evaluate(r, 0.0)
        th.append(float(np.float32(np.quantile(np.abs(lg[:, 0] - lg[:, 1]), 0.5))))
    th.append(0.0)
    table = [evaluate(r, t) for r, t in zip(rs, th)]
    first = np.full(n, len(rs) - 1)
    for t in range(n):
        d = [i for i in range(len(rs)) if table[i][1][t] != -1]
        if d:
            first[t] = d[0]
    o = K.make_op(K.KVOP_FILTER, op._keep, synth.YES_ID, synth.NO_ID)
    lg = torch.empty(n, 2, dtype=torch.float32, device=device)
    dec = torch.empty(n, dtype=torch.int8, device=device)
    stg = torch.empty(n, dtype=torch.int8, device=device)
    proc = K.kvop_cascade_eval(pool, o, [(r, t, -t, *stage_lists[r]) for r, t in zip(rs, th)], handles, lg, dec, stg)
    torch.cuda.synchronize()
    lg, dec, stg = lg.cpu().numpy(), dec.cpu().numpy(), stg.cpu().numpy()
    ok = (np.array_equal(stg, first) and np.array_equal(dec, [table[s][1][t] for t, s in enumerate(first)])
          and np.array_equal(lg, np.stack([table[s][0][t] for t, s in enumerate(first)]))
          and list(proc) == [int(np.sum(first >= i)) for i in range(len(rs))])
    line = f"cascade at scale: processed {list(proc)}, equals its per-stage evaluations: {ok}"
    say(line)
    if not ok:
        failures.append(line)
    idx, offs = lists[0.25]
    o = K.make_op(K.KVOP_FILTER, op._keep, synth.YES_ID, synth.NO_ID, flags=K.KVOP_FLAG_PADDED)
    lgp = torch.empty(n, 2, dtype=torch.float32, device=device)
    decp = torch.empty(n, dtype=torch.int8, device=device)
    K.kvop_op_eval(pool, o, 0.25, torch.from_numpy(idx).to(device), offs, handles, lgp, decp)
    torch.cuda.synchronize()
    lgp = lgp.cpu().numpy().astype(np.float64)
    ok = np.array_equal(lgp, outs[0.25][0]) and np.array_equal(decp.cpu().numpy(), outs[0.25][1])
    line = (f"padded batching at scale (r = 0.25): equals the unpadded evaluation: {ok} "
            f"(max |difference| {float(np.max(np.abs(lgp - outs[0.25][0]))):.3g}, "
            f"items differing {int(np.sum(np.any(lgp != outs[0.25][0], axis=1)))})")
    say(line)
    if not ok:
        failures.append(line)
    return failures
