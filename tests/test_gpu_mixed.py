"""Batching form: mixed filter/map/join items in one pass (eager, persistent attention,
hipGraph replay across waves) against the FP64 oracle, item by item, in every mode; and the
same outputs exactly as separate per-operator calls."""
import numpy as np
import pytest
import torch

from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, Engine, check_map, decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

SHAPE = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
SHAPE128 = synth.ModelShape(n_layers=2, d_model=512, n_heads=4, n_kv_heads=2, head_dim=128, d_ffn=1024, vocab=512)
MODES = {"eager": 0, "persistent": K.KVOP_MIXED_PERSISTENT, "graph": K.KVOP_MIXED_GRAPH,
         "graph+persistent": K.KVOP_MIXED_PERSISTENT | K.KVOP_MIXED_GRAPH}


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
@pytest.mark.parametrize("shape", [SHAPE, SHAPE128], ids=["d64", "d128"])
def test_mixed_matches_oracle(device, shape, compute, kv):
    """Every item of an interleaved filter/map/join list against the FP64 oracle, in all four
    modes, over several waves (the first eager, full waves captured and replayed, a partial
    last one): filter and join logits within E with decisions agreeing outside the margin
    band; map slice logits within E while the decoded texts agree, and ids equal to the
    oracle's up to each item's first step inside the band."""
    seed = 13
    w = synth.make_weights(shape, seed, gain_jitter=0.1)
    nd = 48
    docs = synth.make_docs_uniform(nd, 1, 100, shape.vocab, seed=seed)
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=seed)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(nd)]
    rng = np.random.default_rng(seed)
    f_docs = rng.choice(nd, 24, replace=False)
    m_docs = rng.choice(nd, 32, replace=False)
    pairs = synth.join_pairs(nd, 12, seed=seed)
    L_idx, L_off, L_h = [], [0], []

    def add(dd):
        L_idx.append(lists[dd]); L_off.append(L_off[-1] + len(lists[dd])); L_h.append(handles[dd])
        return len(L_h) - 1
    items = [(0, add(dd), dd) for dd in f_docs] + [(1, add(dd), dd) for dd in m_docs]
    for a, b in pairs:
        first = add(a)
        add(b)
        items.append((2, first, (a, b)))
    items = [items[i] for i in rng.permutation(len(items))]
    idx = torch.from_numpy(np.concatenate(L_idx).astype(np.int32)).cuda()
    offs, hs = np.array(L_off), np.array(L_h, np.uint64)
    sf, sm, sj = (synth.suffix_tokens(S, shape.vocab, seed=seed, which=k) for k, S in ((0, 7), (1, 5), (2, 9)))
    n_gen, lo, nl = 8, 256, 256
    opf = K.make_op(K.KVOP_FILTER, sf, synth.YES_ID, synth.NO_ID)
    opm = K.make_op(K.KVOP_MAP, sm, label_lo=lo, label_n=nl, n_gen=n_gen)
    opj = K.make_op(K.KVOP_JOIN, sj, synth.YES_ID, synth.NO_ID)
    # the oracle, in each operator's order of appearance
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(nd)]
    ref_f = [om.filter_eval(m, caches[d], lists[d], sf, synth.YES_ID, synth.NO_ID) for k, _, d in items if k == 0]
    ref_m = [om.map_eval(m, caches[d], lists[d], sm, lo, nl, n_gen) for k, _, d in items if k == 1]
    ref_j = [om.join_eval(m, caches[d[0]], lists[d[0]], caches[d[1]], lists[d[1]], sj, synth.YES_ID, synth.NO_ID)
             for k, _, d in items if k == 2]
    nf, nm, nj = len(ref_f), len(ref_m), len(ref_j)
    item_op = np.array([k for k, _, _ in items], np.int32)
    item_list = np.array([li for _, li, _ in items], np.int64)
    E = BOUND[(compute, kv)]
    failures = []
    try:
        K.kvop_set_wave_rows(100)          # several waves: eager first, captured, replayed, partial last
        for name, flags in MODES.items():
            lf = torch.full((nf, 2), np.nan, device=device)
            df = torch.full((nf,), 9, dtype=torch.int8, device=device)
            lm = torch.full((nm, n_gen, nl), np.nan, device=device)
            tm = torch.full((nm, n_gen), -1, dtype=torch.int32, device=device)
            lj = torch.full((nj, 2), np.nan, device=device)
            dj = torch.full((nj,), 9, dtype=torch.int8, device=device)
            say("mixed vs oracle", shape.head_dim, compute, kv, name)
            K.kvop_mixed_eval(eng.pool, [(opf, lf, df, None), (opm, lm, None, tm), (opj, lj, dj, None)], r, idx, offs,
                              hs, item_op, item_list, flags)
            torch.cuda.synchronize()
            line = [f"mixed D {shape.head_dim} {compute}/{kv} {name}:"]
            for tag, lg, dec, refs in (("filter", lf, df, ref_f), ("join", lj, dj, ref_j)):
                lg, dec = lg.cpu().numpy().astype(np.float64), dec.cpu().numpy()
                err = float(np.max(np.abs(lg - np.stack([x.logits for x in refs]))))
                bad, band = decisions_agree_outside_band([x.log_odds for x in refs], dec, E)
                line.append(f"{tag} max-abs logit error {err:.3g}, decisions outside the band that disagree {bad}, "
                            f"in-band fraction {band:.2f};")
                if not err <= E or bad:
                    failures.append(line[-1])
            checked, whole, err, fails = check_map(tm.cpu().numpy(), lm.cpu().numpy().astype(np.float64), ref_m, E)
            line.append(f"map max-abs slice-logit error {err:.3g}, ids outside the band checked {checked} of "
                        f"{nm * n_gen} (items with all ids outside {whole})")
            failures += fails
            if checked == 0:
                failures.append("map id check vacuous")
            say(" ".join(line))
    finally:
        K.kvop_set_wave_rows(131072)
    eng.close()
    assert not failures, failures[:6]


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "fp8")])
def test_mixed_equals_separate_calls(device, compute, kv):
    w = synth.make_weights(SHAPE, 12)
    docs = synth.make_docs_uniform(70, 1, 80, SHAPE.vocab, seed=12)
    eng = Engine(SHAPE, w, compute, kv)
    handles = eng.build(docs)
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=12)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(70)]
    rng = np.random.default_rng(12)
    f_docs = rng.choice(70, 25, replace=False)
    m_docs = rng.choice(70, 20, replace=False)
    pairs = synth.join_pairs(70, 10, seed=12)
    # flat lists/handles: filter items, map items, join items (2 each)
    L_idx, L_off, L_h = [], [0], []

    def add(dd):
        L_idx.append(lists[dd]); L_off.append(L_off[-1] + len(lists[dd])); L_h.append(handles[dd])
        return len(L_h) - 1
    items = [(0, add(dd)) for dd in f_docs] + [(1, add(dd)) for dd in m_docs]
    for a, b in pairs:
        first = add(a)
        add(b)
        items.append((2, first))
    order = rng.permutation(len(items))
    items = [items[i] for i in order]
    idx = torch.from_numpy(np.concatenate(L_idx).astype(np.int32)).cuda()
    offs = np.array(L_off)
    hs = np.array(L_h, np.uint64)
    sf, sm, sj = (synth.suffix_tokens(S, SHAPE.vocab, seed=12, which=k) for k, S in ((0, 7), (1, 5), (2, 9)))
    n_gen, lo, nl = 4, 256, 64
    opf = K.make_op(K.KVOP_FILTER, sf, 1, 0)
    opm = K.make_op(K.KVOP_MAP, sm, label_lo=lo, label_n=nl, n_gen=n_gen)
    opj = K.make_op(K.KVOP_JOIN, sj, 1, 0)
    nf, nm, nj = 25, 20, 10
    # reference: one op_eval per operator, items in each operator's order of appearance
    ref = {}
    for k, op in ((0, opf), (1, opm), (2, opj)):
        mine = [li for (kk, li) in items if kk == k]
        sel_lists = []
        for li in mine:
            sel_lists += [li, li + 1] if k == 2 else [li]
        sub_idx = np.concatenate([L_idx[i] for i in sel_lists]).astype(np.int32)
        sub_off = np.concatenate([[0], np.cumsum([len(L_idx[i]) for i in sel_lists])])
        sub_h = hs[sel_lists]
        if k == 1:
            ref[k] = eng.map(sub_h, sub_idx, sub_off, sm, lo, nl, n_gen, r=r)
        else:
            ref[k] = eng.filter(sub_h, sub_idx, sub_off, sf if k == 0 else sj, r=r,
                                kind=K.KVOP_FILTER if k == 0 else K.KVOP_JOIN)
    item_op = np.array([k for k, _ in items], np.int32)
    item_list = np.array([li for _, li in items], np.int64)
    try:
        K.kvop_set_wave_rows(100)          # several waves: eager first, captured, replayed, partial last
        for flags in (0, K.KVOP_MIXED_PERSISTENT, K.KVOP_MIXED_PERSISTENT | K.KVOP_MIXED_GRAPH,
                      K.KVOP_MIXED_GRAPH):
            say("mixed", compute, kv, "flags", flags)
            lf = torch.full((nf, 2), np.nan, device=device)
            df = torch.full((nf,), 9, dtype=torch.int8, device=device)
            lm = torch.full((nm, n_gen, nl), np.nan, device=device)
            tm = torch.full((nm, n_gen), -1, dtype=torch.int32, device=device)
            lj = torch.full((nj, 2), np.nan, device=device)
            dj = torch.full((nj,), 9, dtype=torch.int8, device=device)
            K.kvop_mixed_eval(eng.pool, [(opf, lf, df, None), (opm, lm, None, tm), (opj, lj, dj, None)], r, idx, offs,
                              hs, item_op, item_list, flags)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(lf.cpu().numpy(), ref[0][0].astype(np.float32))
            np.testing.assert_array_equal(df.cpu().numpy(), ref[0][1])
            np.testing.assert_array_equal(lj.cpu().numpy(), ref[2][0].astype(np.float32))
            np.testing.assert_array_equal(dj.cpu().numpy(), ref[2][1])
            np.testing.assert_array_equal(tm.cpu().numpy(), ref[1][1])
            np.testing.assert_array_equal(lm.cpu().numpy(), ref[1][0].astype(np.float32))
    finally:
        K.kvop_set_wave_rows(131072)
    eng.close()
