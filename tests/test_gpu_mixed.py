"""Batching form: mixed filter/map/join items in one pass (eager, persistent attention,
hipGraph replay across waves) give exactly the results of separate per-operator calls."""
import numpy as np
import pytest
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import Engine, say

pytestmark = pytest.mark.gpu

SHAPE = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)


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
