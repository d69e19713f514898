"""GPU parity: the HIP path through the C ABI against the FP64 oracle (and, for the
projections, against a float64 product of the same rounded operands)."""
import os

import numpy as np
import pytest
import torch

from oracle import model as om
from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import BOUND, E_F32, Engine, check_map, decisions_agree_outside_band, say

pytestmark = pytest.mark.gpu

MICRO_GQA = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)


# ----------------------------------------------------------------------------- projections

def _bf16(x):
    return x.to(torch.bfloat16)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_gemm_every_tile_matches_float64(device, dtype, epi):
    rng = np.random.default_rng(0)
    dt = K.KVOP_F32 if dtype == "f32" else K.KVOP_BF16
    # K slabs of 64: 1, 2, 3, 4 and 8; several 256-row and 256-column tiles with ragged edges
    shapes = [(1, 128, 64), (520, 512, 128), (77, 256, 192), (300, 384, 256), (1000, 128, 512)]
    if epi != 2:
        shapes.append((37, 198, 96))       # ragged column edge, rows not 16-byte aligned
    for M, N, Kd in shapes:
        A = torch.from_numpy(rng.standard_normal((M, Kd)).astype(np.float32))
        B = torch.from_numpy(rng.standard_normal((N, Kd)).astype(np.float32))
        if dtype == "bf16":
            A, B = _bf16(A).float(), _bf16(B).float()
        ref = A.double() @ B.double().T
        if epi == 2:
            g = ref.reshape(M, N // 32, 2, 16)
            ref = (torch.nn.functional.silu(g[:, :, 0]) * g[:, :, 1]).reshape(M, N // 2)
        C0 = torch.from_numpy(rng.standard_normal(ref.shape).astype(np.float32))
        if epi == 1:
            ref = ref + C0.double()
        for tile in range(K.kvop_gemm_num_tiles(dt)):
            say("gemm", dtype, epi, M, N, Kd, K.kvop_gemm_tile_name(dt, tile))
            Ad = (A if dtype == "f32" else _bf16(A)).to(device)
            Bd = (B if dtype == "f32" else _bf16(B)).to(device)
            out_f32 = dtype == "f32" or epi == 1
            Cd = C0.clone().to(device) if out_f32 else _bf16(C0).to(device)
            ldc = ref.shape[1]
            try:
                K.kvop_debug_gemm(dt, K.KVOP_F32 if out_f32 else K.KVOP_BF16, epi, tile, Ad, Bd, Cd, M, N, Kd, Kd, Kd,
                                  ldc)
            except K.KvopError as e:        # direct-load tiles read whole K slabs only
                assert "lds" in K.kvop_gemm_tile_name(dt, tile) and Kd % 32 != 0 or Kd % 64 != 0, (tile, e)
                continue
            torch.cuda.synchronize()
            got = Cd.float().cpu().double()
            scale = max(1.0, float(ref.abs().max()))
            tol = 2e-5 * np.sqrt(Kd) * scale if out_f32 else 1.6e-2 * scale
            err = float((got - ref).abs().max())
            assert err <= tol, (dtype, epi, M, N, Kd, tile, err, tol)


@pytest.mark.parametrize("D", [32, 64, 128])
def test_rotary_epilogue_every_tile(device, D):
    """The projection with its rotary epilogue, for every BF16 tile: bit-identical to the plain
    projection followed by the separate rotation pass, rotated columns within two BF16 units in
    the last place (plus the FP32 rounding of a cancelling rotation) of a float64 rotation of
    the tile's own plain products, and the columns
    past rot_cols equal to those products.  Ragged rows and a column edge inside a tile."""
    rng = np.random.default_rng(D)
    M, N, Kd = 300, 640, 256
    rot = N - 2 * D
    half = D // 2
    A = _bf16(torch.from_numpy(rng.standard_normal((M, Kd)).astype(np.float32) * 0.5)).to(device)
    B = _bf16(torch.from_numpy(rng.standard_normal((N, Kd)).astype(np.float32) * 0.05)).to(device)
    n_pos = 4096
    pos = rng.integers(0, n_pos, M).astype(np.int32)
    inv = 10000.0 ** (-np.arange(half) * 2.0 / D)
    ang = np.arange(n_pos)[:, None] * inv[None, :]
    cos_t = torch.from_numpy(np.cos(ang).astype(np.float32)).to(device)
    sin_t = torch.from_numpy(np.sin(ang).astype(np.float32)).to(device)
    pos_d = torch.from_numpy(pos).to(device)
    c64, s64 = np.cos(ang).astype(np.float32).astype(np.float64), np.sin(ang).astype(np.float32).astype(np.float64)
    checked = 0
    for tile in range(K.kvop_gemm_num_tiles(K.KVOP_BF16)):
        outs = []
        for fused in (True, False):
            C = torch.full((M, N), float("nan"), dtype=torch.bfloat16, device=device)
            K.kvop_debug_gemm_rope(tile, A, B, C, M, N, Kd, D, rot, pos_d, cos_t, sin_t, fused)
            outs.append(C)
        plain = torch.full((M, N), float("nan"), dtype=torch.bfloat16, device=device)
        K.kvop_debug_gemm(K.KVOP_BF16, K.KVOP_BF16, 0, tile, A, B, plain, M, N, Kd, Kd, Kd, N)
        torch.cuda.synchronize()
        fz, sp, pl = (t.float().cpu().numpy().astype(np.float64) for t in (outs[0], outs[1], plain))
        assert np.array_equal(fz, sp), (tile, K.kvop_gemm_tile_name(K.KVOP_BF16, tile))
        np.testing.assert_array_equal(fz[:, rot:], pl[:, rot:])
        x = pl[:, :rot].reshape(M, rot // D, 2, half)
        c, s_ = c64[pos][:, None, :], s64[pos][:, None, :]
        ref = np.stack([x[:, :, 0] * c - x[:, :, 1] * s_, x[:, :, 1] * c + x[:, :, 0] * s_], axis=2).reshape(M, rot)
        # two BF16 units in the last place, plus the FP32 rounding of the rotation itself where
        # the result cancels towards zero
        err = np.abs(fz[:, :rot] - ref)
        assert np.all(err <= 2.0 ** -6 * np.abs(ref) + 2.0 ** -20 * np.abs(x).max()), (tile, float(err.max()))
        checked += 1
    say(f"rotary epilogue, D={D}: {checked} tiles fused == separate pass, within 2 BF16 ulp of float64")
    assert checked == K.kvop_gemm_num_tiles(K.KVOP_BF16)


# ----------------------------------------------------------------------------- kv_build

@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
def test_kv_build_cache_rows_match_oracle(device, compute, kv):
    shape = MICRO_GQA
    w = synth.make_weights(shape, 3, gain_jitter=0.1)
    docs = synth.make_docs_uniform(6, 1, 70, shape.vocab, seed=3)
    eng = Engine(shape, w, compute, kv)
    say("kv_build", compute, kv, docs.lengths.tolist())
    handles, pooled = eng.build(docs, pooled=True)
    m = om.Model(shape, w)
    tol = {"f32": 2e-5, "bf16": 3e-2, "fp8": 8e-2}[kv]
    for i in range(len(docs.lengths)):
        ref = om.kv_build(m, docs.doc(i))
        L = int(docs.lengths[i])
        out = torch.empty(L, shape.head_dim, dtype=torch.float32, device=device)
        for l in range(shape.n_layers):
            for h in range(shape.n_kv_heads):
                for kvsel, R in ((0, ref.K), (1, ref.V)):
                    K.kvop_debug_read_cache(eng.pool, handles[i], l, h, kvsel, out)
                    torch.cuda.synchronize()
                    got = out.cpu().numpy().astype(np.float64)
                    exp = R[l, h]
                    err = np.max(np.abs(got - exp)) / max(1e-6, np.max(np.abs(exp)))
                    assert err <= tol, (i, l, h, kvsel, err)
        perr = np.max(np.abs(pooled[i].cpu().numpy() - ref.pooled)) / np.max(np.abs(ref.pooled))
        assert perr <= {"f32": 2e-5, "bf16": 3e-2, "fp8": 5e-2}[kv], (i, perr)
    eng.close()


# ----------------------------------------------------------------------------- filter

def _golden_tiny():
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny_filter_fp64.txt")
    return np.loadtxt(path, comments="#")


def test_tiny_filter_fp32_all_tuples_match_stored_oracle(device):
    """The small plain-filter workload (64 tuples, r = 1) against the stored FP64 values."""
    wl = synth.tiny_filter(0)
    w = synth.make_weights(wl.shape, 0)
    eng = Engine(wl.shape, w, "f32", "f32")
    handles = eng.build(wl.docs)
    idx, offs = synth.full_lists(wl.docs.lengths)
    say("tiny filter f32")
    lg, dec = eng.filter(handles, idx, offs, wl.suffix)
    ref = _golden_tiny()
    err = np.max(np.abs(lg - ref[:, 1:3]))
    say("tiny filter f32 max-abs logit error", err)
    assert err <= E_F32
    bad, band = decisions_agree_outside_band(ref[:, 3], dec, E_F32)
    assert bad == 0
    assert set(np.unique(dec)) <= {0, 1}
    eng.close()


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
@pytest.mark.parametrize("r", [1.0, 0.5, 0.1])
def test_filter_gqa_retention_matches_oracle(device, compute, kv, r):
    shape = MICRO_GQA
    w = synth.make_weights(shape, 5, gain_jitter=0.1)
    docs = synth.make_docs_uniform(20, 1, 150, shape.vocab, seed=5)
    suffix = synth.suffix_tokens(21, shape.vocab, seed=5)
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    idx, offs = synth.retained_lists(docs.lengths, r, seed=5)
    say("filter", compute, kv, r)
    lg, dec = eng.filter(handles, idx, offs, suffix, r=r)
    m = om.Model(shape, w)
    E = BOUND[(compute, kv)]
    ref_lo = []
    for i in range(len(docs.lengths)):
        c = om.kv_build(m, docs.doc(i))
        res = om.filter_eval(m, c, idx[offs[i]:offs[i + 1]], suffix, synth.YES_ID, synth.NO_ID)
        err = np.max(np.abs(lg[i] - res.logits))
        assert err <= E, (i, err, E)
        ref_lo.append(res.log_odds)
    bad, band = decisions_agree_outside_band(ref_lo, dec, E)
    assert bad == 0
    eng.close()


# ----------------------------------------------------------------------------- error paths

def test_error_paths(device):
    shape = MICRO_GQA
    w = synth.make_weights(shape, 6)
    docs = synth.make_docs_uniform(4, 10, 40, shape.vocab, seed=6)
    suffix = synth.suffix_tokens(5, shape.vocab, seed=6)
    eng = Engine(shape, w, "f32", "f32", pool_bytes=4 << 20)
    handles = eng.build(docs)
    idx, offs = synth.full_lists(docs.lengths)

    def status(fn):
        try:
            fn()
        except K.KvopError as e:
            return e.status
        return K.KVOP_OK

    assert status(lambda: eng.filter(handles, idx, offs, suffix, r=0.0)) == K.KVOP_EINVAL
    assert status(lambda: eng.filter(handles, idx, offs, suffix, r=0.5)) == K.KVOP_EINVAL      # wrong count
    bad = idx.copy()
    bad[1], bad[2] = bad[2], bad[1]                                                            # unsorted
    assert status(lambda: eng.filter(handles, bad, offs, suffix)) == K.KVOP_EINVAL
    oob = idx.copy()
    oob[offs[1] - 1] = docs.lengths[0] + 5                                                     # out of range
    assert status(lambda: eng.filter(handles, oob, offs, suffix, flags=K.KVOP_FLAG_ANY_COUNT)) == K.KVOP_EINVAL
    # a valid call still works after the rejected ones
    lg, dec = eng.filter(handles, idx, offs, suffix)
    assert np.all(np.isfinite(lg))
    K.kvop_kv_release(eng.pool, handles[:1])
    assert status(lambda: eng.filter(handles, idx, offs, suffix)) == K.KVOP_EBADHANDLE
    assert status(lambda: K.kvop_kv_release(eng.pool, handles[:1])) == K.KVOP_EBADHANDLE
    # empty inputs: no documents, no items (outputs untouched); an empty document is refused
    empty = synth.Docs(np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(1, np.int64))
    assert len(eng.build(empty)) == 0
    lg0 = torch.full((1, 2), 5.0, device="cuda")
    K.kvop_op_eval(eng.pool, K.make_op(K.KVOP_FILTER, suffix), 1.0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                   [0], np.zeros(0, np.uint64), lg0)
    torch.cuda.synchronize()
    assert bool((lg0 == 5.0).all())
    hole = synth.Docs(np.array([3, 0, 2], np.int64), np.zeros(5, np.int32), np.array([0, 3, 3, 5], np.int64))
    assert status(lambda: eng.build(hole)) == K.KVOP_EINVAL
    # token ids outside [0, vocab) are refused before anything is built or written
    u_tok = K.kvop_pool_stats(eng.pool)
    for bad_id in (shape.vocab, -1):
        bad_doc = synth.Docs(np.array([3, 2], np.int64), np.array([1, 2, 3, bad_id, 0], np.int32),
                             np.array([0, 3, 5], np.int64))
        assert status(lambda: eng.build(bad_doc, pooled=True)) == K.KVOP_EINVAL
    assert K.kvop_pool_stats(eng.pool) == u_tok
    big = synth.make_docs_uniform(200, 400, 400, shape.vocab, seed=7)                          # too big for 4 MiB
    u0 = K.kvop_pool_stats(eng.pool)
    assert status(lambda: eng.build(big)) == K.KVOP_ENOMEM
    assert K.kvop_pool_stats(eng.pool) == u0                                                   # nothing leaked
    eng.close()


def test_calls_on_two_streams_match_one_stream(device):
    """Calls on one model share its workspaces and its pool's freed regions.  A filter on one
    stream, then (without any host synchronisation) a release of some of its documents, a
    build that reuses their regions and a second filter, all on another stream: every output
    equals the same calls made one after another on one stream."""
    shape = MICRO_GQA
    w = synth.make_weights(shape, 11)
    docs = synth.make_docs_uniform(160, 200, 600, shape.vocab, seed=11)
    new_docs = synth.make_docs_uniform(40, 200, 600, shape.vocab, seed=12)
    sa, sb = synth.suffix_tokens(16, shape.vocab, seed=11, which=0), synth.suffix_tokens(16, shape.vocab, seed=11, which=1)
    opa = K.make_op(K.KVOP_FILTER, sa, synth.YES_ID, synth.NO_ID)
    opb = K.make_op(K.KVOP_FILTER, sb, synth.YES_ID, synth.NO_ID)
    idx, offs = synth.full_lists(docs.lengths)
    nidx, noffs = synth.full_lists(new_docs.lengths)
    idx_d, nidx_d = torch.from_numpy(idx).cuda(), torch.from_numpy(nidx).cuda()
    ntok = torch.from_numpy(new_docs.tokens).cuda()

    def run(st1, st2):
        eng = Engine(shape, w, "bf16", "bf16", pool_bytes=256 << 20)
        handles = eng.build(docs)
        la = torch.full((160, 2), np.nan, device=device)
        lb = torch.full((40, 2), np.nan, device=device)
        torch.cuda.synchronize()
        K.kvop_op_eval(eng.pool, opa, 1.0, idx_d, offs, handles, la, stream=st1)
        K.kvop_kv_release(eng.pool, handles[120:])                  # regions freed while the filter may run
        nh = K.kvop_kv_build(eng.pool, ntok, noffs, stream=st2)     # and reused on the other stream
        K.kvop_op_eval(eng.pool, opb, 1.0, nidx_d, noffs, nh, lb, stream=st2)
        torch.cuda.synchronize()
        out = la.cpu().numpy(), lb.cpu().numpy()
        eng.close()
        return out

    say("two streams")
    one = torch.cuda.current_stream().cuda_stream
    ref = run(one, one)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    got = run(s1.cuda_stream, s2.cuda_stream)
    assert np.all(np.isfinite(ref[0])) and np.all(np.isfinite(ref[1]))
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])


@pytest.mark.parametrize("kind", ["filter", "join"])
def test_stage_readout_matches_oracle_layer_by_layer(device, kind):
    """kvop_debug_stage: the suffix rows' residual stream after every layer of a 3-layer model
    equals the oracle's, layer by layer (at the last layer, the last row that feeds the head)."""
    shape = synth.ModelShape(n_layers=3, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
    w = synth.make_weights(shape, 14, gain_jitter=0.1)
    docs = synth.make_docs_uniform(6, 5, 70, shape.vocab, seed=14)
    suffix = synth.suffix_tokens(7, shape.vocab, seed=14)
    S = len(suffix)
    eng = Engine(shape, w, "f32", "f32")
    handles = eng.build(docs)
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=14)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(6)]
    items = [(i,) for i in range(6)] if kind == "filter" else [(0, 3), (5, 1), (2, 2)]
    sel = [d for it in items for d in it]
    idx = np.concatenate([lists[d] for d in sel])
    offs = np.concatenate([[0], np.cumsum([len(lists[d]) for d in sel])])
    op = K.make_op(K.KVOP_FILTER if kind == "filter" else K.KVOP_JOIN, suffix, synth.YES_ID, synth.NO_ID)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(6)]
    # the oracle's suffix pass, layer by layer
    ref = []
    for it in items:
        if kind == "filter":
            a = it[0]
            ctxK = [caches[a].K[l][:, lists[a]] for l in range(shape.n_layers)]
            ctxV = [caches[a].V[l][:, lists[a]] for l in range(shape.n_layers)]
            n_ctx, pos0 = len(lists[a]), caches[a].length
        else:
            a, b = it
            ctxK, ctxV, n_ctx = om.join_context(m, caches[a], lists[a], caches[b], lists[b])
            pos0 = caches[a].length + caches[b].length
        x = m.w["embed"][suffix]
        vis = np.concatenate([np.ones((S, n_ctx), bool), np.tril(np.ones((S, S), bool))], axis=1)
        per = []
        for l in range(shape.n_layers):
            x, _, _ = m.layer(l, x, pos0 + np.arange(S), ctxK[l], ctxV[l], vis)
            per.append(x)
        ref.append(per)
    for layer in range(shape.n_layers):
        out = torch.full((len(items), S, shape.d_model), np.nan, dtype=torch.float32, device=device)
        say("stage readout", kind, "layer", layer)
        K.kvop_debug_stage(eng.pool, op, r, torch.from_numpy(idx).cuda(), offs, np.array([handles[d] for d in sel]),
                           layer, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        rows = slice(0, S) if layer + 1 < shape.n_layers else slice(S - 1, S)
        err = max(float(np.max(np.abs(got[i, rows] - ref[i][layer][rows]))) for i in range(len(items)))
        say(f"stage readout {kind} layer {layer}: max-abs difference from the oracle {err:.3g}")
        assert err <= 1e-4, (layer, err)
    bad = torch.zeros(1, S, shape.d_model, device=device)
    with pytest.raises(K.KvopError):
        K.kvop_debug_stage(eng.pool, op, r, torch.from_numpy(idx).cuda(), offs, np.array([handles[d] for d in sel]),
                           shape.n_layers, bad)
    eng.close()


# ----------------------------------------------------------------------------- map and join

@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
def test_map_greedy_decode_matches_oracle(device, compute, kv):
    """Greedy decode of 8 ids over a 256-label slice.  64 documents, so that the oracle has
    ids outside the margin band for every bound (the count of such ids depends on the oracle
    alone: 504 at FP32's bound, 40 at BF16's and 4 at FP8's for these seeded inputs)."""
    shape = MICRO_GQA
    w = synth.make_weights(shape, 8, gain_jitter=0.1)
    docs = synth.make_docs_uniform(64, 1, 90, shape.vocab, seed=8)
    suffix = synth.suffix_tokens(12, shape.vocab, seed=8)
    lo, nsl, n_gen = 256, 256, 8
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    r = 0.5
    idx, offs = synth.retained_lists(docs.lengths, r, seed=8)
    say("map", compute, kv)
    lg, tk = eng.map(handles, idx, offs, suffix, lo, nsl, n_gen, r=r)
    m = om.Model(shape, w)
    E = BOUND[(compute, kv)]
    refs = [om.map_eval(m, om.kv_build(m, docs.doc(i)), idx[offs[i]:offs[i + 1]], suffix, lo, nsl, n_gen)
            for i in range(len(docs.lengths))]
    checked, whole, err, fails = check_map(tk, lg, refs, E)
    say(f"map {compute}/{kv}: max-abs slice-logit error {err:.3g} (bound {E}); ids outside the band checked "
        f"{checked} of {len(refs) * n_gen}; items with all {n_gen} ids outside the band {whole}")
    assert not fails, fails[:5]
    assert checked >= 4, checked                                     # the id check is not vacuous
    if compute == "f32":
        assert whole >= len(docs.lengths) // 2, whole
    eng.close()


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
def test_join_pairs_match_oracle(device, compute, kv):
    shape = MICRO_GQA
    w = synth.make_weights(shape, 9, gain_jitter=0.1)
    docs = synth.make_docs_uniform(8, 1, 100, shape.vocab, seed=9)
    suffix = synth.suffix_tokens(17, shape.vocab, seed=9)
    pairs = synth.join_pairs(8, 12, seed=9)
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=9)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(8)]
    idx, offs, hs = [], [0], []
    for a, b in pairs:
        for x in (a, b):
            idx.append(lists[x])
            offs.append(offs[-1] + len(lists[x]))
            hs.append(handles[x])
    idx = np.concatenate(idx)
    say("join", compute, kv)
    lg, dec = eng.filter(np.array(hs, np.uint64), idx, np.array(offs), suffix, r=r, kind=K.KVOP_JOIN)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(8)]
    E = BOUND[(compute, kv)]
    lo_ref = []
    for p, (a, b) in enumerate(pairs):
        res = om.join_eval(m, caches[a], lists[a], caches[b], lists[b], suffix, synth.YES_ID, synth.NO_ID)
        assert np.max(np.abs(lg[p] - res.logits)) <= E, (p, np.max(np.abs(lg[p] - res.logits)))
        lo_ref.append(res.log_odds)
    assert decisions_agree_outside_band(lo_ref, dec, E)[0] == 0
    eng.close()


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16"), ("bf16", "fp8")])
@pytest.mark.parametrize("S", [1, 2, 33])
@pytest.mark.parametrize("n_items", [1, 5])
def test_suffix_length_and_batch_edges(device, compute, kv, S, n_items):
    """Filter, join and map at the edges of the suffix-row paths: a one-token suffix (layer 0's
    shared projection with period 1, no last-layer query trimming), a single item (no shared
    projection), and a suffix longer than one attention work item (33 rows against 32 per
    unit for two query heads per kv head: the last layer's work list takes the second unit)."""
    shape = MICRO_GQA
    w = synth.make_weights(shape, 40 + S, gain_jitter=0.1)
    docs = synth.make_docs_uniform(2 * n_items, 1, 90, shape.vocab, seed=40 + S)
    suffix = synth.suffix_tokens(S, shape.vocab, seed=40 + S)
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    m = om.Model(shape, w)
    caches = [om.kv_build(m, docs.doc(i)) for i in range(2 * n_items)]
    E = BOUND[(compute, kv)]
    r = 0.5
    idx1, offs1 = synth.retained_lists(docs.lengths, r, seed=40 + S)
    lists = [idx1[offs1[i]:offs1[i + 1]] for i in range(2 * n_items)]
    say("suffix edges", compute, S, n_items)
    # filter over the first n_items documents
    sel = list(range(n_items))
    idx = np.concatenate([lists[i] for i in sel])
    offs = np.concatenate([[0], np.cumsum([len(lists[i]) for i in sel])])
    lg, dec = eng.filter(handles[:n_items], idx, offs, suffix, r=r)
    lo = []
    for j, i in enumerate(sel):
        ref = om.filter_eval(m, caches[i], lists[i], suffix, synth.YES_ID, synth.NO_ID)
        assert np.max(np.abs(lg[j] - ref.logits)) <= E, ("filter", j)
        lo.append(ref.log_odds)
    assert decisions_agree_outside_band(lo, dec, E)[0] == 0
    # join of pairs (i, n_items + i)
    hs, jidx, joffs = [], [], [0]
    for i in range(n_items):
        for x in (i, n_items + i):
            hs.append(handles[x])
            jidx.append(lists[x])
            joffs.append(joffs[-1] + len(lists[x]))
    lg, dec = eng.filter(np.array(hs, np.uint64), np.concatenate(jidx), np.array(joffs), suffix, r=r,
                         kind=K.KVOP_JOIN)
    lo = []
    for i in range(n_items):
        ref = om.join_eval(m, caches[i], lists[i], caches[n_items + i], lists[n_items + i], suffix, synth.YES_ID,
                           synth.NO_ID)
        assert np.max(np.abs(lg[i] - ref.logits)) <= E, ("join", i)
        lo.append(ref.log_odds)
    assert decisions_agree_outside_band(lo, dec, E)[0] == 0
    # map (three greedy ids)
    mlg, tk = eng.map(handles[:n_items], idx, offs, suffix, 256, 256, 3, r=r)
    refs = [om.map_eval(m, caches[i], lists[i], suffix, 256, 256, 3) for i in sel]
    checked, whole, err, fails = check_map(tk, mlg, refs, E)
    assert not fails, fails
    eng.close()


# ----------------------------------------------------------------------------- invariances

@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "fp8")])
def test_permutation_and_batch_split_invariance(device, compute, kv):
    """Results of an item do not depend on the other items of the call or their order."""
    shape = MICRO_GQA
    w = synth.make_weights(shape, 10)
    docs = synth.make_docs_uniform(40, 1, 120, shape.vocab, seed=10)
    suffix = synth.suffix_tokens(9, shape.vocab, seed=10)
    eng = Engine(shape, w, compute, kv)
    handles = eng.build(docs)
    r = 0.25
    idx, offs = synth.retained_lists(docs.lengths, r, seed=10)
    lg, dec = eng.filter(handles, idx, offs, suffix, r=r)
    perm = np.random.default_rng(10).permutation(40)
    lists = [idx[offs[i]:offs[i + 1]] for i in range(40)]
    pidx = np.concatenate([lists[i] for i in perm])
    poffs = np.concatenate([[0], np.cumsum([len(lists[i]) for i in perm])])
    lg2, dec2 = eng.filter(handles[perm], pidx, poffs, suffix, r=r)
    np.testing.assert_array_equal(lg2, lg[perm])
    np.testing.assert_array_equal(dec2, dec[perm])
    # split into two calls
    h1 = eng.filter(handles[:13], idx[:offs[13]], offs[:14], suffix, r=r)
    h2 = eng.filter(handles[13:], idx[offs[13]:], offs[13:] - offs[13], suffix, r=r)
    np.testing.assert_array_equal(np.concatenate([h1[0], h2[0]]), lg)
    # an explicit full list at r = 1 is the r = 1 path
    fidx, foffs = synth.full_lists(docs.lengths)
    a = eng.filter(handles, fidx, foffs, suffix, r=1.0)
    b = eng.filter(handles, fidx, foffs, suffix, r=0.999, flags=K.KVOP_FLAG_ANY_COUNT)
    np.testing.assert_array_equal(a[0], b[0])
    eng.close()
