#!/usr/bin/env python3
"""Throughput of the KV-cached semantic filter on one MI355X.

Workload: the 16-layer d_model-2048 GQA decoder (16 query / 8 kv heads of 128, SwiGLU
5632, vocab 32000, normal(0, 0.02) weights, seed 0) over 4096 seeded synthetic documents
with log-normal lengths (median 512, sigma 1, clipped to [64, 4096]) and one 32-token
instruction suffix.  Caches are built once (kv_build, timed separately), then one step
is one op_eval of the filter over all 4096 documents at retention r; the retained rows
are seeded index lists (first four rows always, the rest uniform, sorted).

Paths timed: BF16 weights/activations with a BF16 cache (the headline), the same with an
FP8-E4M3 cache, and the plain FP32 path (FP32 cache; it exceeds HBM, so it runs in waves
that each build, evaluate and release part of the documents; only op_eval is timed).
Inputs are resident in HBM before every timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tuples/sec KV-cached semantic filter, BF16+proxy vs FP32 plain at ≤1% disagreement"
PEAK_BF16_TFLOPS = 2500.0
PEAK_F32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096, help="documents (the workload has 4096)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 path")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8-cache variant")
    ap.add_argument("--cpu-sample", type=int, default=4, help="documents the oracle is timed on (0: skip)")
    ap.add_argument("--tuning", default=None,
                    help="import this GEMM tuning table instead of running the autotuner (profiling runs)")
    ap.add_argument("--export-tuning", default=None, help="write the GEMM tuning table used to this file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with plain 1 GiB device copies (calibration of HBM byte counters)")
    ap.add_argument("--proxy-train", type=int, default=50000,
                    help="documents the proxy is trained on (labels from the full BF16 r=1 operator)")
    ap.add_argument("--proxy-eval", type=int, default=20000, help="fresh documents the proxy is evaluated on")
    ap.add_argument("--proxy-epochs", type=int, default=20)
    ap.add_argument("--no-proxy", action="store_true")
    ap.add_argument("--no-compression", action="store_true",
                    help="skip the expected-attention profiles (scored rebuild, selection, op_eval on them)")
    ap.add_argument("--workload", choices=["filter", "mixed"], default="filter",
                    help="filter: the plain filter at scale (default); mixed: filter/map/join in one pass")
    ap.add_argument("--no-padded", action="store_true", help="skip the padded-batching ablation")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--rs", type=float, nargs="*", default=None,
                    help="retention values to time besides r = 1 (default: the whole grid 1, 0.5, 0.25, 0.1)")
    ap.add_argument("--attention-variant", type=int, default=None,
                    help="attention kernel variant for the BF16/FP8 caches (default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the operator path has no multi-GPU mode (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2602_04430_amd import kvop as K
    from paper_2602_04430_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.attention_variant is not None:
        K.kvop_set_attention_kernel(args.attention_variant)
    if args.workload == "mixed":
        return bench_mixed(args, K, synth, dev)
    shape = synth.SCALE
    t0 = time.time()
    wl = synth.scale_filter(0, n=args.n)
    if args.rs:
        # a subset of the retention grid (profiling runs); r = 1 always stays in
        keep = tuple(r for r in wl.r_grid if r == 1.0 or r in args.rs)
        wl = synth.Workload(wl.name, wl.shape, wl.docs, wl.suffix, keep, wl.extra)
    docs = wl.docs
    n = len(docs.lengths)
    log(f"workload: {n} docs, sum L = {int(docs.lengths.sum())}, mean L = {docs.lengths.mean():.1f}")
    w = synth.make_weights(shape, 0)
    flat = torch.from_numpy(synth.pack_weights(shape, w)).to(dev)
    log(f"weights ready ({time.time() - t0:.1f} s)")
    cfg = K.make_cfg(shape)
    toks = torch.from_numpy(docs.tokens).to(dev)
    lists = {}
    for r in wl.r_grid:
        idx, offs = synth.retained_lists(docs.lengths, r, seed=0)
        lists[r] = (torch.from_numpy(idx).to(dev), offs)
    op = K.make_op(K.KVOP_FILTER, wl.suffix, synth.YES_ID, synth.NO_ID)
    stream = torch.cuda.current_stream()

    def timed_eval(pool, r, handles, sel=None, steps=1, warmup=0, lst=None):
        """op_eval over the documents (the seeded lists at r, or lst = (idx, offsets)); returns
        (ms per step, logits, decisions)."""
        idx, offs = lists[r] if lst is None else lst
        if sel is not None:
            # restrict to a contiguous range of documents [a, b)
            a, b = sel
            idx = idx[int(offs[a]):int(offs[b])]
            offs = offs[a:b + 1] - offs[a]
        m = len(handles)
        lg = torch.empty(m, 2, dtype=torch.float32, device=dev)
        dec = torch.empty(m, dtype=torch.int8, device=dev)
        for _ in range(warmup):
            K.kvop_op_eval(pool, op, r, idx, offs, handles, lg, dec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            K.kvop_op_eval(pool, op, r, idx, offs, handles, lg, dec)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, lg.cpu().numpy().astype(np.float64), dec.cpu().numpy()

    def build(pool, a, b, pooled=None):
        offs = docs.offsets[a:b + 1] - docs.offsets[a]
        sub = toks[int(docs.offsets[a]):int(docs.offsets[b])]
        torch.cuda.synchronize()
        tb = time.time()
        h = K.kvop_kv_build(pool, sub, offs, pooled)
        torch.cuda.synchronize()
        return h, time.time() - tb

    result = {}
    # ------------------------------------------------------------------ BF16 path
    mb = K.kvop_model_create(cfg, flat, K.KVOP_BF16)
    if args.tuning:
        with open(args.tuning) as f:
            K.kvop_tuning_import(f.read())
        tune_report = {"imported": os.path.basename(args.tuning)}
    else:
        tune_report = autotune(K, mb, [n * 32, 60000, n], "bf16")
    proxy, proxy_info = None, None
    if not args.no_proxy:
        proxy, proxy_info = train_proxy(K, synth, mb, shape, wl.suffix, args, dev, torch.cuda.current_stream())
    probe = K.kvop_pool_create(mb, K.KVOP_KV_BF16, 1 << 20)
    need = sum(K.kvop_doc_bytes(probe, int(L)) for L in docs.lengths)
    K.kvop_pool_destroy(probe)
    free = torch.cuda.mem_get_info()[0]
    log(f"BF16 cache needs {need / 2**30:.1f} GiB, free {free / 2**30:.1f} GiB")
    prof8, fp8_dec1 = None, None
    pool = K.kvop_pool_create(mb, K.KVOP_KV_BF16, need + (64 << 20))
    pooled = torch.empty(n, shape.d_model, dtype=torch.float32, device=dev)
    hb, t_build = build(pool, 0, n, pooled)
    tokens_total = int(docs.lengths.sum())
    log(f"BF16 kv_build: {t_build:.2f} s ({tokens_total / t_build:.0f} tokens/s)")
    result["kv_build_bf16_s"] = t_build
    per_r = {}
    bf16_out = {}
    cascade = None
    for r in wl.r_grid:
        steps = args.steps if r == 1.0 else max(1, args.steps // 2)
        ms, lg, dec = timed_eval(pool, r, hb, steps=steps, warmup=args.warmup)
        per_r[str(r)] = {"bf16_bf16kv_tuples_per_s": n / (ms / 1e3), "ms": ms}
        bf16_out[r] = (lg, dec)
        log(f"BF16 r={r}: {ms:.1f} ms/step, {n / (ms / 1e3):.0f} tuples/s")
        if r == 1.0 and proxy is not None:
            # the cascade is timed right after the plain r = 1 steps, so that both rates are
            # taken under the same clock (the GPU's clock drifts under long MFMA load)
            cascade = time_cascade(K, proxy, proxy_info, pool, hb, pooled, lists[1.0], op, bf16_out[1.0], n, args,
                                   dev, stream)
    headline_ms = per_r["1.0"]["ms"]
    padded = None
    if not args.no_padded:
        padded = time_padded(K, synth, pool, hb, lists, docs, wl, shape, per_r, args, dev)
    # per-kernel timing inside one r = 1 op_eval
    K.kvop_profile_start()
    timed_eval(pool, 1.0, hb, steps=1)
    prof = K.kvop_profile_stop()
    gu_launches = K.kvop_profile_launches("gemm_gate_up")
    log("profile (ms, launches):", {k: (round(v[0], 2), v[1]) for k, v in prof.items()})
    compression = None
    if not args.no_compression:
        compression = time_compression(K, pool, hb, op, lists[1.0], headline_ms, docs, toks, n, wl, t_build,
                                       timed_eval, bf16_out, args, dev, stream)
    K.kvop_pool_destroy(pool)
    # ------------------------------------------------------------------ FP8 cache
    if not args.no_fp8:
        probe = K.kvop_pool_create(mb, K.KVOP_KV_FP8, 1 << 20)
        need8 = sum(K.kvop_doc_bytes(probe, int(L)) for L in docs.lengths)
        K.kvop_pool_destroy(probe)
        pool8 = K.kvop_pool_create(mb, K.KVOP_KV_FP8, need8 + (64 << 20))
        h8, t8 = build(pool8, 0, n)
        log(f"FP8 kv_build: {t8:.2f} s")
        for r in wl.r_grid:
            ms, lg, dec = timed_eval(pool8, r, h8, steps=max(1, args.steps // 2), warmup=args.warmup)
            per_r[str(r)]["bf16_fp8kv_tuples_per_s"] = n / (ms / 1e3)
            per_r[str(r)]["fp8kv_vs_bf16kv_decision_disagreement"] = float(np.mean(dec != bf16_out[r][1]))
            if r == 1.0:
                fp8_dec1 = dec
            log(f"FP8 r={r}: {ms:.1f} ms/step")
        K.kvop_profile_start()
        timed_eval(pool8, 1.0, h8, steps=1)
        prof8 = K.kvop_profile_stop()
        log("profile FP8 cache, r = 1 (ms, launches):", {k: (round(v[0], 2), v[1]) for k, v in prof8.items()})
        K.kvop_pool_destroy(pool8)
    K.kvop_model_destroy(mb)
    # ------------------------------------------------------------------ FP32 plain path (waves)
    fp32 = None
    if not args.no_fp32:
        mf = K.kvop_model_create(cfg, flat, K.KVOP_F32)
        if not args.tuning:
            tune_report.update(autotune(K, mf, [n * 32, 60000, n], "f32"))
        probe = K.kvop_pool_create(mf, K.KVOP_KV_F32, 1 << 20)
        sizes = [K.kvop_doc_bytes(probe, int(L)) for L in docs.lengths]
        K.kvop_pool_destroy(probe)
        cap = min(torch.cuda.mem_get_info()[0] - (24 << 30), sum(sizes) + (2 << 30))
        poolf = K.kvop_pool_create(mf, K.KVOP_KV_F32, cap)
        ms_tot, t_build32, logits32, dec32 = 0.0, 0.0, [], []
        a = 0
        while a < n:
            b, acc = a, 0
            while b < n and acc + sizes[b] <= cap - (1 << 30):
                acc += sizes[b]
                b += 1
            hf, tb = build(poolf, a, b)
            t_build32 += tb
            ms, lg, dec = timed_eval(poolf, 1.0, hf, sel=(a, b), steps=max(10, args.steps), warmup=args.warmup)
            ms_tot += ms
            logits32.append(lg)
            dec32.append(dec)
            log(f"FP32 wave [{a}, {b}): build {tb:.1f} s, op_eval {ms:.1f} ms")
            K.kvop_kv_release(poolf, hf)
            a = b
        K.kvop_pool_destroy(poolf)
        K.kvop_model_destroy(mf)
        dec32 = np.concatenate(dec32)
        fp32 = {"tuples_per_s": n / (ms_tot / 1e3), "ms": ms_tot, "kv_build_s": t_build32,
                "logits": np.concatenate(logits32), "dec": dec32}
        log(f"FP32 plain: {fp32['tuples_per_s']:.0f} tuples/s")
    del flat
    torch.cuda.empty_cache()

    # ------------------------------------------------------------------ CPU baseline: the oracle
    cpu = None
    if args.cpu_sample > 0:
        cpu = oracle_baseline(shape, w, docs, wl.suffix, args.cpu_sample, bf16_out[1.0][0],
                              None if fp32 is None else fp32["logits"])

    # ------------------------------------------------------------------ roofline of the dominant kernel
    # the gate/up launches of layers 0..14 run all n * 32 suffix rows; the last layer's runs n rows
    gu_big = gu_launches[:shape.n_layers - 1]
    rows_main = n * 32
    gu_ms = sum(gu_big) / len(gu_big)
    gu_flops = 2.0 * shape.d_model * 2 * shape.d_ffn * rows_main
    achieved = gu_flops / (gu_ms / 1e3) / 1e12
    traffic = counted_traffic(tune_report.get("bf16/gate_up/M=%d" % rows_main))
    roofline = {"bound": "mfma", "kernel": "gemm_gate_up (bf16, SwiGLU epilogue, M=%d N=%d K=%d)"
                % (rows_main, 2 * shape.d_ffn, shape.d_model), "achieved": achieved,
                "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_TFLOPS, "traffic": traffic,
                "launches": len(gu_big), "avg_launch_ms": gu_ms, "flops_per_launch": gu_flops}
    tr_us = trace_launch_us()
    roofline["frac_from_committed_trace"] = None if tr_us is None else gu_flops / (tr_us * 1e-6) / 1e12 / PEAK_BF16_TFLOPS
    roofline["committed_trace_avg_launch_ms"] = None if tr_us is None else tr_us / 1e3
    att_ms, att_cnt = prof["attention"]
    k1 = int(docs.lengths.sum())
    att_bytes = (k1 + 32 * n) * 2 * shape.n_kv_heads * shape.head_dim * 2 * shape.n_layers
    roof_att = {"bound": "hbm", "achieved": att_bytes / (att_ms / 1e3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": att_bytes / (att_ms / 1e3) / 1e9 / PEAK_HBM_GBS, "avg_launch_ms": att_ms / max(1, att_cnt),
                "ms_per_step": att_ms}
    roof_att8 = None
    if prof8 is not None:
        # FP8 cache rows (1 byte per element, FP32 scales per 16-row block) plus the 32 own
        # rows per item in BF16, keys and values, 8 heads x 128, 16 layers
        a8_ms, a8_cnt = prof8["attention"]
        a8_bytes = (k1 * (shape.head_dim + 4 / 16) + 32 * n * shape.head_dim * 2) * 2 * shape.n_kv_heads * \
            shape.n_layers
        roof_att8 = {"bound": "hbm", "achieved": a8_bytes / (a8_ms / 1e3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": a8_bytes / (a8_ms / 1e3) / 1e9 / PEAK_HBM_GBS, "avg_launch_ms": a8_ms / max(1, a8_cnt),
                     "ms_per_step": a8_ms, "bf16_cache_attention_ms_per_step": att_ms}
    plain_value = n / (headline_ms / 1e3)
    value, step_ms, path = plain_value, headline_ms, "bf16 weights/activations, bf16 KV cache, no proxy"
    if cascade is not None:
        value, step_ms = cascade["tuples_per_s"], cascade["ms"]
        path = (f"learned proxy (tau={cascade['tau']}) answers the tuples it is confident on "
                f"({cascade['coverage']:.1%} of them), the full bf16 operator (bf16 KV cache, r=1) the rest; "
                f"{value / plain_value - 1:+.1%} over the plain bf16 rate")
    elif proxy_info is not None:
        path += " (the trained proxy met no tau at <= 1% held-out disagreement and is not used)"
    line = {
        "metric": METRIC, "value": value, "unit": "tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "plain semantic filter at scale: 16-layer d2048 GQA decoder, 4096 docs "
                               "lognormal(median 512, sigma 1) in [64,4096], 32-token suffix, r=1.0",
                   "path": path,
                   "docs": n, "sum_L": k1},
        "roofline": roofline,
        "roofline_attention": roof_att,
        "roofline_attention_fp8_cache": roof_att8,
        "kernel_ms_per_step": {k: round(v[0], 3) for k, v in prof.items()},
        "attention_kernel": K.kvop_get_attention_kernel(),
        "gemm_tiles": tune_report,
        "bf16_plain_tuples_per_s": plain_value,
        "proxy": cascade if cascade is not None else (None if proxy_info is None else
                                                       {"used": False, "training": proxy_info}),
        "per_r": per_r,
        "compression": compression,
        "padded_batching": padded,
        "kv_build_bf16_s": result["kv_build_bf16_s"],
        "cpu_baseline": cpu,
    }
    final_dec = None
    if fp32 is not None and cascade is not None:
        final_dec = cascade.pop("_final")
        cascade["vs_fp32_plain_decision_disagreement"] = float(np.mean(final_dec != fp32["dec"]))
    elif cascade is not None:
        cascade.pop("_final")
    if fp32 is not None:
        d16 = bf16_out[1.0][1]
        lo32 = fp32["logits"][:, 0] - fp32["logits"][:, 1]
        line["fp32_plain"] = {"tuples_per_s": fp32["tuples_per_s"], "ms": fp32["ms"],
                              "kv_build_s": fp32["kv_build_s"],
                              "bf16_vs_fp32_decision_disagreement": float(np.mean(d16 != fp32["dec"])),
                              "bf16_vs_fp32_max_abs_logit_diff": float(np.max(np.abs(bf16_out[1.0][0] - fp32["logits"]))),
                              "speedup_bf16_over_fp32": value / fp32["tuples_per_s"]}
        # decisions against the FP32 path (pinned by the oracle to 1e-4) outside the margin band
        # of each form's error bound, over all tuples at r = 1; the bounds are the ones the
        # full-size parity test derives from the oracle alone
        bounds = load_scale_bounds()
        if bounds:
            band = {}
            for tag, dec, E in (("bf16_bf16kv", d16, bounds.get("E_bf16")),
                                ("bf16_fp8kv", fp8_dec1, bounds.get("E_fp8")),
                                ("bf16_proxy_cascade", None if cascade is None else final_dec, bounds.get("E_bf16"))):
                if dec is None or E is None:
                    continue
                out = np.abs(lo32) >= 2 * (E + 1e-4)
                band[tag] = {"E": E, "in_band_fraction": float(1 - out.mean()),
                             "disagreement_outside_band": float(np.mean((dec != fp32["dec"]) & out)),
                             "disagreement_all": float(np.mean(dec != fp32["dec"]))}
            line["fp32_plain"]["decisions_vs_fp32_outside_band"] = band
    print(json.dumps(line), flush=True)
    if args.export_tuning:
        with open(args.export_tuning, "w") as f:
            f.write(K.kvop_tuning_export())
    if args.copy_probe:
        copy_probe(dev)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(json.dumps(line) + "\n")


WAVE_ROWS = 32768            # suffix rows per wave in the mixed bench
DEFAULT_WAVE_ROWS = 131072   # the library's default
SMALL_WAVE_ROWS = 2048       # launch-bound regime of the mixed bench


def compare(acc, ref, out):
    """Accumulate the differences of one mode's outputs (lf, df, lm, tm, lj, dj) from ref."""
    acc["filter_logits"] = max(acc["filter_logits"], float(np.max(np.abs(ref[0] - out[0]), initial=0)))
    acc["map_logits"] = max(acc["map_logits"], float(np.max(np.abs(ref[2] - out[2]), initial=0)))
    acc["join_logits"] = max(acc["join_logits"], float(np.max(np.abs(ref[4] - out[4]), initial=0)))
    acc["map_tokens"] += int(np.sum(np.any(ref[3] != out[3], axis=1)))
    acc["decisions"] += int(np.sum(ref[1] != out[1]) + np.sum(ref[5] != out[5]))


def bench_mixed(args, K, synth, dev):
    """Mixed operators (batching form): 16384 documents, lengths lognormal (median 384,
    sigma 1) in [16, 8192]; one third filter items, one third map items (8 greedy ids over
    the label slice [256, 512)), one third join-side documents forming 2048 pairs; one
    32-token suffix per operator; r = 1; BF16 weights/activations and BF16 cache.  The
    caches exceed HBM, so the items are processed in groups whose documents fit: each
    group's caches are built (untimed), then its items are evaluated (timed)."""
    import torch
    from paper_2602_04430_amd import batching
    shape = synth.SCALE
    wl = synth.mixed_batch(0)
    docs = wl.docs
    fdocs, mdocs, pairs = wl.extra["filter_docs"], wl.extra["map_docs"], wl.extra["join_pairs"]
    n_gen, lo, nl = synth.MAP_TOKENS, synth.MAP_SLICE[0], synth.MAP_SLICE[1]
    w = synth.make_weights(shape, 0)
    flat = torch.from_numpy(synth.pack_weights(shape, w)).to(dev)
    del w
    mb = K.kvop_model_create(K.make_cfg(shape), flat, K.KVOP_BF16)
    del flat
    torch.cuda.empty_cache()
    opf = K.make_op(K.KVOP_FILTER, wl.suffix, synth.YES_ID, synth.NO_ID)
    opm = K.make_op(K.KVOP_MAP, wl.extra["suffix_map"], label_lo=lo, label_n=nl, n_gen=n_gen)
    opj = K.make_op(K.KVOP_JOIN, wl.extra["suffix_join"], synth.YES_ID, synth.NO_ID)
    probe = K.kvop_pool_create(mb, K.KVOP_KV_BF16, 1 << 20)
    dbytes = np.array([K.kvop_doc_bytes(probe, int(L)) for L in docs.lengths])
    K.kvop_pool_destroy(probe)
    cap = torch.cuda.mem_get_info()[0] - (48 << 30)
    pool = K.kvop_pool_create(mb, K.KVOP_KV_BF16, cap)
    G = batching.plan_groups(dbytes, fdocs, mdocs, pairs, cap - (2 << 30))
    log(f"mixed workload: {len(fdocs)} filter, {len(mdocs)} map, {len(pairs)} join items in {G} groups")
    # tune the projections at the row counts the waves run: full waves, and the per-operator
    # last-layer rows and decode rows
    sizes = [len(np.array_split(x, G)[0]) for x in (fdocs, mdocs, pairs)]
    n_waves = -(-32 * sum(sizes) // WAVE_ROWS)
    per = [-(-x // n_waves) for x in sizes]
    tiles = autotune(K, mb, sorted({32 * sum(per), per[0], per[1], per[2], sizes[1]}), "bf16")
    stream = torch.cuda.current_stream()
    modes = {"graph_persistent": K.KVOP_MIXED_PERSISTENT | K.KVOP_MIXED_GRAPH,
             "persistent": K.KVOP_MIXED_PERSISTENT, "eager": 0}
    t_mode = {k: 0.0 for k in list(modes) + ["separate_calls"]}
    diff = {k: {"filter_logits": 0.0, "join_logits": 0.0, "map_logits": 0.0, "map_tokens": 0, "decisions": 0}
            for k in t_mode if k != "graph_persistent"}
    t_build = 0.0
    n_items = 0
    small = {"wave_rows": SMALL_WAVE_ROWS, "group": 0, "items_per_s": {}, "differences": {}}
    # waves of WAVE_ROWS suffix rows: each group then runs several full waves, so the
    # captured graph is replayed (the first wave and a partial last wave run directly)
    K.kvop_set_wave_rows(WAVE_ROWS)
    for g in range(G):
        fg, mg, pg = batching.group_parts(fdocs, mdocs, pairs, G, g)
        need = batching.group_docs(fg, mg, pg)
        sub = docs.subset(need)
        pos = {dd: i for i, dd in enumerate(need)}
        torch.cuda.synchronize()
        t0 = time.time()
        hsub = K.kvop_kv_build(pool, torch.from_numpy(sub.tokens).to(dev), sub.offsets)
        torch.cuda.synchronize()
        t_build += time.time() - t0
        fidx, foffs = synth.full_lists(sub.lengths)
        idx = torch.from_numpy(fidx).to(dev)
        # lists/handles per item: filter docs, map docs, join pairs (two lists each)
        lists_f = [pos[dd] for dd in fg]
        lists_m = [pos[dd] for dd in mg]
        lists_j = [x for a, b in pg for x in (pos[a], pos[b])]
        all_lists = lists_f + lists_m + lists_j
        L_off = np.concatenate([[0], np.cumsum(sub.lengths[all_lists])])
        sel_idx = torch.cat([idx[int(foffs[i]):int(foffs[i + 1])] for i in all_lists])
        hs = hsub[all_lists]
        nf, nm, nj = len(lists_f), len(lists_m), len(pg)
        item_op, item_list = batching.interleave(nf, nm, nj, seed=g)      # operators interleaved
        # a mixed call writes operator k's outputs in the order its items appear in the
        # interleaved list; the separate calls write them in list order
        order = batching.output_order(item_op, item_list, nf, nm)
        n_items += nf + nm + nj
        lf = torch.empty(nf, 2, device=dev)
        df = torch.empty(nf, dtype=torch.int8, device=dev)
        lm = torch.empty(nm, n_gen, nl, device=dev)
        tm = torch.empty(nm, n_gen, dtype=torch.int32, device=dev)
        lj = torch.empty(nj, 2, device=dev)
        dj = torch.empty(nj, dtype=torch.int8, device=dev)
        ops = [(opf, lf, df, None), (opm, lm, None, tm), (opj, lj, dj, None)]

        def timed(fn):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.time()
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return max(e0.elapsed_time(e1), (time.time() - t0) * 1e3)

        def outputs(reorder=False):
            o = [x.cpu().numpy() for x in (lf, df, lm, tm, lj, dj)]
            if reorder:
                o = [o[0][order[0]], o[1][order[0]], o[2][order[1]], o[3][order[1]], o[4][order[2]], o[5][order[2]]]
            return o

        ref = None
        for name, flags in modes.items():
            K.kvop_mixed_eval(pool, ops, 1.0, sel_idx, L_off, hs, item_op, item_list, flags)     # warm-up
            t_mode[name] += timed(lambda: K.kvop_mixed_eval(pool, ops, 1.0, sel_idx, L_off, hs, item_op, item_list,
                                                            flags))
            out = outputs()
            if ref is None:
                ref = out
            else:
                compare(diff[name], ref, out)

        def separate():
            K.kvop_op_eval(pool, opf, 1.0, sel_idx, L_off[:nf + 1], hs[:nf], lf, df)
            K.kvop_op_eval(pool, opm, 1.0, sel_idx, L_off[nf:nf + nm + 1], hs[nf:nf + nm], lm, None, tm)
            K.kvop_op_eval(pool, opj, 1.0, sel_idx, L_off[nf + nm:], hs[nf + nm:], lj, dj)
        t_mode["separate_calls"] += timed(separate)
        compare(diff["separate_calls"], ref, outputs(reorder=True))
        if g == 0:
            # launch-bound regime: the same items in waves of SMALL_WAVE_ROWS rows, where the
            # per-launch cost of ~10 launches per layer per wave is no longer hidden
            K.kvop_set_wave_rows(SMALL_WAVE_ROWS)
            for name, flags in (("eager", 0), ("graph", K.KVOP_MIXED_GRAPH),
                                ("graph_persistent", K.KVOP_MIXED_GRAPH | K.KVOP_MIXED_PERSISTENT)):
                K.kvop_mixed_eval(pool, ops, 1.0, sel_idx, L_off, hs, item_op, item_list, flags)   # warm-up
                ms_small = timed(lambda: K.kvop_mixed_eval(pool, ops, 1.0, sel_idx, L_off, hs, item_op, item_list,
                                                           flags))
                small["items_per_s"][name] = (nf + nm + nj) / (ms_small / 1e3)
                compare(small["differences"].setdefault(name, {"filter_logits": 0.0, "join_logits": 0.0,
                                                               "map_logits": 0.0, "map_tokens": 0, "decisions": 0}),
                        ref, outputs())
            K.kvop_set_wave_rows(WAVE_ROWS)
            log(f"waves of {SMALL_WAVE_ROWS} rows (group 0): {small}")
        if g == 0:        # where the time goes: per-class profile of one eager call and of the separate calls
            K.kvop_profile_start()
            K.kvop_mixed_eval(pool, ops, 1.0, sel_idx, L_off, hs, item_op, item_list, 0)
            prof_mixed = {k: round(v[0], 1) for k, v in K.kvop_profile_stop().items()}
            K.kvop_profile_start()
            separate()
            prof_sep = {k: round(v[0], 1) for k, v in K.kvop_profile_stop().items()}
            log(f"profile (ms) eager mixed: {prof_mixed}")
            log(f"profile (ms) separate calls: {prof_sep}")
        log(f"group {g}: {len(need)} docs, {nf}/{nm}/{nj} items, graph {t_mode['graph_persistent']:.0f} ms so far; "
            f"differences from the graph mode: {diff}")
        K.kvop_kv_release(pool, hsub)
    K.kvop_set_wave_rows(DEFAULT_WAVE_ROWS)
    K.kvop_pool_destroy(pool)
    K.kvop_model_destroy(mb)
    # the value is the library's default mode (plain launches, two-stage attention); the graph
    # and persistent modes are reported beside it
    ms = t_mode["eager"]
    # summed roofline bound of the mix (r = 1, BF16 cache): per item, its projections at the
    # BF16 MFMA peak (1.510 GFLOP per suffix row, 32 rows; a map adds 7 decode rows and its
    # slice head) plus the keys/values its attention must read at 8 TB/s (65 536 bytes per
    # row: 16 layers x 8 kv heads x 128 x K and V x 2 bytes): a filter reads L + 32 rows, a join
    # L_A + L_B + 32, a map L + 32 for the suffix and L + 32 + t at decode step t = 1..7
    gf_row = shape.gemm_flops_per_token()
    kv_row = shape.kv_elems_per_token() * 2
    Lf = docs.lengths[fdocs].astype(np.float64)
    Lm = docs.lengths[mdocs].astype(np.float64)
    Lj = (docs.lengths[pairs[:, 0]] + docs.lengths[pairs[:, 1]]).astype(np.float64)
    flops = gf_row * 32 * (len(Lf) + len(Lm) + len(Lj)) + len(Lm) * (n_gen - 1) * (gf_row + 2 * shape.d_model * nl)
    kv_bytes = kv_row * (np.sum(Lf + 32) + np.sum(Lj + 32) + np.sum(Lm + 32) +
                         np.sum([np.sum(Lm + 32 + t) for t in range(1, n_gen)]))
    bound_ms = (flops / (PEAK_BF16_TFLOPS * 1e12) + kv_bytes / (PEAK_HBM_GBS * 1e9)) * 1e3
    roof = {"bound": "mfma+hbm (summed per item)", "bound_ms": bound_ms, "gemm_tflop": flops / 1e12,
            "kv_gb": kv_bytes / 1e9, "frac_by_mode": {k: bound_ms / v for k, v in t_mode.items()}}
    line = {"metric": "tuples/sec mixed filter/map/join, one pass per wave (batching form)",
            "value": n_items / (ms / 1e3), "unit": "items/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic",
            "config": {"workload": "mixed operators: 16384 docs lognormal(median 384, sigma 1) in [16, 8192]; "
                                   "5462 filter, 5461 map (8 ids over 256 labels), 2048 join pairs; r=1; bf16",
                       "groups": G, "items": n_items},
            "modes_items_per_s": {k: n_items / (v / 1e3) for k, v in t_mode.items()},
            "differences_from_graph_mode": diff, "wave_rows": WAVE_ROWS, "small_waves": small,
            "profile_group0_ms": {"eager_mixed": prof_mixed, "separate_calls": prof_sep},
            "kv_build_s": t_build, "gemm_tiles": tiles, "roofline_summed_bound": roof}
    print(json.dumps(line), flush=True)


PAD_BUDGET = 32 << 30    # bytes of padded cache one batch may hold (the padded form's batch rule)


def time_padded(K, synth, pool, handles, lists, docs, wl, shape, per_r, args, dev):
    """Padded batching as an ablation (KVOP_FLAG_PADDED: every item's attention runs over its
    batch's largest key count).  Two forms per r: one batch of all documents (padding alone),
    and batches formed in input order as the largest that keep batch size x padded length
    within PAD_BUDGET of cache (padding plus the smaller batches it forces); each against the
    variable-length rate of the same r."""
    import torch
    n = len(docs.lengths)
    row_bytes = shape.n_layers * 2 * shape.n_kv_heads * shape.head_dim * 2
    op = K.make_op(K.KVOP_FILTER, wl.suffix, synth.YES_ID, synth.NO_ID, flags=K.KVOP_FLAG_PADDED)
    out = {"budget_bytes": PAD_BUDGET, "per_r": {}}
    lg = torch.empty(n, 2, dtype=torch.float32, device=dev)
    dec = torch.empty(n, dtype=torch.int8, device=dev)
    for r in wl.r_grid:
        idx, offs = lists[r]
        k = np.diff(offs)
        batches, a = [], 0
        while a < n:
            b, kmax = a + 1, int(k[a])
            while b < n and (b + 1 - a) * max(kmax, int(k[b])) * row_bytes <= PAD_BUDGET:
                kmax = max(kmax, int(k[b]))
                b += 1
            batches.append((a, b))
            a = b

        def run(bs):
            for a, b in bs:
                sub = idx[int(offs[a]):int(offs[b])]
                K.kvop_op_eval(pool, op, r, sub, offs[a:b + 1] - offs[a], handles[a:b], lg[a:b], dec[a:b])

        row = {"varlen_ms": per_r[str(r)]["ms"], "real_keys": int(k.sum())}
        for name, bs in (("one_batch", [(0, n)]), ("budget_batches", batches)):
            run(bs)
            torch.cuda.synchronize()
            t0 = time.time()
            for _ in range(max(1, args.steps // 2)):
                run(bs)
            torch.cuda.synchronize()
            ms = (time.time() - t0) * 1e3 / max(1, args.steps // 2)
            padded_keys = sum((b - a) * int(k[a:b].max()) for a, b in bs)
            row[name] = {"batches": len(bs), "ms": ms, "tuples_per_s": n / (ms / 1e3),
                         "padded_keys_over_real": padded_keys / int(k.sum()),
                         "varlen_speedup": ms / per_r[str(r)]["ms"]}
        out["per_r"][str(r)] = row
        log(f"padded r={r}: one batch {row['one_batch']['ms']:.1f} ms "
            f"(keys x{row['one_batch']['padded_keys_over_real']:.2f}), {len(batches)} budget batches "
            f"{row['budget_batches']['ms']:.1f} ms (keys x{row['budget_batches']['padded_keys_over_real']:.2f}); "
            f"varlen {row['varlen_ms']:.1f} ms")
    return out


def time_compression(K, pool, handles, op, lists1, ms1, docs, toks, n, wl, t_build, timed_eval, bf16_out, args,
                     dev, stream):
    """Compressed profiles by expected attention: the caches are rebuilt with scoring (timed
    against the plain build), retained lists are selected at each r < 1 (timed), and the
    filter runs over them; decisions and log-odds are compared with r = 1 next to those of
    the seeded random lists at the same r."""
    import torch
    K.kvop_kv_release(pool, handles)
    n_future = len(wl.suffix)
    scores = torch.empty(int(docs.lengths.sum()), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    K.kvop_profile_start()
    t0 = time.time()
    hs = K.kvop_kv_build_scored(pool, toks, docs.offsets, n_future, scores)
    torch.cuda.synchronize()
    t_scored = time.time() - t0
    prof = K.kvop_profile_stop()
    log(f"kv_build with expected-attention scores: {t_scored:.2f} s (plain {t_build:.2f} s), "
        f"scoring kernels {prof['ea_scores'][0]:.0f} ms")
    lo1 = bf16_out[1.0][0][:, 0] - bf16_out[1.0][0][:, 1]
    dec1 = bf16_out[1.0][1]
    out = {"method": f"expected attention, future queries at L .. L+{n_future - 1}", "kv_build_s": t_build,
           "kv_build_scored_s": t_scored, "scoring_kernels_ms": prof["ea_scores"][0], "per_r": {}}
    ea_lists, ea_lo = {}, {}
    for r in wl.r_grid:
        if r == 1.0:
            continue
        total = sum(K.kvop_retained_count(r, int(L)) for L in docs.lengths)
        idx = torch.empty(total, dtype=torch.int32, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        io = K.kvop_ea_select(pool, scores, docs.offsets, r, idx)
        e1.record(stream)
        torch.cuda.synchronize()
        sel_ms = e0.elapsed_time(e1)
        ms, lg, dec = timed_eval(pool, r, hs, steps=max(1, args.steps // 2), warmup=args.warmup, lst=(idx, io))
        lo = lg[:, 0] - lg[:, 1]
        ea_lists[r], ea_lo[r] = (idx, io), lo
        lo_rand = bf16_out[r][0][:, 0] - bf16_out[r][0][:, 1]
        row = {"select_ms": sel_ms, "tuples_per_s": n / (ms / 1e3), "ms": ms,
               "decision_agreement_vs_r1": float(np.mean(dec == dec1)),
               "random_lists_decision_agreement_vs_r1": float(np.mean(bf16_out[r][1] == dec1)),
               "mean_abs_logodds_change_vs_r1": float(np.mean(np.abs(lo - lo1))),
               "random_lists_mean_abs_logodds_change_vs_r1": float(np.mean(np.abs(lo_rand - lo1)))}
        out["per_r"][str(r)] = row
        log(f"expected-attention lists r={r}: select {sel_ms:.2f} ms, op_eval {ms:.1f} ms; decisions agree with r=1 "
            f"{row['decision_agreement_vs_r1']:.3f} (random lists {row['random_lists_decision_agreement_vs_r1']:.3f}), "
            f"mean |dLO| {row['mean_abs_logodds_change_vs_r1']:.3f} (random {row['random_lists_mean_abs_logodds_change_vs_r1']:.3f})")
    ms_r = {float(r): row["ms"] for r, row in out["per_r"].items()}
    ms_r[1.0] = ms1
    ea_lo[1.0] = lo1
    out["ladder"] = time_ladder(K, pool, hs, op, n, ea_lists, lists1, ea_lo, dec1, ms_r, args, dev)
    return out


LADDER = (0.1, 0.25, 0.5, 1.0)
CALIB_DOCS = 512         # documents the thresholds are calibrated on
CALIB_PRECISION = 0.99   # agreement with r = 1 required of an early stage's decisions


def calibrate_theta(lo, ref_dec, target):
    """Smallest symmetric threshold theta such that the items with |LO| > theta, decided by
    sign, agree with the reference decisions on at least `target` of them (inf if none)."""
    a = np.abs(lo)
    order = np.argsort(-a, kind="stable")
    agree = np.cumsum((lo[order] > 0).astype(np.int8) == ref_dec[order]) / np.arange(1, len(lo) + 1)
    ok = np.flatnonzero(agree >= target)
    if len(ok) == 0:
        return float("inf")
    k = int(ok[-1]) + 1                       # the top-k items by |LO| meet the target
    return float(np.float32(a[order[k]] if k < len(a) else 0.0))


def time_ladder(K, pool, handles, op, n, ea_lists, lists1, ea_lo, dec1, ms_r, args, dev):
    """Filter cascade over the expected-attention profiles r = 0.1 -> 0.25 -> 0.5 -> 1, one
    kvop_cascade_eval over all documents timed per step, under two threshold rules fixed on
    the first documents: (a) the smallest thresholds whose decisions agree with r = 1 at the
    target precision; (b) thresholds deciding half of the remaining items at each early stage
    (a rule that exercises the forwarding whatever the model's quality).  Each is reported
    with Eq. 4's cost predicted from the measured per-profile step times, so the executor's
    own overhead is the difference."""
    import torch
    c = min(CALIB_DOCS, n)
    rules = {"precision_%g" % CALIB_PRECISION:
             [calibrate_theta(ea_lo[r][:c], dec1[:c], CALIB_PRECISION) for r in LADDER[:-1]] + [0.0],
             "half_per_stage": [float(np.float32(np.quantile(np.abs(ea_lo[r][:c]), 0.5))) for r in LADDER[:-1]] + [0.0]}
    lg = torch.empty(n, 2, dtype=torch.float32, device=dev)
    dec = torch.empty(n, dtype=torch.int8, device=dev)
    stg = torch.empty(n, dtype=torch.int8, device=dev)
    out = {"stages_r": list(LADDER), "calibration_docs": c}
    for name, th in rules.items():
        stages = [(r, t, -t, *(ea_lists[r] if r < 1.0 else lists1)) for r, t in zip(LADDER, th)]
        for _ in range(args.warmup):
            K.kvop_cascade_eval(pool, op, stages, handles, lg, dec, stg)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(args.steps):
            proc = K.kvop_cascade_eval(pool, op, stages, handles, lg, dec, stg)
        torch.cuda.synchronize()
        ms = (time.time() - t0) * 1e3 / args.steps
        d = dec.cpu().numpy()
        pred = sum(int(p) / n * ms_r[r] for p, r in zip(proc, LADDER))
        row = {"theta": th, "tuples_per_s": n / (ms / 1e3), "ms": ms, "processed": [int(x) for x in proc],
               "eq4_predicted_ms": pred, "decision_agreement_vs_r1": float(np.mean(d == dec1)),
               "decision_agreement_vs_r1_outside_calibration": float(np.mean(d[c:] == dec1[c:])) if n > c else None}
        out[name] = row
        log(f"cascade ladder {LADDER} [{name}]: theta {[round(x, 3) for x in th]}, processed {row['processed']}, "
            f"{ms:.1f} ms (Eq. 4 predicts {pred:.1f}), {row['tuples_per_s']:.0f} tuples/s, "
            f"agreement with r=1 {row['decision_agreement_vs_r1']:.4f}")
    out["optimized"] = optimized_plan(K, pool, handles, op, n, ea_lists, lists1, ea_lo, dec1, ms_r, args, dev, c)
    return out


PLAN_TARGETS = (0.9, 0.9, 0.95)   # recall target, precision target, credible level


def optimized_plan(K, pool, handles, op, n, ea_lists, lists1, ea_lo, dec1, ms_r, args, dev, c):
    """The optimizer (kvop_plan_optimize) on the profiled log-odds of the first c documents
    at every profile of the ladder, costs = measured per-tuple times, gold = the r = 1
    decisions; its plan then runs over all documents through kvop_cascade_eval, and the
    realised recall and precision against r = 1 are reported beside the sample's bounds."""
    import torch
    lo = np.stack([ea_lo[r][:c] for r in LADDER[:-1]] + [ea_lo[1.0][:c]])
    cost = np.array([ms_r[r] / n for r in LADDER])
    gold = (dec1[:c] == 1).astype(np.int8)
    pb = K.PlanProblem([lo], [cost], [gold], *PLAN_TARGETS)
    t0 = time.time()
    res = K.kvop_plan_optimize(pb, steps=300)
    opt_ms = (time.time() - t0) * 1e3
    sel = [i for i in range(len(LADDER)) if res["selected"][i]]
    rep = res["report"]
    row = {"targets": {"recall": PLAN_TARGETS[0], "precision": PLAN_TARGETS[1], "alpha": PLAN_TARGETS[2]},
           "sample_docs": c, "optimizer_ms": opt_ms, "selected_r": [LADDER[i] for i in sel],
           "theta_pos": [float(res["theta_pos"][i]) for i in sel], "theta_neg": [float(res["theta_neg"][i]) for i in sel],
           "sample_report": rep}
    if sel:
        stages = [(LADDER[i], float(res["theta_pos"][i]), float(res["theta_neg"][i]),
                   *(ea_lists[LADDER[i]] if LADDER[i] < 1.0 else lists1)) for i in sel]
        lg = torch.empty(n, 2, dtype=torch.float32, device=dev)
        dec = torch.empty(n, dtype=torch.int8, device=dev)
        stg = torch.empty(n, dtype=torch.int8, device=dev)
        K.kvop_cascade_eval(pool, op, stages, handles, lg, dec, stg)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(args.steps):
            proc = K.kvop_cascade_eval(pool, op, stages, handles, lg, dec, stg)
        torch.cuda.synchronize()
        ms = (time.time() - t0) * 1e3 / args.steps
        acc = dec.cpu().numpy() == 1
        g = dec1 == 1
        tp = int(np.sum(acc & g))
        row.update({"tuples_per_s": n / (ms / 1e3), "ms": ms, "processed": [int(x) for x in proc],
                    "recall_vs_r1": tp / max(1, int(g.sum())), "precision_vs_r1": tp / max(1, int(acc.sum()))})
    log(f"optimized plan: r {row['selected_r']}, theta+ {[round(x, 3) for x in row['theta_pos']]}, "
        f"sample bounds R {rep['recall_lb']:.3f} P {rep['precision_lb']:.3f}, cost {rep['cost_frac']:.3f}; "
        f"optimizer {opt_ms:.0f} ms; all docs: {row.get('tuples_per_s', 0):.0f} tuples/s, "
        f"recall {row.get('recall_vs_r1', 0):.4f} precision {row.get('precision_vs_r1', 0):.4f}")
    return row


def autotune(K, model, rows_list, tag):
    """Time every projection tile candidate at the row counts the run uses and keep the
    fastest (the library's own autotuner); returns the chosen tiles."""
    chosen = {}
    for rows in rows_list:
        rep = K.kvop_autotune(model, rows, 3)
        for line in rep.splitlines():
            if line.startswith("best "):
                _, name, m, tile = line.split()
                chosen[f"{tag}/{name}/{m}"] = tile
    log(f"autotune {tag}: {chosen}")
    return chosen


TAUS = (0.9, 0.95, 0.99)


def _proxy_waves(K, synth, mb, docs, suffix, dev, per_wave=None):
    """Build the documents' caches in waves that fit HBM; for each wave write the pooled
    features and the full BF16 r=1 operator's log-odds, call per_wave(a, b, pool, handles,
    idx, ioffs, op, feats) while the caches are resident, then release them.  Returns
    (features [n, d] on the device, log-odds [n])."""
    import torch
    n = len(docs.lengths)
    feats = torch.empty(n, synth.SCALE.d_model, dtype=torch.float32, device=dev)
    lo = np.empty(n, np.float64)
    probe = K.kvop_pool_create(mb, K.KVOP_KV_BF16, 1 << 20)
    sizes = [K.kvop_doc_bytes(probe, int(L)) for L in docs.lengths]
    K.kvop_pool_destroy(probe)
    cap = min(torch.cuda.mem_get_info()[0] - (40 << 30), sum(sizes) + (1 << 30))
    pool = K.kvop_pool_create(mb, K.KVOP_KV_BF16, cap)
    toks = torch.from_numpy(docs.tokens).to(dev)
    op = K.make_op(K.KVOP_FILTER, suffix, synth.YES_ID, synth.NO_ID)
    a = 0
    while a < n:
        b, acc = a, 0
        while b < n and acc + sizes[b] <= cap - (1 << 28):
            acc += sizes[b]
            b += 1
        offs = docs.offsets[a:b + 1] - docs.offsets[a]
        h = K.kvop_kv_build(pool, toks[int(docs.offsets[a]):int(docs.offsets[b])], offs, feats[a:b])
        idx, ioffs = synth.full_lists(docs.lengths[a:b])
        idx = torch.from_numpy(idx).to(dev)
        lg = torch.empty(b - a, 2, dtype=torch.float32, device=dev)
        K.kvop_op_eval(pool, op, 1.0, idx, ioffs, h, lg, None)
        lgc = lg.cpu().numpy().astype(np.float64)
        lo[a:b] = lgc[:, 0] - lgc[:, 1]
        if per_wave is not None:
            per_wave(a, b, pool, h, idx, ioffs, op, feats)
        K.kvop_kv_release(pool, h)
        a = b
    K.kvop_pool_destroy(pool)
    return feats, lo


def train_proxy(K, synth, mb, shape, suffix, args, dev, stream):
    """The learned proxy at its full configuration: a 2048 -> 256 -> 2 MLP on pooled features,
    trained on args.proxy_train seeded documents labelled by the full BF16 r = 1 operator
    (a tenth held out for early stopping and the choice of tau), then evaluated on
    args.proxy_eval fresh documents from another seed stream.  On the fresh documents, per
    tau: coverage, disagreement with the full operator (over all tuples and over the
    answered ones) and the timed rate of the cascade (proxy, then the full operator on the
    tuples it leaves unsure) beside the full operator's own rate.  tau* is the smallest tau
    whose held-out disagreement is at most 1%; if none qualifies the proxy is not used."""
    import torch
    t0 = time.time()
    tr_docs, ev_docs = synth.proxy_split(0, n_train=args.proxy_train, n_eval=args.proxy_eval)
    feats, lo = _proxy_waves(K, synth, mb, tr_docs, suffix, dev)
    n = len(lo)
    t_data = time.time() - t0
    labels_np = (lo > 0).astype(np.int32)
    pos_frac = float(labels_np.mean())
    log(f"proxy training data: {n} documents in {t_data:.1f} s, {pos_frac:.3f} accepted")
    n_tr = n - n // 10
    labels = torch.from_numpy(labels_np).to(dev)
    p0 = synth.proxy_init(shape.d_model, 256, 2, 0)
    packed = np.concatenate([p0["w1"].ravel(), p0["b1"], p0["w2"].ravel(), p0["b2"]]).astype(np.float32)
    px = K.kvop_proxy_create(shape.d_model, 256, torch.from_numpy(packed).to(dev))
    K.kvop_proxy_fit_standardizer(px, feats[:n_tr])
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    bs = 512
    nh = n - n_tr
    cls = torch.empty(nh, dtype=torch.int8, device=dev)
    conf = torch.empty(nh, dtype=torch.float32, device=dev)
    ans = torch.empty(nh, dtype=torch.int8, device=dev)
    best = torch.empty(shape.d_model * 256 + 3 * 256 + 2, dtype=torch.float32, device=dev)
    best_loss, best_ep = float("inf"), -1

    def val_loss():
        K.kvop_proxy_infer(px, feats[n_tr:], 0.5, cls, conf, ans)
        c, cf = cls.cpu().numpy(), conf.cpu().numpy().astype(np.float64)
        p_true = np.where(c == labels_np[n_tr:], cf, 1.0 - cf)
        return float(-np.mean(np.log(np.maximum(p_true, 1e-12))))

    t1 = time.time()
    history = []
    for ep in range(args.proxy_epochs):
        order = torch.from_numpy(synth.proxy_order(n_tr, ep, 0)).to(dev)
        for s0 in range(0, n_tr - bs + 1, bs):
            K.kvop_proxy_train_step(px, feats, labels, order[s0:s0 + bs], bs, 1e-3, loss)
        vl = val_loss()
        history.append(round(vl, 5))
        if vl < best_loss:
            best_loss, best_ep = vl, ep
            K.kvop_proxy_params(px, best)
        log(f"proxy epoch {ep}: train loss {float(loss.item()):.4f}, validation loss {vl:.4f}")
    torch.cuda.synchronize()
    t_train = time.time() - t1
    # early stopping: keep the parameters of the best validation epoch
    K.kvop_proxy_destroy(px)
    px = K.kvop_proxy_create(shape.d_model, 256, best)
    K.kvop_proxy_fit_standardizer(px, feats[:n_tr])
    held = {}
    tau_star = None
    for tau in TAUS:
        K.kvop_proxy_infer(px, feats[n_tr:], tau, cls, conf, ans)
        c, an = cls.cpu().numpy(), ans.cpu().numpy().astype(bool)
        dis = float(np.mean((c != labels_np[n_tr:]) & an))
        held[str(tau)] = {"coverage": float(an.mean()), "disagreement": dis}
        if tau_star is None and dis <= 0.01:
            tau_star = tau
    log(f"proxy held-out: {held}, best epoch {best_ep}, tau* = {tau_star}")
    del feats, labels
    torch.cuda.empty_cache()
    # fresh documents: labels and timed rates wave by wave (caches resident, not timed)
    ne = len(ev_docs.lengths)
    ev = {"full_ms": 0.0, "cascade_ms": {str(t): 0.0 for t in TAUS}}
    ev_cls = {str(t): np.empty(ne, np.int8) for t in TAUS}
    ev_ans = {str(t): np.empty(ne, bool) for t in TAUS}

    def per_wave(a, b, pool, h, idx, ioffs, op, feats_ev):
        m = b - a
        lg = torch.empty(m, 2, dtype=torch.float32, device=dev)
        dec = torch.empty(m, dtype=torch.int8, device=dev)
        ev["full_ms"] += _timed(lambda: K.kvop_op_eval(pool, op, 1.0, idx, ioffs, h, lg, dec), stream)
        c = torch.empty(m, dtype=torch.int8, device=dev)
        cf = torch.empty(m, dtype=torch.float32, device=dev)
        an = torch.empty(m, dtype=torch.int8, device=dev)
        f = feats_ev[a:b]
        for t in TAUS:
            def cascade():
                K.kvop_proxy_infer(px, f, t, c, cf, an)
                sel = np.nonzero(an.cpu().numpy() == 0)[0].astype(np.int32)   # the host routes the unsure tuples
                if len(sel):
                    K.kvop_op_eval_select(pool, op, 1.0, idx, ioffs, h, sel, lg, dec)
            ev["cascade_ms"][str(t)] += _timed(cascade, stream)
            ev_cls[str(t)][a:b] = c.cpu().numpy()
            ev_ans[str(t)][a:b] = an.cpu().numpy().astype(bool)

    t2 = time.time()
    feats_ev, lo_ev = _proxy_waves(K, synth, mb, ev_docs, suffix, dev, per_wave=per_wave)
    del feats_ev
    full_ev = (lo_ev > 0).astype(np.int8)
    fresh = {"documents": ne, "label_accept_frac": float(full_ev.mean()),
             "full_operator_tuples_per_s": ne / (ev["full_ms"] / 1e3), "per_tau": {}}
    for t in TAUS:
        k = str(t)
        an, c = ev_ans[k], ev_cls[k]
        wrong = (c != full_ev) & an
        fresh["per_tau"][k] = {
            "coverage": float(an.mean()), "disagreement_vs_full_operator": float(wrong.mean()),
            "disagreement_among_answered": float(wrong.sum() / max(1, an.sum())),
            "cascade_tuples_per_s": ne / (ev["cascade_ms"][k] / 1e3),
            "gain_over_full_operator": ev["full_ms"] / ev["cascade_ms"][k]}
    log(f"proxy on {ne} fresh documents ({time.time() - t2:.1f} s): {fresh}")
    info = {"train_docs": n_tr, "heldout_docs": nh, "label_accept_frac": pos_frac, "train_s": t_train,
            "epochs": args.proxy_epochs, "best_epoch": best_ep, "heldout_loss": best_loss, "loss_history": history,
            "data_s": t_data, "heldout": held, "tau": tau_star, "fresh": fresh}
    if tau_star is None:
        log("no tau meets 1% held-out disagreement: the proxy is not used")
        K.kvop_proxy_destroy(px)
        px = None
    return px, info


def _timed(fn, stream):
    """ms of fn() on the stream (HIP events), or the host's clock if that is longer (fn may
    synchronise on the host)."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return max(e0.elapsed_time(e1), (time.time() - t0) * 1e3)


def time_cascade(K, px, info, pool, handles, pooled, lists, op, full_out, n, args, dev, stream):
    """Timed step: proxy inference on the documents' pooled features, then the full operator
    on the tuples the proxy leaves unsure (a two-stage cascade)."""
    import torch
    idx, offs = lists
    tau = info["tau"]
    cls = torch.empty(n, dtype=torch.int8, device=dev)
    conf = torch.empty(n, dtype=torch.float32, device=dev)
    ans = torch.empty(n, dtype=torch.int8, device=dev)
    lg = torch.empty(n, 2, dtype=torch.float32, device=dev)
    dec = torch.empty(n, dtype=torch.int8, device=dev)
    final = None

    def step():
        K.kvop_proxy_infer(px, pooled, tau, cls, conf, ans)
        a = ans.cpu().numpy().astype(bool)            # synchronises: the host routes the unsure tuples
        sel = np.nonzero(~a)[0].astype(np.int32)
        if len(sel):
            K.kvop_op_eval_select(pool, op, 1.0, idx, offs, handles, sel, lg, dec)
        return a, sel

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.time()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        a, sel = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1), (time.time() - t0) * 1e3) / args.steps
    full_dec = full_out[1]
    c = cls.cpu().numpy()
    d = dec.cpu().numpy()
    final = np.where(a, c, d)
    per_tau = {}
    for t in (0.9, 0.95, 0.99):
        K.kvop_proxy_infer(px, pooled, t, cls, conf, ans)
        cc, an = cls.cpu().numpy(), ans.cpu().numpy().astype(bool)
        per_tau[str(t)] = {"coverage": float(an.mean()),
                           "disagreement_vs_full_operator": float(np.mean((cc != full_dec) & an))}
    out = {"tau": tau, "tuples_per_s": n / (ms / 1e3), "ms": ms, "coverage": float(a.mean()),
           "sent_to_full_operator": int(len(sel)),
           "disagreement_vs_full_operator": float(np.mean(final != full_dec)),
           "per_tau_on_workload": per_tau, "training": info, "_final": final}
    log(f"cascade: {out['tuples_per_s']:.0f} tuples/s, coverage {out['coverage']:.3f}, "
        f"disagreement {out['disagreement_vs_full_operator']:.4f}")
    return out


def counted_traffic(tile):
    """HBM bytes per gate/up launch from the committed rocprofv3 counter summary, or None when
    the GEMM source or the tile differs from the one the counters were taken on."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "gemm_gate_up_bf16_filter4096_hbm.md")
    src = os.path.join(here, "paper_2602_04430_amd", "csrc", "gemm.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line
                      and line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "gemm_hip_sha256", "tile"))
        same_src = hashlib.sha256(open(src, "rb").read()).hexdigest() == fields["gemm_hip_sha256"].strip()
        same_tile = tile is None or tile == fields.get("tile", tile).strip()
        return float(fields["traffic_bytes_per_launch"]) if same_src and same_tile else None
    except (OSError, KeyError, ValueError):
        return None


def load_scale_bounds():
    """The error bounds of the full-size parity test (tests/golden/scale_bounds.txt, derived
    there from the oracle alone), or {} when absent."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "scale_bounds.txt")
    out = {}
    try:
        for ln in open(path):
            f = ln.split()
            if len(f) == 2 and ln[0].isalpha():
                out[f[0]] = float(f[1])
    except (OSError, ValueError):
        return {}
    return out


def trace_launch_us():
    """Average gate/up launch duration from the committed rocprofv3 kernel trace, or None when
    the GEMM source differs from the one the trace was taken on."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "filter4096_bf16_kernel_trace.md")
    src = os.path.join(here, "paper_2602_04430_amd", "csrc", "gemm.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line
                      and line.split(": ", 1)[0] in ("gate_up_trace_avg_us", "gemm_hip_sha256"))
        same_src = hashlib.sha256(open(src, "rb").read()).hexdigest() == fields["gemm_hip_sha256"].strip()
        return float(fields["gate_up_trace_avg_us"]) if same_src else None
    except (OSError, KeyError, ValueError):
        return None


def copy_probe(dev):
    """Three plain device-to-device copies of 1 GiB: each reads and writes exactly 2^30 bytes,
    which calibrates the HBM byte counters (FETCH_SIZE, WRITE_SIZE) against known traffic."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy probe: 3 x 1 GiB device copies done")


def oracle_baseline(shape, w, docs, suffix, n_sample, gpu_bf16_logits, gpu_f32_logits, min_seconds=10.0):
    """Time the FP64 oracle's filter evaluation (the suffix over cached rows) on the first
    n_sample documents, after building their caches with the oracle (not timed)."""
    from oracle import model as om
    from paper_2602_04430_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    t0 = time.time()
    m = om.Model(shape, w)
    caches = []
    for i in range(n_sample):
        caches.append(om.kv_build(m, docs.doc(i)))
        log(f"oracle kv_build doc {i} (L={docs.lengths[i]}) done at {time.time() - t0:.1f} s")
    t_build = time.time() - t0
    # evaluate the sampled tuples in passes until at least min_seconds of CPU work is timed
    t1 = time.time()
    evals = 0
    while True:
        res = []
        for i in range(n_sample):
            res.append(om.filter_eval(m, caches[i], np.arange(docs.lengths[i]), suffix, synth.YES_ID, synth.NO_ID))
        evals += n_sample
        if time.time() - t1 >= min_seconds:
            break
    t_eval = time.time() - t1
    ref = np.stack([r.logits for r in res])
    # the same evaluation on one thread (BLAS limited to 1), a bounded number of evaluations
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t2 = time.time()
            e1 = 0
            while e1 < n_sample and time.time() - t2 < min_seconds:
                om.filter_eval(m, caches[e1], np.arange(docs.lengths[e1]), suffix, synth.YES_ID, synth.NO_ID)
                e1 += 1
            one = {"value": e1 / (time.time() - t2), "evaluations": e1, "seconds": time.time() - t2}
    except ImportError:
        pass
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    out = {"value": evals / t_eval, "unit": "tuples/s", "cores": int(threads), "kind": "oracle",
           "blas_threads": int(threads), "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model,
           "one_thread": one,
           "sample": f"FP64 NumPy oracle filter evaluation (r=1) of the first {n_sample} of the 4096 documents "
                     f"(L={[int(x) for x in docs.lengths[:n_sample]]}), {evals // n_sample} passes, {evals} "
                     f"evaluations; caches built by the oracle beforehand ({t_build:.1f} s, not in the rate)",
           "seconds": t_eval,
           "bf16_max_abs_logit_err_vs_oracle": float(np.max(np.abs(gpu_bf16_logits[:n_sample] - ref)))}
    if gpu_f32_logits is not None:
        out["fp32_max_abs_logit_err_vs_oracle"] = float(np.max(np.abs(gpu_f32_logits[:n_sample] - ref)))
    log(f"oracle: {out['value']:.3f} tuples/s on {threads} threads")
    return out


if __name__ == "__main__":
    main()
