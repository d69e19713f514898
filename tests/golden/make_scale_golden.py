"""Writes the stored expected values of the full-size parity tests from the FP64 oracle only.

The decoder is the 16-layer d_model-2048 model (16 query / 8 kv heads of 128, SwiGLU 5632,
vocab 32000, normal(0, 0.02) weights, seed 0).  Nothing here calls the GPU library.

  python -m tests.golden.make_scale_golden filter   # scale_filter_oracle.txt, scale_ea_scores.txt
  python -m tests.golden.make_scale_golden fp8w     # scale_filter_oracle_fp8w.txt
  python -m tests.golden.make_scale_golden bf16fp8  # scale_filter_oracle_bf16fp8.txt
    (fp8w- / bf16fp8-: the same in reverse document order, to share the work with a second run)
  python -m tests.golden.make_scale_golden mixed    # mixed_sample_oracle.txt

filter: 64 documents of the 4096-document filter workload (lognormal lengths, median 512, in
  [64, 4096]; one shared 32-token suffix), chosen at evenly spaced ranks of the length order
  so that they span the distribution (the shortest and a longest document included).  For
  every r in {1, 0.5, 0.25, 0.1} and the workload's seeded retained lists, the yes/no logits
  of four oracles:
    fp64      the oracle proper (FP32 master weights in float64)
    bf16w     the oracle with the weights rounded to BF16
    bf16form  the float64 emulation of the BF16 form (BF16 weights; every projection's input
              and output, the rotated queries, the cached keys/values, the unnormalised
              probabilities and the attention output rounded to BF16)
    fp8fmt    the oracle whose cache holds the FP8-E4M3 format (16-row blocks with FP32 scales)
  and the expected-attention row scores of three short documents under the BF16 form.  Two
  more oracles of the same documents (files of their own, written by separate runs) serve the
  FP8 cache's bound:
    fp8w      the FP8-format oracle with the weights rounded to BF16
    bf16fp8   the float64 emulation of the BF16 form whose cache holds the FP8 format (the
              BF16-rounded projections' keys and values, rotated, quantised to FP8 blocks)
mixed: items of the mixed-operator workload (16384 documents, lognormal median 384 in
  [16, 8192]; filter / map / join thirds; 2048 pairs) that every grouping of the benchmark
  with at most four groups places in its first group: 8 filter documents, 8 map documents and
  4 join pairs spread over their lengths, at r = 1.  Filter and join: yes/no logits.  Map: the
  8 greedy ids over the label slice [256, 512) and the slice logits of every step.

Lines are appended as they are computed (to a .partial file), so an interrupted run resumes.
"""
import os
import sys
import time

import numpy as np

from oracle import codecs
from oracle import compress as oc
from oracle import model as om
from paper_2602_04430_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
FILTER_FILE = os.path.join(HERE, "scale_filter_oracle.txt")
EA_FILE = os.path.join(HERE, "scale_ea_scores.txt")
MIXED_FILE = os.path.join(HERE, "mixed_sample_oracle.txt")
N_FILTER_SAMPLE = 64
EA_SAMPLE = [81, 100, 7]          # L = 64, 149, 123
MIXED_FIRST_GROUP = 4             # items every grouping into <= 4 groups puts in group 0
VARIANTS = ("fp64", "bf16w", "bf16form", "fp8fmt")
FP8_VARIANTS = ("fp8w", "bf16fp8")


def variant_file(var):
    return os.path.join(HERE, f"scale_filter_oracle_{var}.txt")


def filter_sample(lengths, n=N_FILTER_SAMPLE):
    """Documents at evenly spaced ranks of the (length, index) order, ascending by index."""
    L = np.asarray(lengths)
    order = np.lexsort((np.arange(len(L)), L))
    return sorted(int(x) for x in order[np.rint(np.linspace(0, len(L) - 1, n)).astype(int)])


def _spread(items, length, n):
    """n items at evenly spaced ranks of their length order (ties by position)."""
    ln = np.array([length(x) for x in items])
    order = np.lexsort((np.arange(len(ln)), ln))
    return [items[int(i)] for i in order[np.rint(np.linspace(0, len(ln) - 1, n)).astype(int)]]


def mixed_sample(wl):
    """(filter docs, map docs, join pairs) of the stored mixed sample."""
    L = wl.docs.lengths
    f = wl.extra["filter_docs"][: len(wl.extra["filter_docs"]) // MIXED_FIRST_GROUP]
    m = wl.extra["map_docs"][: len(wl.extra["map_docs"]) // MIXED_FIRST_GROUP]
    p = wl.extra["join_pairs"][: len(wl.extra["join_pairs"]) // MIXED_FIRST_GROUP]
    fs = _spread([int(x) for x in f], lambda d: L[d], 8)
    ms = _spread([int(x) for x in m], lambda d: L[d], 8)
    ps = _spread([tuple(int(v) for v in x) for x in p], lambda ab: L[ab[0]] + L[ab[1]], 4)
    return fs, ms, ps


def _done_keys(path, nkey):
    keys = set()
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                if line.strip() and not line.startswith("#"):
                    keys.add(tuple(line.split()[:nkey]))
    return keys


def make_filter():
    shape = synth.SCALE
    wl = synth.scale_filter(0)
    docs = wl.docs
    w = synth.make_weights(shape, 0)
    wb = {k: (codecs.bf16_round(v) if v.ndim == 2 else v).astype(np.float64) for k, v in w.items()}
    models = {"fp64": (om.Model(shape, w), None),
              "bf16w": (om.Model(shape, wb), None),
              "bf16form": (om.Model(shape, wb, act=codecs.bf16_round), codecs.bf16_round)}
    models["fp8fmt"] = (models["fp64"][0], codecs.fp8_cache_roundtrip)
    lists = {r: synth.retained_lists(docs.lengths, r, seed=0) for r in wl.r_grid}
    part = FILTER_FILE + ".partial"
    done = _done_keys(part, 4)
    with open(part, "a") as fh:
        if not done:
            fh.write("# written by tests/golden/make_scale_golden.py (FP64 oracle only); "
                     "columns: document L r variant logit_yes logit_no\n")
        for i in filter_sample(docs.lengths):
            L = int(docs.lengths[i])
            for var in VARIANTS:
                if all((str(i), str(L), str(r), var) in done for r in wl.r_grid):
                    continue
                t0 = time.time()
                m, store = models[var]
                c = om.kv_build(m, docs.doc(i), store=store)
                for r in wl.r_grid:
                    idx, offs = lists[r]
                    res = om.filter_eval(m, c, idx[offs[i]:offs[i + 1]], wl.suffix, synth.YES_ID, synth.NO_ID)
                    fh.write(f"{i} {L} {r} {var} {res.logits[0]:.17g} {res.logits[1]:.17g}\n")
                fh.flush()
                print(f"filter document {i} L {L} {var}: {time.time() - t0:.1f} s", flush=True)
    os.replace(part, FILTER_FILE)
    me = models["bf16form"][0]
    with open(EA_FILE, "w") as fh:
        fh.write("# written by tests/golden/make_scale_golden.py (FP64 oracle only): expected-attention row "
                 "scores under the BF16 form, future queries at L .. L+31; columns: document row score\n")
        for i in EA_SAMPLE:
            sc = oc.ea_scores(me, docs.doc(i), len(wl.suffix))
            for row, v in enumerate(sc):
                fh.write(f"{i} {row} {v:.17g}\n")
    print("wrote", FILTER_FILE, EA_FILE, flush=True)


def make_filter_variant(var, reverse=False):
    """One extra oracle of the 64 sampled filter documents (fp8w or bf16fp8).  Two runs may
    share the work, one forward and one in reverse order (`<var>-`): each skips documents
    already present in either's partial file, and the run that finds every document done
    writes the merged file."""
    shape = synth.SCALE
    wl = synth.scale_filter(0)
    docs = wl.docs
    w = synth.make_weights(shape, 0)
    wb = {k: (codecs.bf16_round(v) if v.ndim == 2 else v).astype(np.float64) for k, v in w.items()}
    del w
    m = om.Model(shape, wb, act=codecs.bf16_round if var == "bf16fp8" else None)
    lists = {r: synth.retained_lists(docs.lengths, r, seed=0) for r in wl.r_grid}
    path = variant_file(var)
    parts = [path + ".partial", path + ".rev.partial"]
    mine = parts[1] if reverse else parts[0]

    def done_all():
        keys = set()
        for p in parts:
            keys |= _done_keys(p, 4)
        return keys
    sample = filter_sample(docs.lengths)
    with open(mine, "a") as fh:
        for i in (reversed(sample) if reverse else sample):
            L = int(docs.lengths[i])
            if all((str(i), str(L), str(r), var) in done_all() for r in wl.r_grid):
                continue
            t0 = time.time()
            c = om.kv_build(m, docs.doc(i), store=codecs.fp8_cache_roundtrip)
            for r in wl.r_grid:
                idx, offs = lists[r]
                res = om.filter_eval(m, c, idx[offs[i]:offs[i + 1]], wl.suffix, synth.YES_ID, synth.NO_ID)
                fh.write(f"{i} {L} {r} {var} {res.logits[0]:.17g} {res.logits[1]:.17g}\n")
            fh.flush()
            print(f"filter document {i} L {L} {var}: {time.time() - t0:.1f} s", flush=True)
    keys = done_all()
    if all((str(i), str(int(docs.lengths[i])), str(r), var) in keys for i in sample for r in wl.r_grid):
        lines = {}
        for p in parts:
            if os.path.exists(p):
                for line in open(p):
                    if line.strip() and not line.startswith("#"):
                        lines[tuple(line.split()[:4])] = line
        with open(path, "w") as out:
            out.write("# written by tests/golden/make_scale_golden.py (FP64 oracle only); "
                      "columns: document L r variant logit_yes logit_no\n")
            for key in sorted(lines, key=lambda k: (int(k[0]), -float(k[2]))):
                out.write(lines[key])
        for p in parts:
            if os.path.exists(p):
                os.remove(p)
        print("wrote", path, flush=True)


def make_mixed():
    shape = synth.SCALE
    wl = synth.mixed_batch(0)
    docs = wl.docs
    m = om.Model(shape, synth.make_weights(shape, 0))
    fs, ms, ps = mixed_sample(wl)
    lo, nl = synth.MAP_SLICE
    part = MIXED_FILE + ".partial"
    done = _done_keys(part, 2)
    caches = {}

    def cache(d):
        if d not in caches:
            caches[d] = om.kv_build(m, docs.doc(d))
        return caches[d]

    with open(part, "a") as fh:
        if not done:
            fh.write("# written by tests/golden/make_scale_golden.py (FP64 oracle only), mixed workload, r = 1.\n"
                     "# filter <doc> <L> <logit_yes> <logit_no> | join <docA>,<docB> <LA>,<LB> <logit_yes> "
                     "<logit_no> | map <doc> <L> <8 ids> then 8 lines 'step <doc> <t> <256 slice logits>'\n")
        for d in fs:
            if ("filter", str(d)) in done:
                continue
            t0 = time.time()
            res = om.filter_eval(m, cache(d), np.arange(docs.lengths[d]), wl.suffix, synth.YES_ID, synth.NO_ID)
            fh.write(f"filter {d} {docs.lengths[d]} {res.logits[0]:.17g} {res.logits[1]:.17g}\n")
            fh.flush()
            caches.clear()
            print(f"filter {d} L {docs.lengths[d]}: {time.time() - t0:.1f} s", flush=True)
        for d in ms:
            if ("map", str(d)) in done:
                continue
            t0 = time.time()
            res = om.map_eval(m, cache(d), np.arange(docs.lengths[d]), wl.extra["suffix_map"], lo, nl,
                              synth.MAP_TOKENS)
            fh.write(f"map {d} {docs.lengths[d]} " + " ".join(str(int(t)) for t in res.tokens) + "\n")
            for t in range(synth.MAP_TOKENS):
                fh.write(f"step {d} {t} " + " ".join(f"{v:.10g}" for v in res.step_logits[t]) + "\n")
            fh.flush()
            caches.clear()
            print(f"map {d} L {docs.lengths[d]}: {time.time() - t0:.1f} s", flush=True)
        for a, b in ps:
            if ("join", f"{a},{b}") in done:
                continue
            t0 = time.time()
            res = om.join_eval(m, cache(a), np.arange(docs.lengths[a]), cache(b), np.arange(docs.lengths[b]),
                               wl.extra["suffix_join"], synth.YES_ID, synth.NO_ID)
            fh.write(f"join {a},{b} {docs.lengths[a]},{docs.lengths[b]} {res.logits[0]:.17g} {res.logits[1]:.17g}\n")
            fh.flush()
            caches.clear()
            print(f"join {a},{b} L {docs.lengths[a]}+{docs.lengths[b]}: {time.time() - t0:.1f} s", flush=True)
    os.replace(part, MIXED_FILE)
    print("wrote", MIXED_FILE, flush=True)


def main():
    what = sys.argv[1:] or ["filter", "fp8w", "bf16fp8", "mixed"]
    for w in what:
        if w.rstrip("-") in FP8_VARIANTS:
            make_filter_variant(w.rstrip("-"), reverse=w.endswith("-"))
        else:
            {"filter": make_filter, "mixed": make_mixed}[w]()
    return 0


if __name__ == "__main__":
    sys.exit(main())
