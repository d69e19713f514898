"""Writes the stored expected values under tests/golden/ from the FP64 oracle only.

tiny_filter_fp64.txt: the small plain-filter workload (2-layer d_model-128 decoder with
normal(0, 0.02) weights, 64 documents of uniform length in [32, 128], one shared 16-token
suffix, retention 1, yes id 1 / no id 0, seed 0): per document its length, the yes and no
logits and their log-odds, printed with 17 significant digits.

Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import model as om  # noqa: E402
from paper_2602_04430_amd import synth  # noqa: E402


def tiny_filter_rows(seed=0):
    wl = synth.tiny_filter(seed)
    m = om.Model(wl.shape, synth.make_weights(wl.shape, seed))
    rows = []
    for i in range(len(wl.docs.lengths)):
        doc = wl.docs.doc(i)
        c = om.kv_build(m, doc)
        r = om.filter_eval(m, c, np.arange(len(doc)), wl.suffix, synth.YES_ID, synth.NO_ID)
        rows.append((len(doc), r.logits[0], r.logits[1], r.log_odds))
    return rows


def main():
    path = os.path.join(HERE, "tiny_filter_fp64.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle, small plain filter workload, seed 0: length logit_yes logit_no log_odds\n")
        for L, a, b, lo in tiny_filter_rows():
            f.write(f"{L} {a:.17g} {b:.17g} {lo:.17g}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
