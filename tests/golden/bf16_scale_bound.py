"""Derives the BF16 error bound of the full-size filter parity test from the oracle alone.

The BF16 form rounds its weights, every projection's input and output, the rotated queries,
the cached keys and values, the unnormalised attention probabilities and the attention
output to BF16 (round to nearest even); accumulation, the residual stream and the
normalisation statistics stay FP32.  The oracle emulates that form in float64 with its
activation-format and cache-format hooks.  On the sampled documents of the test, for every r:

  F_w  = |oracle(BF16 weights) - oracle|                 the weights' format effect
  N    = |emulation - oracle(BF16 weights)|              the activation/cache rounding effect
  F    = |emulation - oracle|                            the whole format effect

The GPU rounds at the same points, but its FP32 arithmetic puts values near a rounding
midpoint on either side and it rounds the probabilities relative to a running maximum, so
its activation rounding is another realisation of N: bound against the emulation
E_form = 2 max N, and against the oracle E = max F + E_form.  Writes the figures to
bf16_scale_bound.txt beside this script (run: python -m tests.golden.bf16_scale_bound).
"""
import os
import sys
import time

import numpy as np

from oracle import codecs
from oracle import model as om
from paper_2602_04430_amd import synth

SAMPLE = [0, 1, 7, 19, 81, 100, 2047, 4095]


def main():
    shape = synth.SCALE
    wl = synth.scale_filter(0)
    w = synth.make_weights(shape, 0)
    wb = {k: codecs.bf16_round(v) if v.ndim == 2 else v for k, v in w.items()}
    m = om.Model(shape, w)
    mw = om.Model(shape, wb)
    me = om.Model(shape, wb, act=codecs.bf16_round)
    docs = wl.docs
    lists = {r: synth.retained_lists(docs.lengths, r, seed=0) for r in wl.r_grid}
    rows = []
    for i in SAMPLE:
        t0 = time.time()
        c = om.kv_build(m, docs.doc(i))
        cw = om.kv_build(mw, docs.doc(i))
        ce = om.kv_build(me, docs.doc(i), store=codecs.bf16_round)
        for r in wl.r_grid:
            idx, offs = lists[r]
            R = idx[offs[i]:offs[i + 1]]
            lg = [om.filter_eval(mm, cc, R, wl.suffix, synth.YES_ID, synth.NO_ID).logits
                  for mm, cc in ((m, c), (mw, cw), (me, ce))]
            fw = float(np.abs(lg[1] - lg[0]).max())
            n = float(np.abs(lg[2] - lg[1]).max())
            f = float(np.abs(lg[2] - lg[0]).max())
            rows.append((i, int(docs.lengths[i]), r, fw, n, f))
            print(f"document {i} L {docs.lengths[i]} r {r}: F_w {fw:.4f} N {n:.4f} F {f:.4f}", flush=True)
        print(f"  {time.time() - t0:.0f} s", flush=True)
    max_n = max(x[4] for x in rows)
    max_f = max(x[5] for x in rows)
    e_form = 2 * max_n
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bf16_scale_bound.txt")
    with open(out, "w") as fh:
        fh.write("# written by tests/golden/bf16_scale_bound.py (oracle only); columns: document L r F_w N F\n")
        for x in rows:
            fh.write(f"{x[0]} {x[1]} {x[2]} {x[3]:.5f} {x[4]:.5f} {x[5]:.5f}\n")
        fh.write(f"max_N {max_n:.5f}\nmax_F {max_f:.5f}\nE_form {e_form:.5f}\nE {max_f + e_form:.5f}\n")
    print(f"max N {max_n:.4f}, max F {max_f:.4f}: E_form {e_form:.4f}, E {max_f + e_form:.4f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
