"""Derives the error bounds of the full-size filter parity test from the stored oracle values
alone (scale_filter_oracle.txt, written by make_scale_golden.py); no GPU result enters.

BF16 form.  It rounds its weights, every projection's input and output, the rotated queries,
the cached keys and values, the unnormalised attention probabilities and the attention output
to BF16 (round to nearest even); accumulation, the residual stream and the normalisation
statistics stay FP32.  Over the sampled documents and every r:

  F_w = |oracle(BF16 weights) - oracle|                the weights' format effect
  N   = |emulation of the BF16 form - oracle(BF16 weights)|   the activation/cache rounding
  F   = |emulation - oracle|                           the whole format effect

The GPU rounds at the same points, but its FP32 arithmetic sends values near a rounding
midpoint to either side and it rounds the probabilities relative to a running maximum, so
its activation rounding is another realisation of N: against the emulation
E_bf16_form = 2 max N, against the oracle E_bf16 = max F + E_bf16_form.

FP8-E4M3 cache (BF16 compute).  Against the oracle of the same cache format the stated
bound is E_fp8_format = 0.15: the GPU rounds its codes from BF16-computed keys/values, so
near a rounding midpoint it picks the neighbouring code (up to 0.06 of logit in an FP64
emulation with BF16 weights, doubled), plus the BF16 arithmetic error (0.03).  Against
the oracle E_fp8 = max |oracle of the format - oracle| + E_fp8_format.

Writes scale_bounds.txt beside this script:  python -m tests.golden.scale_bounds
"""
import os
import sys
from collections import defaultdict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
E_FP8_FORMAT = 0.15


def load_filter_oracle(path=os.path.join(HERE, "scale_filter_oracle.txt")):
    """{(document, r, variant): np.array([logit_yes, logit_no])} and {document: L}."""
    out, lengths = {}, {}
    with open(path) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            d, L, r, var, a, b = line.split()
            out[(int(d), float(r), var)] = np.array([float(a), float(b)])
            lengths[int(d)] = int(L)
    return out, lengths


def derive(ref):
    keys = sorted({(d, r) for d, r, _ in ref})
    rows = []
    for d, r in keys:
        o, w, e, f8 = (ref[(d, r, v)] for v in ("fp64", "bf16w", "bf16form", "fp8fmt"))
        rows.append((d, r, float(np.abs(w - o).max()), float(np.abs(e - w).max()), float(np.abs(e - o).max()),
                     float(np.abs(f8 - o).max())))
    max_n = max(x[3] for x in rows)
    max_f = max(x[4] for x in rows)
    max_f8 = max(x[5] for x in rows)
    b = {"max_N": max_n, "max_F": max_f, "E_bf16_form": 2 * max_n, "E_bf16": max_f + 2 * max_n,
         "max_fp8_format_effect": max_f8, "E_fp8_format": E_FP8_FORMAT, "E_fp8": max_f8 + E_FP8_FORMAT}
    return rows, b


def load_bounds(path=os.path.join(HERE, "scale_bounds.txt")):
    b = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#") and not line[0].isdigit():
                k, v = line.split()
                b[k] = float(v)
    return b


def main():
    ref, lengths = load_filter_oracle()
    rows, b = derive(ref)
    by_r = defaultdict(list)
    for x in rows:
        by_r[x[1]].append(x)
    with open(os.path.join(HERE, "scale_bounds.txt"), "w") as fh:
        fh.write("# written by tests/golden/scale_bounds.py from scale_filter_oracle.txt (oracle only); "
                 "columns: document L r F_w N F fp8_format_effect\n")
        for d, r, fw, n, f, f8 in rows:
            fh.write(f"{d} {lengths[d]} {r} {fw:.5f} {n:.5f} {f:.5f} {f8:.5f}\n")
        for k, v in b.items():
            fh.write(f"{k} {v:.5f}\n")
    for r, xs in sorted(by_r.items()):
        print(f"r {r}: max N {max(x[3] for x in xs):.4f}, max F {max(x[4] for x in xs):.4f}, "
              f"FP8 format {max(x[5] for x in xs):.4f}")
    print(b)
    return 0


if __name__ == "__main__":
    sys.exit(main())
