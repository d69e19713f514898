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

FP8-E4M3 cache (BF16 compute).  The same derivation with the cache format held fixed: the
emulation of the BF16 form whose cache holds the FP8 format (bf16fp8: the BF16-rounded
projections' keys and values, rotated and quantised to FP8 blocks, as the GPU quantises
them), the FP8-format oracle with BF16 weights (fp8w) and the FP8-format oracle (fp8fmt):

  N8  = |bf16fp8 - fp8w|      the activation rounding, and the FP8 codes it moves
  E_fp8_form   = 2 max N8                      GPU vs the emulation bf16fp8
  E_fp8_format = max |bf16fp8 - fp8fmt| + E_fp8_form    GPU vs the FP8-format oracle
  E_fp8        = max |bf16fp8 - fp64|   + E_fp8_form    GPU vs the oracle

(The GPU computes keys and values in BF16 and then picks FP8 codes; values near a code's
rounding midpoint go to either neighbour, which the emulation realises one way.)

Writes scale_bounds.txt beside this script:  python -m tests.golden.scale_bounds
"""
import os
import sys
from collections import defaultdict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
FP8_VARIANT_FILES = [os.path.join(HERE, f"scale_filter_oracle_{v}.txt") for v in ("fp8w", "bf16fp8")]


def load_filter_oracle(path=os.path.join(HERE, "scale_filter_oracle.txt"), extra=FP8_VARIANT_FILES):
    """{(document, r, variant): np.array([logit_yes, logit_no])} and {document: L}, from the
    four-variant file and the FP8-form variant files."""
    out, lengths = {}, {}
    for p in [path] + list(extra):
        with open(p) as fh:
            for line in fh:
                if not line.strip() or line.startswith("#"):
                    continue
                d, L, r, var, a, b = line.split()
                out[(int(d), float(r), var)] = np.array([float(a), float(b)])
                lengths[int(d)] = int(L)
    return out, lengths


def derive(ref):
    """Per (document, r): F_w, N, F, the FP8 format's own effect, N8, and the FP8 form's
    distance to the FP8-format oracle and to the oracle; and the bounds."""
    keys = sorted({(d, r) for d, r, _ in ref})
    rows = []
    for d, r in keys:
        o, w, e, f8, f8w, e8 = (ref[(d, r, v)] for v in ("fp64", "bf16w", "bf16form", "fp8fmt", "fp8w", "bf16fp8"))

        def dist(a, b):
            return float(np.abs(a - b).max())
        rows.append((d, r, dist(w, o), dist(e, w), dist(e, o), dist(f8, o), dist(e8, f8w), dist(e8, f8),
                     dist(e8, o)))
    mx = [max(x[k] for x in rows) for k in range(2, 9)]
    max_n, max_f, max_f8, max_n8, max_e8f, max_e8o = mx[1], mx[2], mx[3], mx[4], mx[5], mx[6]
    b = {"max_N": max_n, "max_F": max_f, "E_bf16_form": 2 * max_n, "E_bf16": max_f + 2 * max_n,
         "max_fp8_format_effect": max_f8, "max_N8": max_n8, "max_fp8_form_vs_format": max_e8f,
         "max_fp8_form_vs_oracle": max_e8o, "E_fp8_form": 2 * max_n8, "E_fp8_format": max_e8f + 2 * max_n8,
         "E_fp8": max_e8o + 2 * max_n8}
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
        fh.write("# written by tests/golden/scale_bounds.py from the stored filter oracle values (oracle only); "
                 "columns: document L r F_w N F fp8_format_effect N8 fp8_form_vs_format fp8_form_vs_oracle\n")
        for x in rows:
            fh.write(f"{x[0]} {lengths[x[0]]} {x[1]} " + " ".join(f"{v:.5f}" for v in x[2:]) + "\n")
        for k, v in b.items():
            fh.write(f"{k} {v:.5f}\n")
    for r, xs in sorted(by_r.items()):
        print(f"r {r}: max N {max(x[3] for x in xs):.4f}, max F {max(x[4] for x in xs):.4f}, "
              f"FP8 format {max(x[5] for x in xs):.4f}, N8 {max(x[6] for x in xs):.4f}")
    print(b)
    return 0


if __name__ == "__main__":
    sys.exit(main())
