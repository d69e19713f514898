"""The optimizer's plan, run by the cascade executor.  Log-odds profiled on the GPU at
r = 0.1, 0.25, 0.5, 1 feed kvop_plan_optimize (gold: the r = 1 decisions); the chosen stages
then run through kvop_cascade_eval over the same documents.  The planner's discrete
evaluation (kvop_plan_evaluate) and the executor must agree exactly: the same accepted
tuples, the same per-stage processed counts — both decide by comparing the FP32 log-odds with
the FP32 thresholds.  A forced plan (every stage selected, fixed thresholds) is checked the
same way, so that the check does not depend on which plan the optimizer picks."""
import numpy as np
import pytest
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth
from tests.gpu_common import Engine, say

pytestmark = pytest.mark.gpu

SHAPE = synth.ModelShape(n_layers=2, d_model=256, n_heads=4, n_kv_heads=2, head_dim=64, d_ffn=512, vocab=512)
RS = (0.1, 0.25, 0.5, 1.0)


def _run_plan(eng, h, suffix, lists, sel, tp, tn):
    stages = [(r, float(tp[i]), float(tn[i]), torch.from_numpy(lists[r][0]).cuda(), lists[r][1])
              for i, r in enumerate(RS) if sel[i]]
    n = len(h)
    op = K.make_op(K.KVOP_FILTER, suffix, synth.YES_ID, synth.NO_ID)
    lg = torch.empty(n, 2, device="cuda")
    dec = torch.empty(n, dtype=torch.int8, device="cuda")
    stg = torch.empty(n, dtype=torch.int8, device="cuda")
    proc = K.kvop_cascade_eval(eng.pool, op, stages, h, lg, dec, stg)
    torch.cuda.synchronize()
    return dec.cpu().numpy(), proc


@pytest.mark.parametrize("compute,kv", [("f32", "f32"), ("bf16", "bf16")])
def test_plan_runs_as_evaluated(device, compute, kv):
    w = synth.make_weights(SHAPE, 61, gain_jitter=0.1)
    docs = synth.make_docs_lognormal(600, 80, 4, 600, SHAPE.vocab, seed=61)
    suffix = synth.suffix_tokens(10, SHAPE.vocab, seed=61)
    eng = Engine(SHAPE, w, compute, kv)
    h = eng.build(docs)
    lists = {r: synth.retained_lists(docs.lengths, r, seed=61) for r in RS}
    say("plan vs executor", compute, kv)
    lo = []
    for r in RS:
        lg, _ = eng.filter(h, *lists[r], suffix, r=r)
        lg32 = lg.astype(np.float32)
        lo.append(lg32[:, 0] - lg32[:, 1])            # the kernel's FP32 log-odds
    lo = np.stack(lo)
    _, dec1 = eng.filter(h, *lists[1.0], suffix, r=1.0)
    gold = (dec1 == 1).astype(np.int8)
    pb = K.PlanProblem([lo], [np.array([1.0, 1.3, 1.8, 3.0])], [gold], 0.9, 0.9, 0.95)
    res = K.kvop_plan_optimize(pb, steps=200)
    forced = (np.ones(4, np.int8), np.array([1.5, 1.0, 0.5, 0.0], np.float32),
              np.array([-1.5, -1.0, -0.5, 0.0], np.float32))
    for name, (sel, tp, tn) in (("optimized", (res["selected"], res["theta_pos"], res["theta_neg"])),
                                ("forced", forced)):
        if not sel.any():
            continue
        ev = K.kvop_plan_evaluate(pb, sel, tp, tn)
        dec, proc = _run_plan(eng, h, suffix, lists, sel, tp, tn)
        np.testing.assert_array_equal(dec == 1, ev["accept"] == 1, err_msg=name)
        np.testing.assert_array_equal(proc, ev["processed"][sel.astype(bool)], err_msg=name)
        rep = ev["report"]
        say(f"{name}: stages {[r for r, s in zip(RS, sel) if s]}, processed {list(proc)}, "
            f"TP {rep['tp']:.0f} FP {rep['fp']:.0f} FN {rep['fn']:.0f}, bounds R {rep['recall_lb']:.3f} "
            f"P {rep['precision_lb']:.3f}, cost {rep['cost_frac']:.3f}")
    eng.close()
