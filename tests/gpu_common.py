"""Shared helpers of the GPU tests: model/pool set-up through the C ABI and the stated
error bounds.

Error bounds (max-abs logit error against the FP64 oracle, stated before measuring):
  E_F32  = 1e-4   FP32 weights, activations and cache
  E_BF16 = 5e-2   BF16 weights/activations, BF16 cache
  E_FP8  = 1.5e-1 BF16 weights/activations, FP8-E4M3 cache with per-16-row scales
A decision is "outside the margin band" when |LO_oracle - theta| >= 2 E: there a correct
result within E on both logits cannot flip, so outside the band decisions must agree.
"""
import numpy as np
import torch

from paper_2602_04430_amd import kvop as K
from paper_2602_04430_amd import synth

E_F32 = 1e-4
E_BF16 = 5e-2
E_FP8 = 1.5e-1
BOUND = {("f32", "f32"): E_F32, ("bf16", "bf16"): E_BF16, ("bf16", "fp8"): E_FP8}
COMPUTE = {"f32": K.KVOP_F32, "bf16": K.KVOP_BF16}
KVDT = {"f32": K.KVOP_KV_F32, "bf16": K.KVOP_KV_BF16, "fp8": K.KVOP_KV_FP8}


def say(*a):
    print(*a, flush=True)


class Engine:
    """A model + pool pair created through the C ABI."""

    def __init__(self, shape, weights, compute="f32", kv="f32", pool_bytes=1 << 30):
        self.shape = shape
        flat = torch.from_numpy(synth.pack_weights(shape, weights)).cuda()
        self.model = K.kvop_model_create(K.make_cfg(shape), flat, COMPUTE[compute])
        del flat
        self.pool = K.kvop_pool_create(self.model, KVDT[kv], pool_bytes)
        self.compute, self.kv = compute, kv

    def build(self, docs: synth.Docs, pooled=False):
        toks = torch.from_numpy(docs.tokens).cuda()
        pl = torch.zeros(len(docs.lengths), self.shape.d_model, dtype=torch.float32, device="cuda") if pooled else None
        h = K.kvop_kv_build(self.pool, toks, docs.offsets, pl)
        torch.cuda.synchronize()
        return (h, pl) if pooled else h

    def filter(self, handles, idx, offs, suffix, r=1.0, theta=(0.0, 0.0), kind=K.KVOP_FILTER, flags=0):
        n = len(handles) // (2 if kind == K.KVOP_JOIN else 1)
        op = K.make_op(kind, suffix, synth.YES_ID, synth.NO_ID, theta[0], theta[1], flags=flags)
        lg = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
        dec = torch.full((n,), 7, dtype=torch.int8, device="cuda")
        K.kvop_op_eval(self.pool, op, r, torch.from_numpy(np.asarray(idx, np.int32)).cuda(), offs, handles, lg, dec)
        torch.cuda.synchronize()
        return lg.cpu().numpy().astype(np.float64), dec.cpu().numpy()

    def map(self, handles, idx, offs, suffix, lo, n, n_gen, r=1.0):
        op = K.make_op(K.KVOP_MAP, suffix, label_lo=lo, label_n=n, n_gen=n_gen)
        m = len(handles)
        lg = torch.full((m, n_gen, n), float("nan"), dtype=torch.float32, device="cuda")
        tk = torch.full((m, n_gen), -1, dtype=torch.int32, device="cuda")
        K.kvop_op_eval(self.pool, op, r, torch.from_numpy(np.asarray(idx, np.int32)).cuda(), offs, handles, lg, None,
                       tk)
        torch.cuda.synchronize()
        return lg.cpu().numpy().astype(np.float64), tk.cpu().numpy()

    def close(self):
        torch.cuda.synchronize()
        K.kvop_pool_destroy(self.pool)
        K.kvop_model_destroy(self.model)


def decisions_agree_outside_band(lo_ref, dec_gpu, E, theta=0.0):
    """Return (number of disagreements outside the band, in-band fraction)."""
    lo_ref = np.asarray(lo_ref)
    ref = np.where(lo_ref > theta, 1, np.where(lo_ref < theta, 0, -1))
    out = np.abs(lo_ref - theta) >= 2 * E
    return int(np.sum((ref != dec_gpu) & out)), float(1 - out.mean())


def check_map(tokens_gpu, logits_gpu, refs, E):
    """Map items against the oracle's greedy decodes (refs: oracle MapResult per item).

    An id is decision-pinned while every oracle step so far, this one included, has a top-1 to
    top-2 margin of at least 2 E over the label slice: there a result within E of the oracle's
    logits cannot pick another id, so the GPU's ids must equal the oracle's up to the item's
    first in-band step.  The slice logits must be within E at every step whose earlier ids
    agree (after a divergence inside the band the two decode different texts).
    Returns (ids checked, items with all ids checked, max-abs logit error, failures)."""
    checked, whole, err, fails = 0, 0, 0.0, []
    for i, res in enumerate(refs):
        srt = np.sort(res.step_logits, axis=1)
        pinned = np.cumprod(srt[:, -1] - srt[:, -2] >= 2 * E).astype(bool)
        for t in range(len(res.tokens)):
            if not np.array_equal(tokens_gpu[i, :t], res.tokens[:t]):
                break
            e = float(np.max(np.abs(logits_gpu[i, t] - res.step_logits[t])))
            err = max(err, e)
            if e > E:
                fails.append(("logits", i, t, e))
        n = int(pinned.sum())
        checked += n
        whole += int(n == len(res.tokens))
        if not np.array_equal(tokens_gpu[i, :n], res.tokens[:n]):
            fails.append(("ids", i, tokens_gpu[i].tolist(), res.tokens.tolist(), n))
    return checked, whole, err, fails
