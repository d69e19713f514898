"""FP64 oracle of a filter cascade over retention profiles.

TEST INFRASTRUCTURE ONLY.  Imported by the tests and nothing else; the GPU library never
imports, calls or links it.

A semantic filter runs as a pipeline of physical operators o_1 -> ... -> o_n of increasing
cost (Section 4.1): here the same filter over cache profiles of increasing retention r.
Every tuple starts unsure; operator o_i sees a tuple only if all earlier operators left it
unsure, and accepts, rejects or again leaves it unsure by its own thresholds (Eqs. 1-3:
accept_i = accept_(i-1) + unsure_(i-1) * accept(o_i); reject likewise; unsure_i =
1 - accept_i - reject_i).  The cost of a tuple is the number of operators that processed it
(Eq. 4, with unit per-operator costs counted per stage here).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import model as om


@dataclass
class Stage:
    retained: List[np.ndarray]   # per item: the rows of its document this profile keeps
    theta_pos: float
    theta_neg: float


@dataclass
class CascadeResult:
    decision: np.ndarray    # [n] 1 accept, 0 reject, -1 unsure after the last stage
    stage: np.ndarray       # [n] index of the last stage that processed the item
    logits: np.ndarray      # [n, 2] that stage's logits
    processed: np.ndarray   # [n_stages] items each stage processed


def cascade_filter(m: om.Model, caches: Sequence[om.Cache], stages: Sequence[Stage], suffix, yes_id: int,
                   no_id: int) -> CascadeResult:
    n = len(caches)
    decision = np.full(n, -1, np.int64)
    stage = np.full(n, -1, np.int64)
    logits = np.zeros((n, 2))
    processed = np.zeros(len(stages), np.int64)
    for i, st in enumerate(stages):
        for t in range(n):
            if decision[t] != -1:          # decided by an earlier operator: not passed on
                continue
            res = om.filter_eval(m, caches[t], st.retained[t], suffix, yes_id, no_id, st.theta_pos, st.theta_neg)
            decision[t], stage[t], logits[t] = res.decision, i, res.logits
            processed[i] += 1
    return CascadeResult(decision, stage, logits, processed)


def recurrence(stage_decisions: np.ndarray):
    """Eqs. 1-3 on a full table of per-stage decisions [n_stages, n] (1 / 0 / -1 for what o_i
    would answer): returns (accept, reject, unsure) after the last stage and the number of
    tuples each stage processes (Eq. 4's unsure_(i-1) summed over tuples)."""
    n_st, n = stage_decisions.shape
    acc = np.zeros(n, np.int64)
    rej = np.zeros(n, np.int64)
    uns = np.ones(n, np.int64)
    processed = np.zeros(n_st, np.int64)
    for i in range(n_st):
        processed[i] = int(uns.sum())
        a_i = (stage_decisions[i] == 1).astype(np.int64)
        r_i = (stage_decisions[i] == 0).astype(np.int64)
        acc = acc + uns * a_i
        rej = rej + uns * r_i
        uns = 1 - acc - rej
    return acc, rej, uns, processed
