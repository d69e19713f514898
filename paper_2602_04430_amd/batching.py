"""Host-side planning of the batching form over a document collection larger than HBM.

The caches of the mixed-operator workload (16384 documents) exceed one GPU's memory, so the
items are processed in groups: each operator's items are split into G consecutive parts and
group g holds part g of every operator, with the documents those items read.  G is the
smallest count whose every group's caches fit the given capacity.  Inside a group the items
of all operators are interleaved in a seeded order and evaluated by one kvop_mixed_eval
call.  No arithmetic of the operator is here: this only decides which items share a call.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def group_parts(filter_docs, map_docs, pairs, G: int, g: int):
    """Part g of G of every operator's items: (filter docs, map docs, join pairs)."""
    return (np.array_split(np.asarray(filter_docs), G)[g], np.array_split(np.asarray(map_docs), G)[g],
            np.array_split(np.asarray(pairs).reshape(-1, 2), G)[g])


def group_docs(fg, mg, pg) -> List[int]:
    """Documents a group reads, ascending."""
    return sorted(set(int(x) for x in fg) | set(int(x) for x in mg) | set(int(x) for x in np.ravel(pg)))


def plan_groups(doc_bytes: Sequence[int], filter_docs, map_docs, pairs, capacity: int) -> int:
    """Smallest G such that every group's documents occupy at most `capacity` bytes."""
    doc_bytes = np.asarray(doc_bytes)
    G = 1
    while True:
        if all(doc_bytes[group_docs(*group_parts(filter_docs, map_docs, pairs, G, g))].sum() <= capacity
               for g in range(G)):
            return G
        G += 1


def interleave(nf: int, nm: int, nj: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Operator index and first list index of every item of one group, in a seeded order.

    The group's lists are laid out filter items first (one list each), then map items (one
    each), then join items (two consecutive lists each)."""
    item_op = np.concatenate([np.zeros(nf), np.ones(nm), 2 * np.ones(nj)]).astype(np.int32)
    item_list = np.concatenate([np.arange(nf), nf + np.arange(nm), nf + nm + 2 * np.arange(nj)]).astype(np.int64)
    perm = np.random.default_rng(seed).permutation(len(item_op))
    return item_op[perm], item_list[perm]


def output_order(item_op, item_list, nf: int, nm: int):
    """For each operator, the item (by its position in that operator's part) behind every
    output row: a mixed call writes an operator's outputs in the order its items appear."""
    item_op, item_list = np.asarray(item_op), np.asarray(item_list)
    return (item_list[item_op == 0], item_list[item_op == 1] - nf, (item_list[item_op == 2] - nf - nm) // 2)
