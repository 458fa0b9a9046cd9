"""Seeded general DAGs for the schedulers: nodes with any number of children.

Structure only (node sizes in bytes and child lists), no method arithmetic.
Trees are grown one after another over a pool of leaves; an inner slot reuses
an already built inner node with probability `share` (which merges trees and
can make one tree reach a node along two paths, so a tree's node set is a DAG),
otherwise it takes a leaf or a fresh node of 1..max_arity distinct children.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def random_general(seed: int, n_leaves: int = 12, n_trees: int = 8, max_arity: int = 4,
                   depth: int = 3, share: float = 0.3, max_size: int = 1000,
                   zero_roots: bool = True) -> Tuple[int, List[int], List[Tuple[int, ...]]]:
    """(n_leaves, sizes, children) of a seeded general DAG.  Node ids are
    topological (children before parents).  With zero_roots the nodes left
    without a parent get size 0, like a root's per-t scalar."""
    rg = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    sizes: List[int] = [int(x) for x in rg.integers(1, max_size + 1, size=n_leaves)]
    children: List[Tuple[int, ...]] = [()] * n_leaves
    inner: List[int] = []

    def make(level: int) -> int:
        if inner and rg.random() < share:
            return int(inner[int(rg.integers(len(inner)))])
        if level == 0 or rg.random() < 0.25:
            return int(rg.integers(n_leaves))
        k = int(rg.integers(1, max_arity + 1))
        kids: List[int] = []
        for _ in range(k):
            x = make(level - 1)
            if x not in kids:
                kids.append(x)
        u = len(children)
        children.append(tuple(kids))
        sizes.append(int(rg.integers(1, max_size + 1)))
        inner.append(u)
        return u

    for _ in range(n_trees):
        k = int(rg.integers(1, max_arity + 1))
        kids: List[int] = []
        for _ in range(k):
            x = make(depth - 1)
            if x not in kids:
                kids.append(x)
        children.append(tuple(kids))
        sizes.append(int(rg.integers(1, max_size + 1)))
        inner.append(len(children) - 1)
    if zero_roots:
        has_parent = [False] * len(children)
        for c in children:
            for x in c:
                has_parent[x] = True
        for u in range(n_leaves, len(children)):
            if not has_parent[u]:
                sizes[u] = 0
    return n_leaves, sizes, children
