"""Seeded DAGs shaped like the six correlation functions of Table corr-func.

The paper gives, per correlation function, its hadron system (MxM, MxMxM,
BxM, BxB, BxBxB), the number of trees k, the tensor dimension N, and the
merged DAG's vertex and edge counts with the runtime factors F_v and F_e
(Sec. III-B).  The physics graphs themselves are not available, so these
generators draw graphs of the same system with the same number of trees, the
same number of leaves (|V| - |E| / 2, every contraction having two operands)
and about the same number of merged contractions, and report the F_v and F_e
they reach.  Structure only: no tensor data, no method arithmetic.

Each system uses tree templates over meson leaves (rank 2) and baryon leaves
(rank 3) with the engine's kinds (K22, K32, K33, the general C1 and C2, HCA):

  MxM, MxMxM  meson rings tr(A_1 ... A_L), products built left to right, so
              rings that share a prefix share its product.
  BxM         HCA(K33(B, B'), M), or HCA(K33(K32(B, M), B'), M').
  BxB         two baryon pairs K33(B, B'), one side optionally through K32
              with a meson first, the other optionally closed by a meson,
              then HCA.
  BxBxB       two baryons contracted over one index into a rank-4 tensor
              (C1, the O(N^5) step), folded with a third and a fourth baryon
              (C2, K33); the other side a baryon pair or the same chain; HCA.
The template mix sets the mean tree size to the row's F_v |V| / k.

Sharing comes from skewed leaf draws: leaf i of a system is drawn with weight
1 / (1 + r_i)^s for a seeded random rank r_i, and `skew` s is set per row so
that the merged DAG has about the row's number of contractions (fitted once
with tests/golden/fit_corr_func.py, which builds the DAGs with the oracle).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

from .workloads import GraphSpec, K22, K32, K33, HCA, C1, C2, Leaf, Workload

# Table corr-func: system, #trees, N, #vertices, #edges, F_v, F_e.
TABLE = {
    "a0-111":   dict(system="MxM",   trees=19041,  N=1024, V=18552,  E=36120,  f_v=5.09,  f_e=4.09),
    "a0-d3":    dict(system="MxM",   trees=3921,   N=1536, V=3826,   E=7232,   f_v=4.83,  f_e=3.83),
    "f0":       dict(system="MxMxM", trees=27999,  N=768,  V=30473,  E=59416,  f_v=4.95,  f_e=3.96),
    "roper":    dict(system="BxM",   trees=84894,  N=64,   V=90378,  E=180008, f_v=5.67,  f_e=4.67),
    "deuteron": dict(system="BxB",   trees=109444, N=64,   V=156508, E=312720, f_v=7.00,  f_e=6.00),
    "tritium":  dict(system="BxBxB", trees=6085,   N=32,   V=7597,   E=15178,  f_v=10.11, f_e=9.75),
}

# Generator settings per row: leaf counts (mesons, baryons), the tree-size
# mix of the system's templates, and the fitted skew.
PARAMS: Dict[str, dict] = {
    "a0-111":   dict(n_mes=492, n_bar=0, mix=(0.22, 0.58, 0.20), skew=1.3624),
    "a0-d3":    dict(n_mes=210, n_bar=0, mix=(0.30, 0.55, 0.15), skew=1.4745),
    "f0":       dict(n_mes=765, n_bar=0, mix=(0.82, 0.15, 0.03), skew=1.3304),
    "roper":    dict(n_mes=187, n_bar=187, mix=(0.48, 0.52), skew=1.2416),
    "deuteron": dict(n_mes=74, n_bar=74, mix=(0.10, 0.30, 0.60), skew=1.3248),
    "tritium":  dict(n_mes=0, n_bar=8, mix=(0.60, 0.40), skew=0.5226),
}


class _Draw:
    """Skewed draws of distinct leaves from one pool."""

    def __init__(self, rg, ids: List[int], skew: float):
        self.rg = rg
        self.ids = np.asarray(ids, dtype=np.int64)
        rank = rg.permutation(len(ids))
        w = 1.0 / (1.0 + rank) ** skew
        self.p = w / w.sum()

    def pick(self, k: int) -> List[int]:
        idx = self.rg.choice(len(self.ids), size=k, replace=False, p=self.p)
        return [int(self.ids[i]) for i in idx]


def _ring(ops, seq, rg) -> GraphSpec:
    """tr(A_1 ... A_L): left-to-right products P = A_1..A_s, Q = A_{s+1}..A_L
    (s = L - 1 for L <= 3, else a uniform cut), root HCA(P, Q)."""
    L = len(seq)

    def product(s):
        acc = s[0]
        for x in s[1:]:
            ops.append((K22, acc, x))
            acc = -len(ops)
        return acc

    cut = L - 1 if L <= 3 else int(rg.integers(1, L))
    p = product(seq[:cut])
    q = product(seq[cut:])
    ops.append((HCA, p, q))
    return GraphSpec(ops)


def _graph(system: str, mix, mes: Optional[_Draw], bar: Optional[_Draw], rg) -> GraphSpec:
    ops: List[Tuple[int, int, int]] = []
    t = int(rg.choice(len(mix), p=np.asarray(mix) / np.sum(mix)))
    if system in ("MxM", "MxMxM"):
        L = (2 if system == "MxM" else 3) + t
        return _ring(ops, mes.pick(L), rg)
    if system == "BxM":
        b1, b2 = bar.pick(2)
        m = mes.pick(2)
        if t == 0:                      # HCA(K33(B, B'), M)
            ops.append((K33, b1, b2))
            ops.append((HCA, -1, m[0]))
            return GraphSpec(ops)
        ops.append((K32, b1, m[0]))     # HCA(K33(K32(B, M), B'), M')
        ops.append((K33, -1, b2))
        ops.append((HCA, -2, m[1]))
        return GraphSpec(ops)
    if system == "BxB":
        b = bar.pick(4)
        m = mes.pick(2)
        left = b[0]
        if t >= 1:                      # one side passes through a meson first
            ops.append((K32, b[0], m[0]))
            left = -len(ops)
        ops.append((K33, left, b[1]))
        x = -len(ops)
        ops.append((K33, b[2], b[3]))
        y = -len(ops)
        if t == 2:                      # and a second meson closes the loop
            ops.append((K22, y, m[1]))
            y = -len(ops)
        ops.append((HCA, x, y))
        return GraphSpec(ops)
    if system == "BxBxB":
        b = bar.pick(6 + 2 * t)
        ops.append((C1, b[0], b[1]))             # two baryons over one index -> rank 4, O(N^5)
        ops.append((C2, -1, b[2]))               # a third baryon over two indices -> rank 3
        ops.append((K33, -2, b[3]))              # -> rank 2
        x = -3
        if t == 0:
            ops.append((K33, b[4], b[5]))        # a baryon pair -> rank 2
            y = -4
        else:                                    # the second side through rank 4 as well
            ops.append((C1, b[4], b[5]))
            ops.append((C2, -4, b[6]))
            ops.append((K33, -5, b[7]))
            y = -6
        ops.append((HCA, x, y))
        return GraphSpec(ops)
    raise KeyError(system)


def corr_func_like(row: str, n_trees: Optional[int] = None, skew: Optional[float] = None,
                   seed: int = 2000, nt: int = 1) -> Workload:
    """A structure-only workload shaped like Table corr-func row `row`.
    n_trees overrides the row's tree count (smaller test instances); skew
    overrides the fitted skew."""
    tab, par = TABLE[row], PARAMS[row]
    rs = np.random.SeedSequence(seed + sorted(TABLE).index(row))
    rg = np.random.Generator(np.random.PCG64(rs))
    N = tab["N"]
    leaves = [Leaf(2, N, nt) for _ in range(par["n_mes"])] + [Leaf(3, N, nt) for _ in range(par["n_bar"])]
    s = par["skew"] if skew is None else skew
    mes = _Draw(rg, list(range(par["n_mes"])), s) if par["n_mes"] else None
    bar = _Draw(rg, list(range(par["n_mes"], par["n_mes"] + par["n_bar"])), s) if par["n_bar"] else None
    k = tab["trees"] if n_trees is None else n_trees
    graphs = [_graph(tab["system"], par["mix"], mes, bar, rg) for _ in range(k)]
    return Workload(row, leaves, graphs, meta=dict(seed=seed, kind="corr_func", system=tab["system"],
                                                   skew=s))


def with_data(wl: Workload, seed: int = 2100, sigma: Optional[float] = None) -> Workload:
    """The same workload with seeded leaf entries (re and im iid N(0, sigma^2),
    sigma = 1/N by default), so that a Table corr-func-shaped DAG can run on
    the device and be checked against the oracle.  Random numbers only."""
    from .workloads import _draw
    rg = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    leaves = []
    for lf in wl.leaves:
        sg = 1.0 / lf.nvec if sigma is None else sigma
        leaves.append(Leaf(lf.rank, lf.nvec, lf.nt, _draw(rg, (lf.nt,) + (lf.nvec,) * lf.rank, sg)))
    return Workload(wl.name, leaves, wl.graphs, meta=dict(wl.meta, data_seed=seed))
