"""Seeded synthetic contraction-DAG workloads (inputs only, no method arithmetic).

A workload is a list of leaf tensors (complex hadron-node tensors batched over
time slices) plus a list of graphs.  Each graph is a binary contraction tree
written as a list of ops; the last op is the root and is always a trace
("contract all") of two rank-2 tensors.

Operand encoding inside a graph: an operand >= 0 is a leaf id; an operand < 0
is -(1 + index of an earlier op of the same graph).

Contraction kinds (index conventions, all per time slice t):
  K22: O[i,j]   = sum_k   X[i,k]   Y[k,j]        (meson x meson)
  K32: O[i,j,l] = sum_k   X[i,j,k] Y[k,l]        (baryon x meson, one index)
  K33: O[i,m]   = sum_jl  X[i,j,l] Y[j,l,m]      (baryon x baryon, two indices)
  HCA: C        = sum_ij  P[i,j]   Q[j,i]        (trace of the product)

Random numbers: numpy PCG64 seeded through SeedSequence(seed), spawned into
two independent streams, one for tensor entries and one for graph structure,
so that a structure-only workload (with_data=False) has exactly the same
graphs as the full one.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

K22, K32, K33, HCA = 0, 1, 2, 3
C1, C2, C3 = 4, 5, 6      # general: last c axes of X against the first c of Y
SPEC_BASE = 16            # op kind SPEC_BASE + i: the workload's contraction spec i
KIND_NAMES = {K22: "K22", K32: "K32", K33: "K33", HCA: "HCA", C1: "C1", C2: "C2", C3: "C3"}


@dataclass
class Leaf:
    rank: int
    nvec: int
    nt: int
    data: Optional[np.ndarray] = None  # complex128, shape [nt] + [nvec]*rank


@dataclass
class Spec:
    """A contraction over any index pairs: operands of ranks rank_l and rank_r,
    axis pairs[k][0] of the left one summed against axis pairs[k][1] of the
    right one; the output holds the left operand's free axes in order, then the
    right one's, arranged so that output axis j is axis perm[j] of that list
    (axes count from 0 after the time slice)."""
    rank_l: int
    rank_r: int
    pairs: Tuple[Tuple[int, int], ...]
    perm: Tuple[int, ...]


@dataclass
class GraphSpec:
    ops: List[Tuple[int, int, int]]
    corr: int = 0
    w: complex = 1.0


@dataclass
class Workload:
    name: str
    leaves: List[Leaf]
    graphs: List[GraphSpec]
    # Budget: an explicit byte count, or None with a named rule in budget_rule
    # ("unlimited", or "quarter_input_peak_live": a quarter of the peak live
    # bytes of the input-order schedule, computed by whoever runs the plan).
    budget_bytes: Optional[int] = None
    budget_rule: str = "unlimited"
    meta: dict = field(default_factory=dict)
    specs: List[Spec] = field(default_factory=list)   # op kinds SPEC_BASE + i

    @property
    def n_corr(self) -> int:
        return 1 + max(g.corr for g in self.graphs) if self.graphs else 0


def _streams(seed: int):
    ts, gs = np.random.SeedSequence(seed).spawn(2)
    return (np.random.Generator(np.random.PCG64(ts)),
            np.random.Generator(np.random.PCG64(gs)))


def _draw(rng, shape, sigma, dtype=np.complex128) -> np.ndarray:
    """Complex tensor with re and im iid N(0, sigma^2), re drawn first.  complex64
    tensors draw float32 normals (a different stream than complex128 ones)."""
    out = np.empty(shape, dtype=dtype)
    if dtype == np.complex64:
        out.real = rng.standard_normal(shape, dtype=np.float32) * np.float32(sigma)
        out.imag = rng.standard_normal(shape, dtype=np.float32) * np.float32(sigma)
    else:
        out.real = rng.standard_normal(shape) * sigma
        out.imag = rng.standard_normal(shape) * sigma
    return out


def _leaf(rng, rank, nvec, nt, sigma, with_data, dtype=np.complex128) -> Leaf:
    shape = (nt,) + (nvec,) * rank
    return Leaf(rank, nvec, nt, _draw(rng, shape, sigma, dtype) if with_data else None)


def _ring_graph(rg, leaf_ids: List[int], lmin: int, lmax: int, n_corr: int) -> GraphSpec:
    """One meson ring trace over distinct leaves, contracted as a random binary tree.

    The ring tr(A_1 ... A_L) is cut at a uniform point into P = A_1..A_s and
    Q = A_{s+1}..A_L (root: HCA(P, Q)); each part is a product split
    recursively at a uniform point.  Ops are emitted children first.
    """
    L = int(rg.integers(lmin, lmax + 1))
    pick = rg.choice(len(leaf_ids), size=L, replace=False)
    seq = [leaf_ids[int(i)] for i in pick]
    ops: List[Tuple[int, int, int]] = []

    def product(s):
        if len(s) == 1:
            return s[0]
        k = int(rg.integers(1, len(s)))
        left = product(s[:k])
        right = product(s[k:])
        ops.append((K22, left, right))
        return -len(ops)

    top = int(rg.integers(1, L))
    p = product(seq[:top])
    q = product(seq[top:])
    ops.append((HCA, p, q))
    corr = int(rg.integers(0, n_corr))
    w = float(rg.choice(np.array([-1.0, 1.0])))
    return GraphSpec(ops, corr, w)


def _chain_graph(rg, bar_ids: List[int], mes_ids: List[int], n_corr: int) -> GraphSpec:
    """One baryon chain: X = K32(B_a, M_b); Y = K33(X, B_c); C = HCA(Y, M_d), a!=c, b!=d."""
    a = int(rg.integers(0, len(bar_ids)))
    c = int(rg.integers(0, len(bar_ids) - 1))
    c += c >= a
    b = int(rg.integers(0, len(mes_ids)))
    d = int(rg.integers(0, len(mes_ids) - 1))
    d += d >= b
    ops = [(K32, bar_ids[a], mes_ids[b]), (K33, -1, bar_ids[c]), (HCA, -2, mes_ids[d])]
    corr = int(rg.integers(0, n_corr))
    w = float(rg.choice(np.array([-1.0, 1.0])))
    return GraphSpec(ops, corr, w)


def meson_ring(n_leaves=16, nvec=64, nt=32, n_graphs=2000, lmin=4, lmax=8, sigma=1 / 8,
               n_corr=8, seed=1002, with_data=True, name="meson_ring") -> Workload:
    rt, rg = _streams(seed)
    leaves = [_leaf(rt, 2, nvec, nt, sigma, with_data) for _ in range(n_leaves)]
    ids = list(range(n_leaves))
    graphs = [_ring_graph(rg, ids, lmin, lmax, n_corr) for _ in range(n_graphs)]
    return Workload(name, leaves, graphs,
                    meta=dict(seed=seed, sigma=sigma, kind="meson_ring"))


def baryon_mix(n_bar=12, n_mes=12, nvec=64, nt=32, n_graphs=500, sigma=1 / 64, n_corr=4,
               seed=1003, with_data=True, name="baryon_mix") -> Workload:
    rt, rg = _streams(seed)
    leaves = [_leaf(rt, 3, nvec, nt, sigma, with_data) for _ in range(n_bar)]
    leaves += [_leaf(rt, 2, nvec, nt, sigma, with_data) for _ in range(n_mes)]
    bar = list(range(n_bar))
    mes = list(range(n_bar, n_bar + n_mes))
    graphs = [_chain_graph(rg, bar, mes, n_corr) for _ in range(n_graphs)]
    return Workload(name, leaves, graphs,
                    meta=dict(seed=seed, sigma=sigma, kind="baryon_mix"))


def tiny_meson_perm(nvec=16, nt=8, n_graphs=6, sigma=1 / 4, seed=1001, with_data=True,
                    name="tiny") -> Workload:
    """Four meson leaves; each graph is tr(A_a A_b A_c A_d) for a distinct seeded
    permutation (a,b,c,d), contracted as HCA(K22(a,b), K22(c,d))."""
    rt, rg = _streams(seed)
    leaves = [_leaf(rt, 2, nvec, nt, sigma, with_data) for _ in range(4)]
    seen, graphs = set(), []
    while len(graphs) < n_graphs:
        p = tuple(int(x) for x in rg.permutation(4))
        if p in seen:
            continue
        seen.add(p)
        w = float(rg.choice(np.array([-1.0, 1.0])))
        graphs.append(GraphSpec([(K22, p[0], p[1]), (K22, p[2], p[3]), (HCA, -1, -2)], 0, w))
    return Workload(name, leaves, graphs, meta=dict(seed=seed, sigma=sigma, kind="tiny"))


def fig1_dag(order: str = "fgh", nvec=4, nt=1, seed=7, with_data=True) -> Workload:
    """Three-tree DAG with leaves a,b,c,d (ids 0..3), all tensors the same size.

    Roots f = a.b, g = a.e, h = e.d with the shared interior node e = b.c.
    `order` gives the order in which the three graphs are listed.
    """
    rt, _ = _streams(seed)
    leaves = [_leaf(rt, 2, nvec, nt, 0.5, with_data) for _ in range(4)]
    a, b, c, d = 0, 1, 2, 3
    spec = {
        "f": GraphSpec([(HCA, a, b)], 0, 1.0),
        "g": GraphSpec([(K22, b, c), (HCA, a, -1)], 0, 1.0),
        "h": GraphSpec([(K22, b, c), (HCA, -1, d)], 0, 1.0),
    }
    return Workload("fig1_" + order, leaves, [spec[ch] for ch in order],
                    meta=dict(seed=seed, kind="fig1"))


def _rank4_graph(rg, bar: List[int], mes: List[int], r4: List[int], n_corr: int) -> GraphSpec:
    """One graph through a rank-4 intermediate; four templates (a..d distinct):
      0: HCA(K33(C2(C1(B_a, B_b), B_c), B_d), M_e)     rank 4 -> 3 -> 2
      1: HCA(C3(C1(B_a, B_b), R_c), M_e)               rank 4 with a rank-4 leaf -> 2
      2: HCA(K33(C1(M_e, B_a), B_b), M_f)              C1 on ranks (2, 3) -> 3 -> 2
      3: HCA(C2(R_c, M_e), M_f)                        rank-4 leaf against a meson -> 2"""
    t = int(rg.integers(0, 4))
    b = [bar[int(i)] for i in rg.choice(len(bar), size=4, replace=False)]
    m = [mes[int(i)] for i in rg.choice(len(mes), size=2, replace=False)]
    r = r4[int(rg.integers(0, len(r4)))]
    if t == 0:
        ops = [(C1, b[0], b[1]), (C2, -1, b[2]), (K33, -2, b[3]), (HCA, -3, m[0])]
    elif t == 1:
        ops = [(C1, b[0], b[1]), (C3, -1, r), (HCA, -2, m[0])]
    elif t == 2:
        ops = [(C1, m[0], b[0]), (K33, -1, b[1]), (HCA, -2, m[1])]
    else:
        ops = [(C2, r, m[0]), (HCA, -1, m[1])]
    corr = int(rg.integers(0, n_corr))
    w = float(rg.choice(np.array([-1.0, 1.0])))
    return GraphSpec(ops, corr, w)


def rank4_mix(n_bar=5, n_mes=4, n_r4=2, nvec=6, nt=3, n_graphs=24, sigma=None, n_corr=2, seed=1006,
              with_data=True, name="rank4") -> Workload:
    """Graphs with rank-4 intermediates and rank-4 leaves through the general
    contractions C1, C2, C3 (tritium-like O(N^5) steps); entries N(0,1)/N."""
    rt, rg = _streams(seed)
    sg = 1.0 / nvec if sigma is None else sigma
    leaves = [_leaf(rt, 3, nvec, nt, sg, with_data) for _ in range(n_bar)]
    leaves += [_leaf(rt, 2, nvec, nt, sg, with_data) for _ in range(n_mes)]
    leaves += [_leaf(rt, 4, nvec, nt, sg, with_data) for _ in range(n_r4)]
    bar = list(range(n_bar))
    mes = list(range(n_bar, n_bar + n_mes))
    r4 = list(range(n_bar + n_mes, n_bar + n_mes + n_r4))
    graphs = [_rank4_graph(rg, bar, mes, r4, n_corr) for _ in range(n_graphs)]
    return Workload(name, leaves, graphs, meta=dict(seed=seed, kind="rank4"))


# Contraction specs over other index pairs than the trailing-against-leading
# ones, with output orders other than the natural one (Spec); the fifth is C1
# on two baryons written as a spec.
PAIR_SPECS = (
    Spec(3, 2, ((0, 1),), (2, 0, 1)),          # X[i,j,l] Y[k,i] -> O[k,j,l]
    Spec(3, 3, ((2, 0), (0, 2)), (1, 0)),      # X[a,b,c] Y[c,e,a] -> O[e,b]
    Spec(2, 2, ((0, 0),), (1, 0)),             # X[i,j] Y[i,k] -> O[k,j]
    Spec(4, 3, ((1, 0), (3, 2)), (0, 2, 1)),   # X[a,b,c,d] Y[b,e,d] -> O[a,e,c]
    Spec(3, 3, ((2, 0),), (0, 1, 2, 3)),       # C1 on two baryons
    Spec(3, 3, ((1, 1),), (3, 1, 0, 2)),       # X[a,b,c] Y[d,b,e] -> O[e,c,a,d]
)


def _pairs_graph(rg, bar: List[int], mes: List[int], r4: List[int], n_corr: int) -> GraphSpec:
    """One graph through contractions over other index pairs (PAIR_SPECS,
    kinds SPEC_BASE + i); templates (distinct leaves a, b, c, ...):
      0: HCA(S1(S0(B_a, M_b), B_c), M_d)
      1: HCA(S2(M_a, M_b), M_c)
      2: HCA(S1(B_a, B_b), S2(M_a, M_b))
      3: HCA(S1(S3(R, B_a), B_b), M_c)
      4: HCA(K33(C2(S4(B_a, B_b), B_c), B_d), M_e)     S4 is C1 written as a spec
      5: HCA(K33(C2(C1(B_a, B_b), B_c), B_d), M_e)     (merges with template 4)
      6: HCA(C2(S5(B_a, B_b), M_c), M_d)"""
    S = [SPEC_BASE + i for i in range(len(PAIR_SPECS))]
    t = int(rg.integers(0, 7))
    b = [bar[int(i)] for i in rg.choice(len(bar), size=4, replace=False)]
    m = [mes[int(i)] for i in rg.choice(len(mes), size=3, replace=False)]
    r = r4[int(rg.integers(0, len(r4)))]
    if t == 0:
        ops = [(S[0], b[0], m[0]), (S[1], -1, b[1]), (HCA, -2, m[1])]
    elif t == 1:
        ops = [(S[2], m[0], m[1]), (HCA, -1, m[2])]
    elif t == 2:
        ops = [(S[1], b[0], b[1]), (S[2], m[0], m[1]), (HCA, -1, -2)]
    elif t == 3:
        ops = [(S[3], r, b[0]), (S[1], -1, b[1]), (HCA, -2, m[0])]
    elif t in (4, 5):
        ops = [(S[4] if t == 4 else C1, b[0], b[1]), (C2, -1, b[2]), (K33, -2, b[3]), (HCA, -3, m[0])]
    else:
        ops = [(S[5], b[0], b[1]), (C2, -1, m[0]), (HCA, -2, m[1])]
    return GraphSpec(ops, int(rg.integers(0, n_corr)), float(rg.choice(np.array([-1.0, 1.0]))))


def pairs_mix(n_bar=5, n_mes=5, n_r4=2, nvec=6, nt=3, n_graphs=30, sigma=None, n_corr=2, seed=1007,
              with_data=True, name="pairs") -> Workload:
    """Graphs through contractions over other index pairs and output orders
    (PAIR_SPECS), beside named and general kinds; entries N(0,1)/N."""
    rt, rg = _streams(seed)
    sg = 1.0 / nvec if sigma is None else sigma
    leaves = [_leaf(rt, 3, nvec, nt, sg, with_data) for _ in range(n_bar)]
    leaves += [_leaf(rt, 2, nvec, nt, sg, with_data) for _ in range(n_mes)]
    leaves += [_leaf(rt, 4, nvec, nt, sg, with_data) for _ in range(n_r4)]
    bar = list(range(n_bar))
    mes = list(range(n_bar, n_bar + n_mes))
    r4 = list(range(n_bar + n_mes, n_bar + n_mes + n_r4))
    graphs = [_pairs_graph(rg, bar, mes, r4, n_corr) for _ in range(n_graphs)]
    return Workload(name, leaves, graphs, meta=dict(seed=seed, kind="pairs"), specs=list(PAIR_SPECS))


BATCHED_NVECS = (32, 48, 64, 96, 128)


def batched_mix(nvecs=BATCHED_NVECS, nt=64, n_mes=8, n_bar=8, n_graphs=13000, lmin=4, lmax=6,
                n_corr_per_family=4, seed=1005, with_data=True, name="batched",
                dtype=np.complex64) -> Workload:
    """Families of equal N, one per entry of `nvecs`; graphs are added round-robin
    over families, alternating meson rings and baryon chains within a family.
    Entries are N(0,1)/N, stored as complex64.  13000 graphs merge into just over
    20,000 contractions at the default sizes."""
    rt, rg = _streams(seed)
    leaves: List[Leaf] = []
    fam = []
    for n in nvecs:
        base = len(leaves)
        leaves += [_leaf(rt, 2, n, nt, 1.0 / n, with_data, dtype) for _ in range(n_mes)]
        leaves += [_leaf(rt, 3, n, nt, 1.0 / n, with_data, dtype) for _ in range(n_bar)]
        fam.append((list(range(base, base + n_mes)),
                    list(range(base + n_mes, base + n_mes + n_bar))))
    graphs: List[GraphSpec] = []
    turn = [0] * len(nvecs)
    for g in range(n_graphs):
        f = g % len(nvecs)
        mes, bar = fam[f]
        if turn[f] % 2 == 0:
            spec = _ring_graph(rg, mes, lmin, lmax, n_corr_per_family)
        else:
            spec = _chain_graph(rg, bar, mes, n_corr_per_family)
        spec.corr += f * n_corr_per_family
        turn[f] += 1
        graphs.append(spec)
    return Workload(name, leaves, graphs, budget_bytes=64 * 10**9, budget_rule="bytes",
                    meta=dict(seed=seed, kind="batched", nvecs=list(nvecs), nt=nt))


CONFIG_NAMES = ("tiny", "meson_ring", "baryon_mix", "batched")


def config(name: str, with_data: bool = True) -> Workload:
    """The named workloads at their full sizes.

    tiny        4 mesons [8][16][16], 6 permutation traces, unlimited memory.
    meson_ring  16 mesons [32][64][64], 2000 ring traces of 4..8 leaves; budget a
                quarter of the input-order schedule's peak live bytes.
    baryon_mix  12 baryons [32][64]^3 + 12 mesons [32][64]^2, 500 chains; 32 GB budget.
    batched     five N families at Nt=64, mixed ranks; 64 GB budget.
    """
    if name == "tiny":
        return tiny_meson_perm(with_data=with_data)
    if name == "meson_ring":
        w = meson_ring(with_data=with_data)
        w.budget_rule = "quarter_input_peak_live"
        return w
    if name == "baryon_mix":
        w = baryon_mix(with_data=with_data)
        w.budget_bytes, w.budget_rule = 32 * 10**9, "bytes"
        return w
    if name == "batched":
        return batched_mix(with_data=with_data)
    raise KeyError(name)
