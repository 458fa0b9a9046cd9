"""Pins of the oracle's DAG build, schedulers and memory model (CPU only).

What pins what:
  * Table sch-mem (Sec. II-C): memory contents and sizes after each contraction of
    S1 and S2 on the Fig. 1 DAG (golden fixture, one cell read as a typo).
  * Fig. 3's initial individual gains (b: -1 in every tree, c in T2: 0).
  * Fig. 4's five PROCESS-CHILD cases, seen through the gain definition M - M'.
  * Eq. (1) ranks; M_n = 0; peak_post <= peak_live; each contraction once; brute
    force optimum <= every heuristic; F_v / F_e by hand on Fig. 1.
  * Node-based gain scheduler: two DAGs worked by hand; every pick is the ready
    contraction with the largest drop in resident bytes by direct set reasoning
    (independent of memsim), lowest id on ties; a chain has one order.
"""
import itertools
import json
import os
import random

import pytest

from synth import workloads as W
from oracle import dag as D
from oracle import schedules as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table_sch_mem.json")
NAMES = dict(a=0, b=1, c=2, d=3)


def fig1(order="fgh"):
    wl = W.fig1_dag(order, with_data=False)
    d = D.build(wl.leaves, wl.graphs)
    names = dict(NAMES)
    # roots and e by structure, independent of creation order
    for u in d.contractions():
        key = (d.left[u], d.right[u])
        names[{(0, 1): "f", (1, 2): "e", (0, 4): "g", (0, 5): "g", (0, 6): "g",
               (0, 7): "g"}.get(key, "?")] = u
    e = names["e"]
    for u in d.contractions():
        if (d.left[u], d.right[u]) == (0, e):
            names["g"] = u
        if (d.left[u], d.right[u]) == (e, 3):
            names["h"] = u
    names.pop("?", None)
    return d, names


def unit(d):
    return d.size(0)


def test_fig1_structure():
    d, n = fig1()
    assert set(n) == set("abcdefgh")
    assert d.node_type(n["e"]) == D.INTERIOR
    for r in "fgh":
        assert d.node_type(n[r]) == D.ROOT
    assert d.n_nodes == 8 and len(d.tree_roots) == 3
    # each contraction is binary: |E| = 2 * #non-leaf nodes
    assert sum(len(p) for p in d.parents) == 2 * len(d.contractions())


@pytest.mark.parametrize("which", ["S1", "S2"])
def test_table_sch_mem(which):
    gold = json.load(open(GOLD))["schedules"][which]
    d, n = fig1()
    inv = {v: k for k, v in n.items()}
    order = [n[x] for x in gold["order"]]
    sim = S.memsim(d, order)
    # unit sizes: every rank-2 tensor here has the same size; roots count 0
    assert [m // unit(d) for m in sim["M"]] == gold["size"]
    assert [sorted(inv[u] for u in c) for c in sim["contents"]] == gold["after"]
    assert sim["M"][-1] == 0


def test_peak_live_vs_post_on_fig1():
    d, n = fig1()
    s1 = S.memsim(d, [n[x] for x in "eghf"])
    s2 = S.memsim(d, [n[x] for x in "fegh"])
    assert (s1["peak_post"], s2["peak_post"]) == (3 * unit(d), 2 * unit(d))
    # while e = b.c runs in S1: b, c and the output e coexist
    assert s1["peak_live"] == 4 * unit(d)
    for s in (s1, s2):
        assert s["peak_post"] <= s["peak_live"]


def test_igain_example():
    gold = json.load(open(GOLD))["igain_example"]
    d, n = fig1("fgh")
    ig = S.tree_initial_igains(d)
    for i in range(3):
        assert ig[i][n["b"]] == gold["b_in_every_tree"] * unit(d)
    # the second tree holds c and e (the tree of g); c's only parent e is in it
    assert ig[1][n["c"]] == gold["c_in_second_tree"]
    assert [sum(g.values()) // unit(d) for g in ig] == [-2, -3, -2]


def test_ranks_eq1():
    d, n = fig1()
    rk = S.ranks(d)
    assert [rk[n[x]] for x in "abcd"] == [0, 0, 0, 0]
    assert rk[n["e"]] == 1 and rk[n["f"]] == 1
    assert rk[n["g"]] == 2 and rk[n["h"]] == 2


def test_tree_and_sibling_on_fig1():
    d, n = fig1("fgh")
    inv = {v: k for k, v in n.items()}
    # Tree: T_f and T_h tie at -2 (lowest index wins), then T_g has gain +1
    assert "".join(inv[u] for u in S.tree(d)) == "fegh"
    # Sibling picks leaf a first; with this input order f and e enter Q1 in that order
    assert "".join(inv[u] for u in S.sibling(d)) == "fegh"
    d2, n2 = fig1("ghf")
    inv2 = {v: k for k, v in n2.items()}
    # with g listed first, e precedes f in b's parent list: Sibling yields S1
    assert "".join(inv2[u] for u in S.sibling(d2)) == "eghf"
    assert "".join(inv2[u] for u in S.input_order(d2)) == "eghf"
    assert "".join(inv[u] for u in S.input_order(d)) == "fegh"


def test_fv_fe_by_hand():
    d, _ = fig1()
    st = D.stats(d)
    assert st["n_edges"] == 8
    assert abs(st["f_v"] - 13 / 8) < 1e-15
    assert abs(st["f_e"] - 10 / 8) < 1e-15


# ------------------------------------------------------------ Fig. 4 cases
class _Leaf:
    def __init__(self, rank, nvec=4, nt=1):
        self.rank, self.nvec, self.nt = rank, nvec, nt


class _G:
    def __init__(self, ops):
        self.ops = ops


def _gain_change(leaves, graphs, first, then, target):
    d = D.build(leaves, graphs)
    st = S._TreeState(d, [d.size(u) for u in range(d.n_nodes)])
    for i in first:
        st.process(i)
    g0 = st.gain(target)
    st.process(then)
    return d, g0, st.gain(target)


def test_case_2a_and_2b():
    # x = leaf 0 is brought in by tree 0; u = root of tree 1 (not in T_i); T_i = tree 2
    L = [_Leaf(2) for _ in range(5)]
    gs = [_G([(W.HCA, 0, 1)]), _G([(W.HCA, 0, 2)]), _G([(W.HCA, 0, 3)])]
    d, g0, g1 = _gain_change(L, gs, [0], 1, 2)
    assert g1 - g0 == d.size(0)            # 2.a: delta(x,T_i) was 1 -> +x.size
    gs.append(_G([(W.HCA, 0, 4)]))         # another outside parent keeps x alive
    d, g0, g1 = _gain_change(L, gs, [0], 1, 2)
    assert g1 - g0 == 0                    # 2.b: delta(x,T_i) > 1 -> no change


def test_case_1a_1b_1c():
    # leaves: x=0, y=1, y2=2, y3=3, y4=4 (rank 3); m=5, m3=6, m4=7, m5=8 (rank 2).
    # Tree 0 brings x in; T' (tree 1) and T_i (tree 2) share u = K33(x, y).
    L = [_Leaf(3) for _ in range(5)] + [_Leaf(2) for _ in range(4)]
    t0 = _G([(W.K33, 0, 2), (W.HCA, -1, 5)])
    tp = _G([(W.K33, 0, 1), (W.HCA, -1, 6)])
    ti = _G([(W.K33, 0, 1), (W.HCA, -1, 7)])
    d, g0, g1 = _gain_change(L, [t0, tp, ti], [0], 1, 2)
    sx, su = d.size(0), d.size(d.left[d.root_of_graph[1]])
    assert sx != su
    # u's own updates give +2 s_u (its igain leaves T_i's sum, then 2.a once T'
    # has used it); case 1.a adds -s_x: x's last AVAIL parent u was in T_i.
    assert g1 - g0 == 2 * su - sx
    # 1.b: tau(x, T_i) = 2 (x also feeds another node of T_i) -> no x term
    ti_b = _G([(W.K33, 0, 1), (W.K33, 0, 3), (W.HCA, -1, -2)])
    d, g0, g1 = _gain_change(L, [t0, tp, ti_b], [0], 1, 2)
    assert g1 - g0 == 2 * su
    # 1.c: tau(x, T_i) = 1 and delta(x, T_i) = 1 (a third, unprocessed tree uses x)
    tz = _G([(W.K33, 0, 4), (W.HCA, -1, 8)])
    d, g0, g1 = _gain_change(L, [t0, tp, ti, tz], [0], 1, 2)
    assert g1 - g0 == 2 * su


# ------------------------------------------------------------ random DAG checks
def random_ring(seed, n_leaves=6, n_graphs=8, lmin=3, lmax=5):
    wl = W.meson_ring(n_leaves=n_leaves, nvec=4, nt=1, n_graphs=n_graphs, lmin=lmin,
                      lmax=lmax, seed=seed, with_data=False)
    return D.build(wl.leaves, wl.graphs)


def random_mixed(seed):
    """Mixed sizes: meson rings and baryon chains of one N in one DAG."""
    rng = random.Random(seed)
    leaves = [_Leaf(3) for _ in range(3)] + [_Leaf(2) for _ in range(4)]
    gs = []
    for _ in range(rng.randint(3, 7)):
        if rng.random() < 0.5:
            a, c = rng.sample(range(3), 2)
            b, dd = rng.sample(range(3, 7), 2)
            gs.append(_G([(W.K32, a, b), (W.K33, -1, c), (W.HCA, -2, dd)]))
        else:
            seq = rng.sample(range(3, 7), rng.randint(2, 4))
            ops = []
            cur = seq[0]
            for x in seq[1:-1]:
                ops.append((W.K22, cur, x))
                cur = -len(ops)
            ops.append((W.HCA, cur, seq[-1]))
            gs.append(_G(ops))
    return D.build(leaves, gs)


@pytest.mark.parametrize("seed", range(40))
def test_heuristics_valid_and_bounded(seed):
    d = random_ring(seed) if seed % 2 == 0 else random_mixed(seed)
    n_contr = len(d.contractions())
    peaks = {}
    for pol in ("input", "sibling", "tree", "node"):
        order = S.schedule(d, pol)
        assert sorted(order) == sorted(d.contractions())      # each processed once
        sim = S.memsim(d, order)                               # raises if not topological
        assert sim["M"][-1] == 0
        assert sim["peak_post"] <= sim["peak_live"]
        peaks[pol] = sim["peak_post"]
    if n_contr <= 8:
        opt = S.optimal_peak(d)
        assert all(opt <= p for p in peaks.values())


@pytest.mark.parametrize("seed", range(30))
def test_tree_gain_cache_matches_full_recompute(seed):
    d = random_ring(seed, n_leaves=7, n_graphs=12) if seed % 2 else random_mixed(seed)
    assert S.tree(d) == S.tree(d, recompute_all=True)


@pytest.mark.parametrize("seed", range(10))
def test_tree_gain_is_memory_difference(seed):
    """tgain of the chosen tree equals M - M' measured by memsim on the prefix."""
    d = random_mixed(seed)
    sizes = [d.size(u) for u in range(d.n_nodes)]
    st = S._TreeState(d, sizes)
    order = []
    alive = set(range(len(d.tree_roots)))
    while alive:
        gains = {i: st.gain(i) for i in alive}
        best = max(sorted(alive), key=lambda i: gains[i])
        before = _mem_after(d, order)
        order += [u for u in st.process(best) if d.kind[u] >= 0]
        after = _mem_after(d, order)
        assert gains[best] == before - after
        alive.discard(best)


def _mem_after(d, prefix):
    """Memory after running `prefix` under Sec. II-C, counting leaves whose users all
    ran as released, by direct set reasoning (independent of memsim)."""
    done = set(prefix)
    total = 0
    for x in range(d.n_nodes):
        used_by = d.parents[x]
        started = (x in done) if d.kind[x] >= 0 else any(p in done for p in used_by)
        if started and any(p not in done for p in used_by):
            total += d.size(x)
    return total


def test_build_validation():
    L = [_Leaf(2), _Leaf(2), _Leaf(3)]
    bad = [
        [(W.K22, 0, 0), (W.HCA, -1, 1)],        # identical operands
        [(W.K22, 0, 1)],                         # root is not a trace
        [(W.HCA, 0, 1), (W.HCA, 0, 1)],          # trace before the end
        [(W.K22, 0, 5), (W.HCA, -1, 1)],         # leaf id out of range
        [(W.K22, 0, -1), (W.HCA, -1, 1)],        # self reference
        [(W.K22, 2, 1), (W.HCA, -1, 1)],         # rank mismatch
        [(W.K22, 0, 1), (W.K22, 1, 0), (W.HCA, -1, 0)],   # op 1 unused
    ]
    for ops in bad:
        with pytest.raises(D.InvalidGraph):
            D.build(L, [_G(ops)])
    with pytest.raises(D.InvalidGraph):
        D.build([_Leaf(2, nvec=4), _Leaf(2, nvec=5)], [_G([(W.HCA, 0, 1)])])
    # general contractions: operand and output ranks must stay within 2..4
    L4 = [_Leaf(2), _Leaf(3), _Leaf(4), _Leaf(4), _Leaf(3)]
    for ops in ([(W.C2, 0, 1), (W.HCA, -1, 0)],          # output rank 1
                [(W.C1, 2, 3), (W.HCA, -1, 0)],          # output rank 6
                [(W.C3, 1, 4), (W.HCA, -1, 0)],          # output rank 0
                [(9, 0, 1), (W.HCA, -1, 0)]):            # no such kind
        with pytest.raises(D.InvalidGraph):
            D.build(L4, [_G(ops)])
    with pytest.raises(D.InvalidGraph):
        D.build([_Leaf(5), _Leaf(2)], [_G([(W.HCA, 0, 1)])])


def test_general_kinds_normalize_and_merge():
    """A general contraction with the ranks of a named kind is that kind, so it
    merges with it; others keep their kind and get the output rank
    rl + rr - 2c."""
    L = [_Leaf(2), _Leaf(2), _Leaf(3), _Leaf(3), _Leaf(2), _Leaf(4)]
    g1 = _G([(W.K22, 0, 1), (W.HCA, -1, 4)])
    g2 = _G([(W.C1, 0, 1), (W.K22, -1, 4), (W.HCA, -2, 0)])
    g3 = _G([(W.C1, 2, 3), (W.C3, -1, 5), (W.HCA, -2, 4)])      # rank 4, then 4x4 over 3 -> 2
    g4 = _G([(W.C2, 2, 3), (W.HCA, -1, 4)])                       # = K33
    d = D.build(L, [g1, g2, g3, g4])
    k22 = d.root_of_graph[0] - 1
    assert d.kind[k22] == W.K22 and d.left[k22] == 0 and d.right[k22] == 1
    assert d.n_nodes == 6 + 10 - 1                                # 10 ops; C1(0, 1) of g2 merged
    c1 = next(u for u in range(d.n_nodes) if d.kind[u] == W.C1)
    assert d.rank[c1] == 4 and (d.left[c1], d.right[c1]) == (2, 3)
    c3 = next(u for u in range(d.n_nodes) if d.kind[u] == W.C3)
    assert d.rank[c3] == 2
    k33 = next(u for u in range(d.n_nodes) if d.kind[u] == W.K33)
    assert (d.left[k33], d.right[k33]) == (2, 3)


def test_hash_consing_and_shared_roots():
    wl = W.tiny_meson_perm(with_data=False)
    d = D.build(wl.leaves, wl.graphs)
    pairs = {tuple(g.ops[0][1:]) for g in wl.graphs} | {tuple(g.ops[1][1:]) for g in wl.graphs}
    n_k22 = sum(1 for u in d.contractions() if d.kind[u] == W.K22)
    assert n_k22 == len(pairs)
    # identical graphs share one root and one tree
    d2 = D.build(wl.leaves, wl.graphs + wl.graphs[:2])
    assert len(d2.tree_roots) == len(d.tree_roots) == 6
    assert d2.root_of_graph[6:] == d2.root_of_graph[:2]


def test_optimal_peak_small_exhaustive():
    d, n = fig1()
    orders = list(S.topo_orders(d))
    assert len(orders) == len(set(map(tuple, orders)))
    # 4 contractions, e before g and h: 4!/... = 8 orders with e ahead of g and h
    assert len(orders) == sum(1 for p in itertools.permutations("efgh")
                              if p.index("e") < p.index("g") and p.index("e") < p.index("h"))
    assert S.optimal_peak(d) == 2 * unit(d)


# ---------------------------------------------------------------- general DAGs (any number of children)
def _hand_general():
    """Leaves a, b, c, d (ids 0-3, sizes 1, 2, 4, 8); x = (a, b, c) of size 16
    (id 4, three children); roots r0 = (x, d) (id 5), r1 = (c, d) (id 6) and
    r2 = (x) (id 7, one child), all of size 0."""
    return D.general(4, [1, 2, 4, 8, 16, 0, 0, 0], [(), (), (), (), (0, 1, 2), (4, 3), (2, 3), (4,)])


def test_general_hand_example():
    """Worked by hand from the gain definition M - M' and Sec. II-C.

    Initially nothing is processed (M = 0), so gain(T) = -(bytes that stay
    resident after T: processed nodes with an unprocessed parent).
      T0 = {a,b,c,d,x,r0}: c (r1 pending) 4 + d (r1) 8 + x (r2) 16  -> -28
      T1 = {c,d,r1}:       c (x pending) 4 + d (r0) 8                -> -12
      T2 = {a,b,c,x,r2}:   c (r1) 4 + x (r0) 16                      -> -20
    T1 is taken (order r1), leaving c and d resident (M = 12).  Then
      T0: before, c and d count 12; after, only x (r2 pending) 16     -> -4
      T2: before, c counts 4; after, x (r0 pending) 16                -> -12
    so T0 (x, r0), then T2 (r2): Tree order [6, 4, 5, 7].  Its memory:
      r1 brings c, d: 12 live, 12 after;  x brings a, b: 12 + 3 + 16 = 31 live,
      a, b, c released -> 24;  r0: d released -> 16;  r2: x released -> 0.
    Input order [4, 5, 6, 7]: x brings a, b, c (23 live, 20 after: c, x);
      r0 brings d (28, nothing released: d feeds r1, x feeds r2); r1 -> 16; r2 -> 0."""
    d = _hand_general()
    assert d.tree_roots == [5, 6, 7]
    assert d.parents[2] == [4, 6] and d.parents[3] == [5, 6] and d.parents[4] == [5, 7]
    st = S._TreeState(d, [d.size(u) for u in range(d.n_nodes)])
    assert [st.gain(i) for i in range(3)] == [-28, -12, -20]
    assert S.tree(d) == [6, 4, 5, 7]
    assert S.input_order(d) == [4, 5, 6, 7]
    t = S.memsim(d, [6, 4, 5, 7])
    assert (t["M"], t["peak_post"], t["peak_live"]) == ([12, 24, 16, 0], 24, 31)
    i = S.memsim(d, [4, 5, 6, 7])
    assert (i["M"], i["peak_post"], i["peak_live"]) == ([20, 28, 16, 0], 28, 28)
    # brute force over the 12 topological orders: 20 (e.g. x, r2, r1, r0)
    assert S.optimal_peak(d) == 20
    with pytest.raises(ValueError):
        S.sibling(d)                                           # x has three children


def test_general_binary_reduces_to_build():
    """A binary DAG given as a general DAG (its own node sizes) schedules and
    simulates exactly like the contraction DAG it came from."""
    for seed in range(6):
        d = random_mixed(seed) if seed % 2 else random_ring(seed)
        g = D.general(d.n_leaves, [d.size(u) for u in range(d.n_nodes)],
                      [d.children(u) for u in range(d.n_nodes)])
        assert g.tree_roots == d.tree_roots                    # first appearance = ascending id
        for pol in ("input", "sibling", "tree"):
            a, b = S.schedule(d, pol), S.schedule(g, pol)
            assert a == b, (seed, pol)
            assert S.memsim(d, a) == S.memsim(g, b)


@pytest.mark.parametrize("seed", range(12))
def test_general_tree_gain_is_memory_difference(seed):
    """On general DAGs too, the chosen tree's gain equals the drop in resident
    bytes measured by direct set reasoning, and the order is valid."""
    from synth.general import random_general
    nl, sz, ch = random_general(seed, n_leaves=5 + seed % 4, n_trees=3 + seed % 5,
                                max_arity=1 + seed % 4, share=(0.0, 0.3, 0.6)[seed % 3])
    d = D.general(nl, sz, ch)
    st = S._TreeState(d, [d.size(u) for u in range(d.n_nodes)])
    order = []
    alive = set(range(len(d.tree_roots)))
    while alive:
        gains = {i: st.gain(i) for i in alive}
        best = max(sorted(alive), key=lambda i: gains[i])
        before = _mem_after(d, order)
        order += [u for u in st.process(best) if d.kind[u] >= 0]
        assert gains[best] == before - _mem_after(d, order)
        alive.discard(best)
    assert order == S.tree(d) == S.tree(d, recompute_all=True)
    assert sorted(order) == sorted(d.contractions())
    sim = S.memsim(d, order)
    assert sim["M"][-1] == 0 and sim["peak_post"] <= sim["peak_live"]
    if len(d.contractions()) <= 7:
        assert S.optimal_peak(d) <= sim["peak_post"]


def test_general_validation():
    ok = ([1, 1, 1], [(), (), (0, 1)])
    D.general(2, *ok)
    for nl, sizes, kids in [
        (2, [1, 1, 1], [(), (), ()]),            # non-leaf without children
        (2, [1, 1, 1], [(), (0,), (0, 1)]),      # leaf with a child
        (2, [1, 1, 1], [(), (), (0, 0)]),        # repeated child
        (2, [1, 1, 1], [(), (), (0, 2)]),        # self reference
        (2, [1, 1, -1], [(), (), (0, 1)]),       # negative size
        (3, [1, 1], [(), ()]),                   # more leaves than nodes
    ]:
        with pytest.raises(D.InvalidGraph):
            D.general(nl, sizes, kids)


# ---------------------------------------------------------------- node-based gain scheduler
def test_node_gain_hand_examples():
    """Worked by hand: gain(v) = released - brought - output under Sec. II-C.

    Fig. 1 (leaves 256 B, e 256 B, roots 0): f and e both start at -512 (f brings
    a, b; e brings b, c, adds e and releases c), the tie goes to f (id 4); then e
    is the only ready node (releases b, c, brings c: 0); then g releases a (+256)
    against h (brings and releases d: 0).  Order f, e, g, h; M 512, 512, 256, 0.

    Leaves p, q, r (ids 0-2, sizes 4, 2, 1); x = (p, q) size 5 (id 3);
    y = (q, r) size 1 (id 4); roots s = (x) (id 5) and t = (y, p) (id 6).
      step 1: x: -6 - 5 = -11;  y: -3 - 1 + 1 (r) = -3            -> y, M 3
      step 2: x: -4 - 5 + 2 (q) = -7;  t: -4 + 1 (y) = -3          -> t, M 6
      step 3: x: -5 + 4 + 2 = +1                                   -> x, M 5
      step 4: s releases x                                         -> s, M 0
    Input order (x, s, y, t) peaks at 11 (x brings p, q and adds x); Tree
    takes the same order; the brute-force optimum is 6, which node gain meets."""
    d, names = fig1()
    order = S.node_gain(d)
    assert order == [names[x] for x in "fegh"]
    assert S.memsim(d, order)["M"] == [512, 512, 256, 0]

    g = D.general(3, [4, 2, 1, 5, 1, 0, 0], [(), (), (), (0, 1), (1, 2), (3,), (4, 0)])
    assert S.node_gain(g) == [4, 6, 3, 5]
    assert S.memsim(g, [4, 6, 3, 5])["M"] == [3, 6, 5, 0]
    assert S.input_order(g) == S.tree(g) == [3, 5, 4, 6]
    assert S.memsim(g, [3, 5, 4, 6])["peak_post"] == 11
    assert S.optimal_peak(g) == 6

    h = _hand_general()
    assert S.node_gain(h) == [6, 4, 5, 7]


def test_node_gain_chain_has_one_order():
    """A chain of contractions has a single topological order."""
    n = 6
    kids = [()] * (n + 1) + [(0, 1)] + [(n + 1 + k, k + 2) for k in range(n - 1)]
    sizes = [1] * (n + 1) + [3] * (n - 1) + [0]
    d = D.general(n + 1, sizes, kids)
    assert S.node_gain(d) == list(range(n + 1, 2 * n + 1))


def _check_node_picks(d, order):
    done = []
    for v in order:
        ready = [u for u in d.contractions() if u not in done
                 and all(d.kind[x] < 0 or x in done for x in d.children(u))]
        before = _mem_after(d, done)
        drop = {u: before - _mem_after(d, done + [u]) for u in ready}
        best = max(drop.values())
        assert v == min(u for u in ready if drop[u] == best)
        done.append(v)


@pytest.mark.parametrize("seed", range(24))
def test_node_gain_picks_the_largest_drop(seed):
    """Every pick of node_gain is the ready contraction whose run lowers the
    resident bytes most, measured by direct set reasoning; ties to the lowest id."""
    if seed < 12:
        d = random_ring(seed, n_leaves=7, n_graphs=10) if seed % 2 else random_mixed(seed)
    else:
        from synth.general import random_general
        nl, sz, ch = random_general(seed, n_leaves=5 + seed % 4, n_trees=3 + seed % 5,
                                    max_arity=1 + seed % 4, share=(0.0, 0.3, 0.6)[seed % 3])
        d = D.general(nl, sz, ch)
    order = S.node_gain(d)
    assert sorted(order) == sorted(d.contractions())
    _check_node_picks(d, order)
