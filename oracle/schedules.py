"""Contraction orders and the memory model (Sec. II-C and Sec. III).

input_order  graphs in input order, each root's subtree in post-order, children
             in operand order (left first), each contraction emitted once (the
             plain baseline).
sibling      the Sibling scheduler, Algs. 1-3 (SB-SCHEDULER, SB-PROCESS,
             SB-PROP-DOWN), Eq. (1) for ranks.
tree         the Tree scheduler written from its definition: repeatedly pick the
             unprocessed tree whose processing changes memory by the largest gain
             M - M' (Sec. III-B), then process its unprocessed nodes in
             topological order, left to right.
node_gain    a node-based gain scheduler, the one the conclusions name as future
             work: repeatedly run the ready contraction whose execution changes
             memory by the largest gain M - M' (the Tree scheduler's gain concept,
             Sec. III-B, taken to single nodes), M and M' measured by memsim.
memsim       the memory model of Sec. II-C: M_i after each contraction, plus the
             live peak during a contraction (inputs, newly brought leaves and the
             output coexist).
optimal_peak brute force over all topological orders (tiny DAGs only).

Readings where the paper is silent (same list as the design notes):
  * Sibling's "random" leaf is the WAITING leaf with the smallest id; queues are
    FIFO; PROP-DOWN visits the left child before the right; the sibling of u
    under parent v is v's other child.
  * Tree ties go to the lowest tree index; trees are indexed by unique root in
    order of first appearance.
  * A leaf costs memory from its first use by a contraction; a root's output
    costs 0.
  * node_gain: a contraction is ready when every non-leaf child has run (leaves
    are always available); ties go to the lowest node id.
"""
from __future__ import annotations

import sys
from collections import deque
from typing import Dict, List, Sequence, Set

from .dag import Dag

sys.setrecursionlimit(100000)


# ---------------------------------------------------------------- input order
def input_order(d: Dag) -> List[int]:
    done: Set[int] = set()
    order: List[int] = []

    def visit(u):
        if u in done or d.kind[u] < 0:
            return
        for c in d.children(u):
            visit(c)
        done.add(u)
        order.append(u)

    for r in d.root_of_graph:
        visit(r)
    return order


# ---------------------------------------------------------------- Sibling (Algs 1-3)
WAITING, QUEUED, INMEM, RELEASED = "WAITING", "QUEUED", "INMEM", "RELEASED"


def ranks(d: Dag) -> List[int]:
    """Eq. (1): rank 0 for leaves, else 1 + the largest child rank."""
    rk = [0] * d.n_nodes
    for u in range(d.n_nodes):   # ids are topological: children precede parents
        if d.kind[u] >= 0:
            rk[u] = 1 + max(rk[c] for c in d.children(u))
    return rk


def sibling(d: Dag) -> List[int]:
    """Algs. 1-3; the sibling of a node is its parent's other child, so every
    contraction must have exactly two children (ValueError otherwise)."""
    if any(len(d.children(u)) != 2 for u in d.contractions()):
        raise ValueError("sibling: every contraction needs two children")
    rank = ranks(d)
    rs = [len(d.parents[u]) for u in range(d.n_nodes)]
    rp = [len(d.children(u)) for u in range(d.n_nodes)]
    state = [WAITING] * d.n_nodes
    queues: Dict[int, deque] = {i: deque() for i in range(1, max(rank, default=0) + 1)}
    n_contr = len(d.contractions())
    order: List[int] = []

    def process(u):                                   # SB-PROCESS
        if d.kind[u] >= 0:
            order.append(u)                           # perform the contraction
        state[u] = INMEM
        if d.kind[u] >= 0:
            for v in d.children(u):                   # releasable inputs
                rs[v] -= 1
                if rs[v] == 0:
                    state[v] = RELEASED
            if not d.parents[u]:                      # a ROOT is released at once
                state[u] = RELEASED
        for v in d.parents[u]:                        # siblings, or enqueue parents
            rp[v] -= 1
            if rp[v] == 1:
                w = d.right[v] if d.left[v] == u else d.left[v]
                if state[w] == WAITING:
                    prop_down(w)
            elif rp[v] == 0:
                queues[rank[v]].append(v)
                state[v] = QUEUED

    def prop_down(u):                                 # SB-PROP-DOWN
        if state[u] != WAITING:
            return
        if d.kind[u] < 0:
            process(u)
            return
        prop_down(d.left[u])
        prop_down(d.right[u])

    while len(order) < n_contr:                       # SB-SCHEDULER
        nonempty = [i for i in queues if queues[i]]
        if not nonempty:
            u = min(x for x in range(d.n_leaves) if state[x] == WAITING)
        else:
            u = queues[max(nonempty)].popleft()
        process(u)
    return order


# ---------------------------------------------------------------- Tree (by definition)
class _TreeState:
    """Processed-node bookkeeping for the Tree scheduler's gain M - M'."""

    def __init__(self, d: Dag, sizes: Sequence[int]):
        self.d = d
        self.sizes = sizes
        self.processed = [False] * d.n_nodes
        self.trees = [d.tree_nodes(i) for i in range(len(d.tree_roots))]
        self.tree_sets = [set(t) for t in self.trees]

    def in_mem(self, x, processed) -> bool:
        """Sec. II-C: a tensor stays in memory while some contraction using it is pending."""
        return processed(x) and any(not processed(p) for p in self.d.parents[x])

    def gain(self, i: int) -> int:
        """M - M' for processing the unprocessed nodes of T_i (no temporaries).

        Only nodes of T_i and their children can change state, so M - M' is summed
        over those; every other node's memory state is unaffected."""
        d, proc = self.d, self.processed
        todo = {u for u in self.trees[i] if not proc[u]}
        touched = set(todo)
        for u in todo:
            touched.update(d.children(u))
        before = (lambda x: proc[x])
        after = (lambda x: proc[x] or x in todo)
        m_before = sum(self.sizes[x] for x in touched if self.in_mem(x, before))
        m_after = sum(self.sizes[x] for x in touched if self.in_mem(x, after))
        return m_before - m_after

    def process(self, i: int) -> List[int]:
        """Process T_i's unprocessed nodes in post-order, left first; return the
        contractions performed, in order."""
        d, out = self.d, []

        def visit(u):
            if self.processed[u]:
                return
            for c in d.children(u):
                visit(c)
            self.processed[u] = True
            out.append(u)

        visit(d.tree_roots[i])
        return out


def tree(d: Dag, elem_bytes: int = 16, recompute_all: bool = False) -> List[int]:
    """Tree scheduler: argmax gain over unprocessed trees (lowest index on ties).

    Gains are cached and refreshed for every tree that contains a node whose
    state, or whose parents' state, changed; recompute_all=True refreshes all
    gains every iteration (used by the tests to check the cache)."""
    sizes = [d.size(u, elem_bytes) for u in range(d.n_nodes)]
    st = _TreeState(d, sizes)
    k = len(st.trees)
    ctree: List[List[int]] = [[] for _ in range(d.n_nodes)]
    for i, t in enumerate(st.trees):
        for u in t:
            ctree[u].append(i)
    gains = [st.gain(i) for i in range(k)]
    alive = [True] * k
    order: List[int] = []
    for _ in range(k):
        best = None
        for i in range(k):
            if alive[i] and (best is None or gains[i] > gains[best]):
                best = i
        alive[best] = False
        changed = st.process(best)
        order.extend(u for u in changed if d.kind[u] >= 0)
        if recompute_all:
            dirty = range(k)
        else:
            hit = set(changed)
            for u in changed:
                hit.update(d.children(u))
            dirty = sorted({i for x in hit for i in ctree[x]})
        for i in dirty:
            if alive[i]:
                gains[i] = st.gain(i)
    return order


def tree_initial_igains(d: Dag, elem_bytes: int = 16) -> List[Dict[int, int]]:
    """igain(u, T_i) at initialisation: -u.size if u has a parent outside T_i, else 0
    (TR-INIT, as the text describes it)."""
    out = []
    for i in range(len(d.tree_roots)):
        nodes = set(d.tree_nodes(i))
        out.append({u: (-d.size(u, elem_bytes) if any(p not in nodes for p in d.parents[u]) else 0)
                    for u in nodes})
    return out


# ---------------------------------------------------------------- memory model
def memsim(d: Dag, order: Sequence[int], elem_bytes: int = 16, partial: bool = False) -> dict:
    """Sec. II-C: for each contraction c_i, (i) bring leaves c_i needs, (ii) perform it,
    (iii) release every tensor nothing pending depends on (the output of a root too).

    Returns M = [M_1..M_n], peak_post = max M_i, peak_live = the largest
    resident total while a contraction runs (M_{i-1} + first-touch leaves +
    output), and the memory contents after each contraction.  With partial,
    the order may be a topological prefix of a complete one."""
    size = [d.size(u, elem_bytes) for u in range(d.n_nodes)]
    remaining = [len(d.parents[u]) for u in range(d.n_nodes)]
    in_mem: Set[int] = set()
    M, Ms, peak_live, contents = 0, [], 0, []
    seen = set()
    for c in order:
        if d.kind[c] < 0 or c in seen:
            raise ValueError("order must list each contraction once")
        seen.add(c)
        brought = 0
        for x in d.children(c):
            if x not in in_mem:
                if d.kind[x] >= 0:
                    raise ValueError("order is not topological")
                in_mem.add(x)
                brought += size[x]
        peak_live = max(peak_live, M + brought + size[c])
        M += brought + size[c]
        in_mem.add(c)
        for x in d.children(c):
            remaining[x] -= 1
            if remaining[x] == 0:
                in_mem.discard(x)
                M -= size[x]
        if remaining[c] == 0:
            in_mem.discard(c)
            M -= size[c]
        Ms.append(M)
        contents.append(sorted(in_mem))
    if not partial and len(seen) != len(d.contractions()):
        raise ValueError("order must cover every contraction")
    return dict(M=Ms, peak_post=max(Ms) if Ms else 0, peak_live=peak_live, contents=contents)


def node_gain(d: Dag, elem_bytes: int = 16) -> List[int]:
    """Node-based gain scheduler, from its definition: with the prefix P run so
    far (memory M after it, by memsim), run next the ready contraction v whose
    M' (memory after P + [v], by memsim) is smallest, i.e. whose gain M - M' is
    largest; ties to the lowest id.  Quadratic in memsim calls: small DAGs."""
    contr = d.contractions()
    done: Set[int] = set()
    order: List[int] = []
    M = 0
    while len(order) < len(contr):
        best, best_gain, best_M = None, None, None
        for v in contr:
            if v in done or any(d.kind[x] >= 0 and x not in done for x in d.children(v)):
                continue
            Mv = memsim(d, order + [v], elem_bytes, partial=True)["M"][-1]
            if best is None or M - Mv > best_gain:
                best, best_gain, best_M = v, M - Mv, Mv
        order.append(best)
        done.add(best)
        M = best_M
    return order


def topo_orders(d: Dag):
    """All topological orders of the contractions (tiny DAGs only)."""
    contr = d.contractions()
    deps = {c: {x for x in d.children(c) if d.kind[x] >= 0} for c in contr}

    def rec(done, prefix):
        if len(prefix) == len(contr):
            yield list(prefix)
            return
        for c in contr:
            if c not in done and deps[c] <= done:
                done.add(c)
                prefix.append(c)
                yield from rec(done, prefix)
                prefix.pop()
                done.discard(c)

    yield from rec(set(), [])


def optimal_peak(d: Dag, elem_bytes: int = 16) -> int:
    """Minimum of peak_post over every topological order (brute force)."""
    return min(memsim(d, o, elem_bytes)["peak_post"] for o in topo_orders(d))


def schedule(d: Dag, policy: str, elem_bytes: int = 16) -> List[int]:
    if policy == "input":
        return input_order(d)
    if policy == "sibling":
        return sibling(d)
    if policy == "tree":
        return tree(d, elem_bytes)
    if policy == "node":
        return node_gain(d, elem_bytes)
    raise KeyError(policy)


__all__ = ["input_order", "sibling", "tree", "node_gain", "ranks", "memsim", "optimal_peak",
           "topo_orders", "tree_initial_igains", "schedule"]
