"""Contraction DAG formation (Sec. II-B, "Notation"), and general DAGs whose
nodes have any number of children (for scheduling only).

Each input graph is a binary contraction tree.  Structurally identical
contractions (same kind, same ordered children) are one DAG node, so trees
share nodes but never roots unless the whole graph is identical; identical
graphs share their root (the tree list then holds that root once).

Node ids: leaves 0..L-1 in input order, then each new contraction in order of
first appearance while graphs are scanned in order, op by op.
parents(u) has one entry per edge, in the order edges are created.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Tuple

LEAF, INTERIOR, ROOT = "LEAF", "INTERIOR", "ROOT"
K22, K32, K33, HCA = 0, 1, 2, 3
# General contractions of the last c axes of the left operand with the first c
# axes of the right one (c = 1, 2, 3), for operand and output ranks 2..4.
C1, C2, C3 = 4, 5, 6
SPEC_BASE = 16   # kind SPEC_BASE + i: the contraction spec i (any index pairs, output order)
MIN_RANK, MAX_RANK = 2, 4

# (left rank, right rank) -> output rank, per named kind; HCA outputs a scalar per t.
_RANKS = {K22: ((2, 2), 2), K32: ((3, 2), 3), K33: ((3, 3), 2), HCA: ((2, 2), 0)}
# The named kinds are the general contractions with these (left rank, right rank, c).
_NAMED = {(2, 2, 1): K22, (3, 2, 1): K32, (3, 3, 2): K33}


def contracted_axes(kind: int) -> int:
    """c of a (named or general) exterior contraction."""
    return {K22: 1, K32: 1, K33: 2, C1: 1, C2: 2, C3: 3}[kind]


def normalize(kind: int, rl: int, rr: int):
    """(kind, output rank) of an exterior contraction of operands of ranks rl, rr:
    a general kind that equals a named one becomes the named kind.  Raises
    InvalidGraph when the ranks do not fit the kind."""
    if kind in (C1, C2, C3):
        c = contracted_axes(kind)
        ro = rl + rr - 2 * c
        if not (MIN_RANK <= rl <= MAX_RANK and MIN_RANK <= rr <= MAX_RANK and MIN_RANK <= ro <= MAX_RANK):
            raise InvalidGraph("operand or output rank out of range")
        return _NAMED.get((rl, rr, c), kind), ro
    (el, er), ro = _RANKS[kind]
    if (rl, rr) != (el, er):
        raise InvalidGraph("operand rank mismatch")
    return kind, ro


class InvalidGraph(ValueError):
    pass


def normalize_spec(spec, rl: int, rr: int):
    """(c, output rank, canonical) of a contraction spec applied to operands of
    ranks rl, rr.  canonical: the spec sums the last c axes of X against the
    first c of Y in order and keeps the natural output order, i.e. it is C_c.
    Raises InvalidGraph for a spec that does not fit the operands or is
    malformed (repeated axes, a perm that is not a permutation)."""
    if (spec.rank_l, spec.rank_r) != (rl, rr):
        raise InvalidGraph("operand ranks differ from the spec's")
    c = len(spec.pairs)
    ro = rl + rr - 2 * c
    if not (1 <= c <= 3 and MIN_RANK <= rl <= MAX_RANK and MIN_RANK <= rr <= MAX_RANK
            and MIN_RANK <= ro <= MAX_RANK):
        raise InvalidGraph("spec ranks out of range")
    xa = [a for a, _ in spec.pairs]
    yb = [b for _, b in spec.pairs]
    if len(set(xa)) != c or len(set(yb)) != c or not all(0 <= a < rl for a in xa) \
            or not all(0 <= b < rr for b in yb):
        raise InvalidGraph("spec axes out of range or repeated")
    if sorted(spec.perm) != list(range(ro)):
        raise InvalidGraph("spec perm is not a permutation of the output axes")
    canonical = xa == list(range(rl - c, rl)) and yb == list(range(c)) and list(spec.perm) == list(range(ro))
    return c, ro, canonical


@dataclass
class Dag:
    n_leaves: int
    kind: List[int] = field(default_factory=list)      # -1 for leaves
    left: List[int] = field(default_factory=list)      # -1 for leaves
    right: List[int] = field(default_factory=list)
    rank: List[int] = field(default_factory=list)
    nvec: List[int] = field(default_factory=list)
    nt: List[int] = field(default_factory=list)
    parents: List[List[int]] = field(default_factory=list)
    root_of_graph: List[int] = field(default_factory=list)
    tree_roots: List[int] = field(default_factory=list)   # unique roots, first-appearance order

    @property
    def n_nodes(self) -> int:
        return len(self.kind)

    def children(self, u: int) -> Tuple[int, ...]:
        return () if self.kind[u] < 0 else (self.left[u], self.right[u])

    def node_type(self, u: int) -> str:
        if self.kind[u] < 0:
            return LEAF
        return ROOT if not self.parents[u] else INTERIOR

    def contractions(self) -> List[int]:
        return [u for u in range(self.n_nodes) if self.kind[u] >= 0]

    def elems(self, u: int) -> int:
        """Complex elements of the tensor of u: Nt * N^rank (0 for a root's scalar output
        is handled by size())."""
        return self.nt[u] * self.nvec[u] ** self.rank[u]

    def size(self, u: int, elem_bytes: int = 16) -> int:
        """u.size in bytes of the device dtype; a root's output is a per-t scalar written
        straight to the correlator buffer and counts 0 (reading of Sec. II-C)."""
        if self.kind[u] == HCA:
            return 0
        return self.elems(u) * elem_bytes

    def tree_nodes(self, i: int) -> List[int]:
        """Node set of tree T_i: the root and all its descendants (post-order, left first)."""
        out, seen = [], set()

        def visit(u):
            if u in seen:
                return
            seen.add(u)
            for c in self.children(u):
                visit(c)
            out.append(u)

        visit(self.tree_roots[i])
        return out


def build(leaves, graphs, specs=()) -> Dag:
    """Merge the graphs into one DAG by hash-consing (kind, left, right).

    `leaves`: sequence of objects with .rank .nvec .nt; `graphs`: sequence with
    .ops = [(kind, left, right), ...]; `specs`: the contraction specs that op
    kinds SPEC_BASE + i name.  A spec equal to C1, C2 or C3 on its operands is
    stored as that kind (and so as K22, K32 or K33 where those apply), so it
    merges with them.  Raises InvalidGraph for malformed input.
    """
    d = Dag(n_leaves=len(leaves))
    for lf in leaves:
        if not MIN_RANK <= lf.rank <= MAX_RANK or lf.nvec < 1 or lf.nt < 1:
            raise InvalidGraph("bad leaf shape")
        d.kind.append(-1)
        d.left.append(-1)
        d.right.append(-1)
        d.rank.append(lf.rank)
        d.nvec.append(lf.nvec)
        d.nt.append(lf.nt)
        d.parents.append([])
    table: Dict[Tuple[int, int, int], int] = {}
    roots_seen = set()
    for gi, g in enumerate(graphs):
        ops = list(g.ops)
        if not ops:
            raise InvalidGraph("empty graph")
        local: List[int] = []
        consumed = [0] * len(ops)
        for oi, (kind, l, r) in enumerate(ops):
            if kind not in _RANKS and kind not in (C1, C2, C3) and not SPEC_BASE <= kind < SPEC_BASE + len(specs):
                raise InvalidGraph("bad kind")
            if (kind == HCA) != (oi == len(ops) - 1):
                raise InvalidGraph("the root, and only the root, must be a trace")
            ids = []
            for x in (l, r):
                if x >= 0:
                    if x >= len(leaves):
                        raise InvalidGraph("leaf id out of range")
                    ids.append(x)
                else:
                    j = -x - 1
                    if j >= oi:
                        raise InvalidGraph("forward or self reference")
                    consumed[j] += 1
                    ids.append(local[j])
            lid, rid = ids
            if lid == rid:
                raise InvalidGraph("identical operands")
            if kind >= SPEC_BASE:
                c, ro, canonical = normalize_spec(specs[kind - SPEC_BASE], d.rank[lid], d.rank[rid])
                if canonical:
                    kind, ro = normalize((C1, C2, C3)[c - 1], d.rank[lid], d.rank[rid])
            else:
                kind, ro = normalize(kind, d.rank[lid], d.rank[rid])
            if d.nvec[lid] != d.nvec[rid] or d.nt[lid] != d.nt[rid]:
                raise InvalidGraph("operand N or Nt mismatch")
            key = (kind, lid, rid)
            u = table.get(key)
            if u is None:
                u = len(d.kind)
                table[key] = u
                d.kind.append(kind)
                d.left.append(lid)
                d.right.append(rid)
                d.rank.append(ro)
                d.nvec.append(d.nvec[lid])
                d.nt.append(d.nt[lid])
                d.parents.append([])
                d.parents[lid].append(u)
                d.parents[rid].append(u)
            local.append(u)
        if any(c != 1 for c in consumed[:-1]):
            raise InvalidGraph("every non-root op must be used exactly once in its graph")
        root = local[-1]
        d.root_of_graph.append(root)
        if root not in roots_seen:
            roots_seen.add(root)
            d.tree_roots.append(root)
    return d


NARY = 7   # a node of a general DAG


@dataclass
class GeneralDag(Dag):
    """A DAG whose nodes may have any number of children, with sizes given per node
    in bytes.  Sec. II-B remarks that the schedulers extend to nodes with any number
    of children, and Sec. III-B that the Tree scheduler needs neither two children
    per node nor trees that are trees.  Only scheduling and the memory model apply:
    there are no tensor shapes."""
    kids: List[Tuple[int, ...]] = field(default_factory=list)
    sizes: List[int] = field(default_factory=list)

    def children(self, u: int) -> Tuple[int, ...]:
        return self.kids[u]

    def size(self, u: int, elem_bytes: int = 16) -> int:
        return self.sizes[u]


def general(n_leaves: int, sizes, children) -> GeneralDag:
    """Nodes 0..n_leaves-1 are leaves; node u lists its children (operand order,
    ids below u, no repeats, at least one for a non-leaf).  Trees are rooted at the
    non-leaf nodes without parents, in ascending id; parents(u) has one entry per
    edge, node by node and children in order.  Raises InvalidGraph on bad input."""
    n = len(sizes)
    if len(children) != n or not 0 <= n_leaves <= n:
        raise InvalidGraph("counts")
    d = GeneralDag(n_leaves=n_leaves)
    for u in range(n):
        kids = tuple(int(x) for x in children[u])
        if sizes[u] < 0:
            raise InvalidGraph("negative size")
        if u < n_leaves and kids:
            raise InvalidGraph("a leaf has no children")
        if u >= n_leaves and not kids:
            raise InvalidGraph("a non-leaf node needs a child")
        if any(not 0 <= x < u for x in kids) or len(set(kids)) != len(kids):
            raise InvalidGraph("child ids must be distinct and below the node")
        d.kids.append(kids)
        d.sizes.append(int(sizes[u]))
        d.kind.append(-1 if u < n_leaves else NARY)
        d.left.append(kids[0] if len(kids) == 2 else -1)
        d.right.append(kids[1] if len(kids) == 2 else -1)
        d.rank.append(0)
        d.nvec.append(0)
        d.nt.append(0)
        d.parents.append([])
        for x in kids:
            d.parents[x].append(u)
    d.tree_roots = [u for u in range(n_leaves, n) if not d.parents[u]]
    d.root_of_graph = list(d.tree_roots)
    return d


def stats(d: Dag) -> dict:
    """|V|, |E|, F_v and F_e as defined in the Tree runtime analysis (Sec. III-B)."""
    trees = [set(d.tree_nodes(i)) for i in range(len(d.tree_roots))]
    ctree = [0] * d.n_nodes
    for t in trees:
        for u in t:
            ctree[u] += 1
    edges = [(c, u) for u in range(d.n_nodes) for c in d.children(u)]
    fe = sum(sum(1 for t in trees if c in t and u in t) for c, u in edges)
    return dict(n_nodes=d.n_nodes, n_edges=len(edges), n_trees=len(trees),
                f_v=sum(ctree) / max(1, d.n_nodes), f_e=fe / max(1, len(edges)))
