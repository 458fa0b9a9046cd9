"""Budgeted execution plan: wave cut, next-use eviction, uploads and releases.

The paper's schedulers fix the contraction order; evictions then happen when a
contraction does not fit in device memory (Sec. IV-C: an eviction happens when
a contraction is to run but memory is short; the metrics are evictions,
transfers and transfer bytes).  The paper's own memory manager is not
specified, so the policy here is the plan this engine defines:

Steps.  Per-contraction mode: one step per contraction in schedule order.
Batched mode: waves of ready contractions taken in schedule order (cut_waves);
with lookahead 0 the order is kept exactly and a wave is closed before
contraction c if (a) an operand of c is produced in the wave, (b) the bytes of
the wave's distinct operands and outputs with c added would exceed the budget,
or (c) the wave already holds wave_max contractions.

Per step s:
  need = bytes of the step's non-resident operands + its outputs.
  While used + need > budget: evict the resident tensor that is not an operand of
  s with the furthest next use (ties: larger size, then smaller id).  A leaf or
  an intermediate with a valid host copy is dropped; any other intermediate is
  copied to the host once (D2H).  Every eviction counts once.  If nothing is
  left to evict the plan fails (BudgetError).
  Upload non-resident operands (H2D, ascending id; first touches count),
  allocate outputs (a root's output is 0 bytes and is never resident), run the
  contractions, then free every operand nothing later needs (ascending id),
  with its host copy.

leaves_resident=True models leaves kept permanently in a device region outside
the budget: they are never uploaded, evicted or counted.

t_chunks = C > 1 runs the DAG as C passes, each over nt / C time slices of
every tensor (every contraction and trace acts on each slice on its own).
Passes alternate between two halves of the budget, so one pass is planned as
above with every size divided by C and budget // 2; the execution's counters
are C times the pass's, its steps C times as many, and its resident peak twice
the pass's (both halves in use).  The op records are those of one pass.

Op records: (op, node, step) with op in D2H, DROP, H2D, ALLOC, EXEC, FREE.
"""
from __future__ import annotations

from typing import List, Sequence

from .dag import Dag, HCA

UNLIMITED = (1 << 64) - 1
WAVE_MAX = 4096


class BudgetError(RuntimeError):
    pass


def cut_waves(d: Dag, order: Sequence[int], size: Sequence[int], budget: int,
              wave_max: int = WAVE_MAX, lookahead: int = 0) -> List[List[int]]:
    """Waves in schedule order.  A contraction is ready when every operand is a leaf
    or was produced by an earlier wave.  Scanning the not yet placed contractions
    in order, a wave takes each ready one and passes over at most `lookahead`
    that are not ready; it closes at the next not-ready one after that, or when
    adding a contraction would make its distinct operands and outputs exceed the
    budget, or when it holds wave_max contractions.  lookahead = 0 keeps the
    order exactly (a wave ends where a contraction needs one of its outputs)."""
    n = len(order)
    placed = [False] * n
    produced = set()
    waves = []
    start = 0
    while start < n:
        wave, members, mbytes, skipped = [], set(), 0, 0
        for pos in range(start, n):
            if placed[pos]:
                continue
            c = order[pos]
            ops = d.children(c)
            if not all(d.kind[x] < 0 or x in produced for x in ops):
                skipped += 1
                if skipped > lookahead:
                    break
                continue
            new = {x for x in set(ops) | {c} if x not in members}
            extra = sum(size[x] for x in new)
            if wave and (mbytes + extra > budget or len(wave) >= wave_max):
                break
            wave.append(c)
            placed[pos] = True
            members |= new
            mbytes += extra
        produced.update(wave)
        waves.append(wave)
        while start < n and placed[start]:
            start += 1
    return waves


def plan(d: Dag, order: Sequence[int], elem_bytes: int = 16, budget: int = UNLIMITED,
         batched: bool = False, wave_max: int = WAVE_MAX, leaves_resident: bool = False,
         lookahead: int = 0, t_chunks: int = 1) -> dict:
    if t_chunks > 1:
        if any(d.nt[u] % t_chunks for u in range(d.n_nodes)):
            raise ValueError("t_chunks must divide every tensor's nt")
        one = _plan(d, order, elem_bytes, min(budget, UNLIMITED) // 2, batched, wave_max,
                    leaves_resident, lookahead, t_chunks)
        out = {k: (t_chunks * v if k in ("n_steps", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes")
                   else v) for k, v in one.items()}
        out["peak_resident"] = 2 * one["peak_resident"]
        return out
    return _plan(d, order, elem_bytes, budget, batched, wave_max, leaves_resident, lookahead, 1)


def _plan(d: Dag, order: Sequence[int], elem_bytes: int, budget: int, batched: bool, wave_max: int,
          leaves_resident: bool, lookahead: int, t_chunks: int) -> dict:
    n = d.n_nodes
    size = [d.size(u, elem_bytes) // t_chunks for u in range(n)]
    if leaves_resident:
        for u in range(d.n_leaves):
            size[u] = 0
    steps = (cut_waves(d, order, size, budget, wave_max, lookahead) if batched
             else [[c] for c in order])

    uses: List[List[int]] = [[] for _ in range(n)]
    for s, wave in enumerate(steps):
        for c in wave:
            for x in d.children(c):
                if not uses[x] or uses[x][-1] != s:
                    uses[x].append(s)
    remaining = [len(d.parents[u]) for u in range(n)]
    ptr = [0] * n

    def next_use(x, s):
        u = uses[x]
        while ptr[x] < len(u) and u[ptr[x]] <= s:
            ptr[x] += 1
        return u[ptr[x]]

    resident = set(range(d.n_leaves)) if leaves_resident else set()
    host_copy = set()
    used = 0
    ops = []
    c = dict(n_steps=len(steps), peak_resident=0, n_evict=0, n_h2d=0, h2d_bytes=0,
             n_d2h=0, d2h_bytes=0)
    for s, wave in enumerate(steps):
        operands = sorted({x for cc in wave for x in d.children(cc)})
        pinned = set(operands)
        need = sum(size[x] for x in operands if x not in resident)
        need += sum(size[cc] for cc in wave)
        while used + need > budget:
            cands = [x for x in resident if x not in pinned
                     and not (leaves_resident and x < d.n_leaves)]
            if not cands:
                raise BudgetError(f"step {s} does not fit in {budget} bytes")
            victim = max(cands, key=lambda x: (next_use(x, s), size[x], -x))
            if d.kind[victim] < 0 or victim in host_copy:
                ops.append(("DROP", victim, s))
            else:
                ops.append(("D2H", victim, s))
                c["n_d2h"] += 1
                c["d2h_bytes"] += size[victim]
                host_copy.add(victim)
            c["n_evict"] += 1
            resident.discard(victim)
            used -= size[victim]
        for x in operands:
            if x not in resident:
                assert d.kind[x] < 0 or x in host_copy, "intermediate lost"
                ops.append(("H2D", x, s))
                c["n_h2d"] += 1
                c["h2d_bytes"] += size[x]
                resident.add(x)
                used += size[x]
        for cc in wave:
            if d.kind[cc] != HCA:
                ops.append(("ALLOC", cc, s))
                resident.add(cc)
                used += size[cc]
        c["peak_resident"] = max(c["peak_resident"], used)
        for cc in wave:
            ops.append(("EXEC", cc, s))
        for cc in wave:
            for x in d.children(cc):
                remaining[x] -= 1
        for x in operands:
            if remaining[x] == 0 and x in resident and not (leaves_resident and x < d.n_leaves):
                ops.append(("FREE", x, s))
                resident.discard(x)
                host_copy.discard(x)
                used -= size[x]
    c["ops"] = ops
    c["steps"] = steps
    return c
