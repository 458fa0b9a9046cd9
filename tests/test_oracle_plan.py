"""Pins of the oracle's budgeted planner (CPU only).

  * With a budget >= peak_live there are no evictions, every leaf is uploaded
    exactly once and peak_resident equals memsim's peak_live.
  * Replaying the op list independently: every operand is resident when its
    contraction runs, resident bytes never exceed the budget, the replayed peak
    equals the reported one, and everything is freed at the end.
  * Belady's furthest-next-use rule minimises uploads for equal-size tensors:
    checked against exhaustive search over every eviction choice on tiny DAGs.
  * Waves never hold a producer and its consumer, and partition the order.
"""
import functools

import pytest

from synth import workloads as W
from oracle import dag as D
from oracle import planner as P
from oracle import schedules as S


def ring(seed, n_leaves=6, n_graphs=8, lmin=3, lmax=5):
    wl = W.meson_ring(n_leaves=n_leaves, nvec=4, nt=1, n_graphs=n_graphs, lmin=lmin,
                      lmax=lmax, seed=seed, with_data=False)
    return D.build(wl.leaves, wl.graphs)


def mix(seed, n_graphs=10):
    wl = W.baryon_mix(n_bar=3, n_mes=4, nvec=4, nt=2, n_graphs=n_graphs, seed=seed,
                      with_data=False)
    return D.build(wl.leaves, wl.graphs)


def replay(d, res, budget, elem=16, leaves_resident=False):
    size = [d.size(u, elem) for u in range(d.n_nodes)]
    if leaves_resident:
        size[:d.n_leaves] = [0] * d.n_leaves
    resident = set(range(d.n_leaves)) if leaves_resident else set()
    host = set()
    used = peak = 0
    counts = dict(n_evict=0, n_h2d=0, h2d_bytes=0, n_d2h=0, d2h_bytes=0)
    for op, x, s in res["ops"]:
        if op in ("D2H", "DROP"):
            assert x in resident
            if op == "D2H":
                assert d.kind[x] >= 0 and x not in host
                host.add(x)
                counts["n_d2h"] += 1
                counts["d2h_bytes"] += size[x]
            else:
                assert d.kind[x] < 0 or x in host
            counts["n_evict"] += 1
            resident.discard(x)
            used -= size[x]
        elif op == "H2D":
            assert x not in resident and (d.kind[x] < 0 or x in host)
            resident.add(x)
            used += size[x]
            counts["n_h2d"] += 1
            counts["h2d_bytes"] += size[x]
        elif op == "ALLOC":
            assert x not in resident
            resident.add(x)
            used += size[x]
        elif op == "EXEC":
            for c in d.children(x):
                assert c in resident, f"operand {c} of {x} not resident"
        elif op == "FREE":
            resident.discard(x)
            host.discard(x)
            used -= size[x]
        assert used <= budget
        peak = max(peak, used)
    assert used == 0 and resident == (set(range(d.n_leaves)) if leaves_resident else set())
    assert peak == res["peak_resident"]
    for k, v in counts.items():
        assert res[k] == v, k
    execs = [x for op, x, _ in res["ops"] if op == "EXEC"]
    return execs


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("policy", ["input", "sibling", "tree"])
def test_unlimited_budget(seed, policy):
    d = ring(seed) if seed % 2 else mix(seed)
    order = S.schedule(d, policy)
    res = P.plan(d, order)
    sim = S.memsim(d, order)
    assert res["n_evict"] == res["n_d2h"] == res["d2h_bytes"] == 0
    assert res["h2d_bytes"] == sum(d.size(u) for u in range(d.n_leaves))
    assert res["n_h2d"] == d.n_leaves
    assert res["peak_resident"] == sim["peak_live"]
    assert replay(d, res, P.UNLIMITED) == order
    res_r = P.plan(d, order, leaves_resident=True)
    assert res_r["n_h2d"] == 0 and res_r["n_evict"] == 0
    replay(d, res_r, P.UNLIMITED, leaves_resident=True)


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("batched", [False, True])
def test_budgeted_replay(seed, batched):
    d = ring(seed, n_leaves=7, n_graphs=10) if seed % 2 else mix(seed)
    for policy in ("input", "tree"):
        order = S.schedule(d, policy)
        live = S.memsim(d, order)["peak_live"]
        for frac in (2, 3, 4):
            budget = live // frac
            try:
                res = P.plan(d, order, budget=budget, batched=batched)
            except P.BudgetError:
                # only legal when one contraction's operands and output exceed it
                need = max(sum(d.size(x) for x in set(d.children(c))) + d.size(c)
                           for c in order)
                assert need > budget
                continue
            execs = replay(d, res, budget)
            assert execs == order
            if batched:
                flat = [c for w in res["steps"] for c in w]
                assert flat == order
                for w in res["steps"]:
                    ws = set(w)
                    assert not any(x in ws for c in w for x in d.children(c))


def _brute_min_uploads(d, order, budget):
    """Exhaustive search over eviction choices (per-contraction steps)."""
    size = [d.size(u) for u in range(d.n_nodes)]
    remaining0 = tuple(len(d.parents[u]) for u in range(d.n_nodes))

    @functools.lru_cache(maxsize=None)
    def go(s, resident, remaining):
        if s == len(order):
            return 0
        c = order[s]
        ops = set(d.children(c))
        used = sum(size[x] for x in resident)
        need = sum(size[x] for x in ops if x not in resident) + size[c]
        if used + need > budget:
            best = None
            for v in resident:
                if v in ops:
                    continue
                r = go(s, resident - {v}, remaining)
                if r is not None and (best is None or r < best):
                    best = r
            return best
        uploads = sum(1 for x in ops if x not in resident)
        res = set(resident) | ops
        if d.kind[c] != W.HCA:
            res.add(c)
        rem = list(remaining)
        for x in ops:
            rem[x] -= 1
            if rem[x] == 0:
                res.discard(x)
        r = go(s + 1, frozenset(res), tuple(rem))
        return None if r is None else r + uploads

    return go(0, frozenset(), remaining0)


@pytest.mark.parametrize("seed", range(25))
def test_belady_optimal_uploads_uniform_sizes(seed):
    d = ring(seed, n_leaves=6, n_graphs=4, lmin=3, lmax=5)
    order = S.schedule(d, "input")
    u = d.size(0)
    live = S.memsim(d, order)["peak_live"]
    for budget in range(3 * u, live, u):
        res = P.plan(d, order, budget=budget)
        assert res["n_h2d"] == _brute_min_uploads(d, order, budget)


def test_budget_error_when_one_step_does_not_fit():
    d = ring(1)
    order = S.schedule(d, "tree")
    with pytest.raises(P.BudgetError):
        P.plan(d, order, budget=2 * d.size(0))


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("lookahead", [1, 4, 1 << 62])
def test_lookahead_waves(seed, lookahead):
    d = ring(seed, n_leaves=7, n_graphs=12) if seed % 2 else mix(seed)
    order = S.schedule(d, "tree")
    live = S.memsim(d, order)["peak_live"]
    for budget in (P.UNLIMITED, live // 2):
        try:
            res = P.plan(d, order, budget=budget, batched=True, lookahead=lookahead)
        except P.BudgetError:
            continue
        execs = replay(d, res, budget)
        assert sorted(execs) == sorted(order)
        done = set()
        for w in res["steps"]:          # every operand produced by an earlier wave
            for c in w:
                assert all(d.kind[x] < 0 or x in done for x in d.children(c))
            done.update(w)
    # unlimited lookahead and budget: waves are the dependency levels
    res = P.plan(d, order, batched=True, lookahead=1 << 62)
    level = {}
    for c in order:
        level[c] = 1 + max([level.get(x, 0) for x in d.children(c)])
    assert [sorted(w) for w in res["steps"]] == [
        sorted(c for c in order if level[c] == k) for k in range(1, max(level.values()) + 1)]


def test_wave_cut_rules():
    d = mix(3, n_graphs=12)
    order = S.schedule(d, "tree")
    res = P.plan(d, order, batched=True, wave_max=2)
    assert all(len(w) <= 2 for w in res["steps"])
    res = P.plan(d, order, batched=True)
    # unlimited budget: a wave closes only when a contraction needs the wave's output
    for w, nxt in zip(res["steps"], res["steps"][1:]):
        produced = set(w)
        assert any(x in produced for x in d.children(nxt[0]))


def test_time_slice_passes_are_plans_of_the_sliced_dag():
    """A pass over nt / C time slices is the plan of the same graphs built on
    tensors of nt / C slices, under half the budget: the counters of C passes
    are C times that plan's and the resident peak twice its peak (both halves).
    With an unlimited budget every leaf moves once in total, a slice per pass."""
    for seed in range(6):
        wl4 = W.meson_ring(n_leaves=6, nvec=4, nt=4, n_graphs=10, lmin=3, lmax=6, seed=seed,
                           with_data=False)
        wl1 = W.meson_ring(n_leaves=6, nvec=4, nt=1, n_graphs=10, lmin=3, lmax=6, seed=seed,
                           with_data=False)
        d4 = D.build(wl4.leaves, wl4.graphs)
        d1 = D.build(wl1.leaves, wl1.graphs)
        order = S.input_order(d4)
        assert order == S.input_order(d1)
        live = S.memsim(d4, order)["peak_live"]
        for budget in (P.UNLIMITED, live // 2, live // 3):
            for batched in (False, True):
                try:
                    one = P.plan(d1, order, budget=budget // 2, batched=batched)
                except P.BudgetError:
                    with pytest.raises(P.BudgetError):
                        P.plan(d4, order, budget=budget, batched=batched, t_chunks=4)
                    continue
                four = P.plan(d4, order, budget=budget, batched=batched, t_chunks=4)
                for k in ("n_steps", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes"):
                    assert four[k] == 4 * one[k], k
                assert four["peak_resident"] == 2 * one["peak_resident"]
                assert four["ops"] == one["ops"]
                if budget == P.UNLIMITED:
                    assert four["h2d_bytes"] == sum(d4.size(u) for u in range(d4.n_leaves))
        with pytest.raises(ValueError):
            P.plan(d4, order, t_chunks=3)
