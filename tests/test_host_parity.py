"""Host parity (CPU only): the C++ library through its C ABI against the oracle.

Schedules, memory-model figures, plan counters and the complete plan op lists
must be identical; malformed input and out-of-order calls must fail cleanly
and leave the context usable.
"""
import json
import os
import re

import numpy as np
import pytest

import paper_2511_02257_amd as X
from paper_2511_02257_amd import binding as B
from synth import workloads as W
from oracle import dag as OD
from oracle import planner as OP
from oracle import schedules as OS

HERE = os.path.dirname(__file__)
HEADER = os.path.join(os.path.dirname(HERE), "include", "cdag.h")


def ctx_for(wl):
    c = X.Context()
    c.build_cdag(wl.leaves, wl.graphs, wl.specs)
    return c


def test_library_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M))
    assert {"build_cdag", "schedule", "set_mem_budget", "execute", "fetch_correlators"} <= declared
    lib = X.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(B.EXPORTED)


def test_binding_constants_match_the_header():
    """Status codes, kinds, policies, precisions and the check flag: the
    binding's numbers are the header's."""
    text = open(HEADER).read()
    val = {k: int(v, 0) for k, v in re.findall(r"\b(CDAG_[A-Z0-9_]+)\s*=\s*(-?(?:0x)?[0-9a-fA-F]+)", text)}
    val.update({k: int(v, 0) for k, v in re.findall(r"#define\s+(CDAG_[A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)", text)})
    assert (B.OK, B.E_INVALID, B.E_STATE, B.E_BUDGET, B.E_HIP, B.E_NOMEM, B.E_RANGE) == tuple(
        val[k] for k in ("CDAG_OK", "CDAG_E_INVALID", "CDAG_E_STATE", "CDAG_E_BUDGET", "CDAG_E_HIP",
                         "CDAG_E_NOMEM", "CDAG_E_RANGE"))
    assert (B.K22, B.K32, B.K33, B.HCA) == tuple(val[f"CDAG_{k}"] for k in ("K22", "K32", "K33", "HCA"))
    assert B.POLICY == {p: val[f"CDAG_SCHED_{p.upper()}"] for p in ("input", "sibling", "tree", "node")}
    assert B.PREC == {"fp64": val["CDAG_FP64"], "fp32": val["CDAG_FP32"], "bf16x3": val["CDAG_BF16X3"],
                      "bf16x6": val["CDAG_BF16X6"]}
    assert B.SCHED_CHECK == val["CDAG_SCHED_CHECK"]
    assert (W.C1, W.C2, W.C3) == (val["CDAG_C1"], val["CDAG_C2"], val["CDAG_C3"])


class _L:
    def __init__(self, rank, nvec=4, nt=1):
        self.rank, self.nvec, self.nt, self.data = rank, nvec, nt, None


class _G:
    def __init__(self, ops, corr=0, w=1.0):
        self.ops, self.corr, self.w = ops, corr, w


def test_table_sch_mem_through_abi():
    gold = json.load(open(os.path.join(HERE, "golden", "table_sch_mem.json")))["schedules"]
    wl = W.fig1_dag("fgh", with_data=False)
    c = ctx_for(wl)
    # node ids from the build: a..d = 0..3, f = 4, e = 5, g = 6, h = 7
    kind, left, right = c.nodes()
    names = {"a": 0, "b": 1, "c": 2, "d": 3}
    for u in range(4, 8):
        key = (int(left[u]), int(right[u]))
        names[{(0, 1): "f", (1, 2): "e", (0, 5): "g", (5, 3): "h"}[key]] = u
    unit = 4 * 4 * 16
    for which, g in gold.items():
        M, pp, pl = c.memsim([names[x] for x in g["order"]], 16)
        assert [int(m) // unit for m in M] == g["size"]
    assert [int(x) for x in c.schedule("tree")] == [names[x] for x in "fegh"]
    assert [int(x) for x in c.schedule("sibling")] == [names[x] for x in "fegh"]
    wl2 = W.fig1_dag("ghf", with_data=False)
    c2 = ctx_for(wl2)
    d2 = OD.build(wl2.leaves, wl2.graphs)
    assert list(c2.schedule("sibling")) == OS.sibling(d2)


def _random_workloads():
    out = []
    for seed in range(30):
        out.append(W.meson_ring(n_leaves=7, nvec=4, nt=2, n_graphs=14, lmin=3, lmax=6, seed=seed,
                                with_data=False))
    for seed in range(30):
        out.append(W.baryon_mix(n_bar=4, n_mes=5, nvec=3, nt=2, n_graphs=12, seed=100 + seed,
                                with_data=False))
    for seed in range(6):
        out.append(W.batched_mix(nvecs=(2, 3), nt=2, n_mes=6, n_bar=4, n_graphs=30, seed=200 + seed,
                                 with_data=False))
    for seed in range(10):
        out.append(W.rank4_mix(nvec=3, nt=2, n_graphs=16, seed=300 + seed, with_data=False))
    for seed in range(6):
        out.append(W.pairs_mix(nvec=3, nt=2, n_graphs=20, seed=400 + seed, with_data=False))
    return out


WORKLOADS = _random_workloads()


@pytest.mark.parametrize("i", range(len(WORKLOADS)))
def test_schedules_and_plans_match_oracle(i):
    wl = WORKLOADS[i]
    d = OD.build(wl.leaves, wl.graphs, wl.specs)
    c = ctx_for(wl)
    kind, left, right = c.nodes()
    assert list(left) == d.left and list(right) == d.right
    assert [int(k) for k in kind[d.n_leaves:]] == d.kind[d.n_leaves:]
    assert list(c.graph_roots()) == d.root_of_graph
    for policy in ("input", "sibling", "tree", "node"):
        order = [int(x) for x in c.schedule(policy, check=(policy in ("tree", "node")))]
        assert order == OS.schedule(d, policy), policy
        for eb in (16, 8):
            M, pp, pl = c.memsim(order, eb)
            sim = OS.memsim(d, order, eb)
            assert list(M) == sim["M"] and pp == sim["peak_post"] and pl == sim["peak_live"]
        live = OS.memsim(d, order)["peak_live"]
        for budget in (None, live // 2, live // 3):
            c.set_mem_budget(budget)
            for batched, look in ((False, 0), (True, 0), (True, 3), (True, B.LOOKAHEAD_ALL)):
                for resident in (False, True):
                    c.set_options(leaves_resident=resident, wave_lookahead=look)
                    ob = OP.UNLIMITED if budget is None else budget
                    try:
                        ref = OP.plan(d, order, budget=ob, batched=batched, leaves_resident=resident,
                                      lookahead=look)
                    except OP.BudgetError:
                        with pytest.raises(X.CdagError) as e:
                            c.plan("fp64", batched)
                        assert e.value.code == B.E_BUDGET
                        continue
                    p = c.plan("fp64", batched)
                    for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes"):
                        assert p[k] == ref[k], (policy, budget, batched, resident, k)
                    assert p["n_steps"] == ref["n_steps"]
                    assert c.plan_ops() == ref["ops"]
                    assert p["tensor_highwater"] >= p["peak_resident"]
        c.set_options(leaves_resident=False, wave_lookahead=0)
        c.set_mem_budget(None)


@pytest.mark.parametrize("i", list(range(0, 76, 5)))
def test_time_slice_pass_plans_match_oracle(i):
    """Plans of an execution in passes over slices of the time axis (sizes / C,
    budget / 2 per pass): counters, steps and the op list of one pass equal
    the oracle's."""
    wl = WORKLOADS[i]
    d = OD.build(wl.leaves, wl.graphs)
    c = ctx_for(wl)
    for policy in ("input", "tree"):
        order = [int(x) for x in c.schedule(policy)]
        live = OS.memsim(d, order)["peak_live"]
        for budget in (None, live // 2, live // 3):
            c.set_mem_budget(budget)
            c.set_time_chunks(2)
            for batched, look, resident in ((False, 0, False), (True, 0, False), (True, 3, True)):
                c.set_options(leaves_resident=resident, wave_lookahead=look)
                ob = OP.UNLIMITED if budget is None else budget
                try:
                    ref = OP.plan(d, order, budget=ob, batched=batched, leaves_resident=resident,
                                  lookahead=look, t_chunks=2)
                except OP.BudgetError:
                    with pytest.raises(X.CdagError) as e:
                        c.plan("fp64", batched)
                    assert e.value.code == B.E_BUDGET
                    continue
                p = c.plan("fp64", batched)
                for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "n_steps"):
                    assert p[k] == ref[k], (policy, budget, batched, resident, k)
                assert c.plan_ops() == ref["ops"]
            c.set_time_chunks(1)
    c.set_options(leaves_resident=False, wave_lookahead=0)
    c.set_mem_budget(None)
    # passes must divide every tensor's time slices
    c.set_time_chunks(3)
    with pytest.raises(X.CdagError) as e:
        c.plan("fp64", True)
    assert e.value.code == B.E_INVALID
    with pytest.raises(X.CdagError) as e:
        c.set_time_chunks(0)
    assert e.value.code == B.E_INVALID
    c.close()


from synth import corr_func as CF   # noqa: E402


@pytest.mark.parametrize("row", sorted(CF.TABLE))
def test_corr_func_shaped_dags_match_oracle(row):
    """Table corr-func-shaped DAGs at 150 trees: DAG statistics, every schedule
    and its memory simulation against the oracle (with the incremental Tree
    gains checked against recomputed ones at every selection)."""
    wl = CF.corr_func_like(row, n_trees=150)
    for lf in wl.leaves:
        lf.nvec = 3
    d = OD.build(wl.leaves, wl.graphs)
    c = ctx_for(wl)
    st, ref = c.dag_stats(), OD.stats(d)
    assert (st["n_vertices"], st["n_edges"], st["n_trees"]) == (ref["n_nodes"], ref["n_edges"], ref["n_trees"])
    assert abs(st["f_v"] - ref["f_v"]) < 1e-12 and abs(st["f_e"] - ref["f_e"]) < 1e-12
    for policy in ("input", "sibling", "tree"):
        order = [int(x) for x in c.schedule(policy, check=(policy in ("tree", "node")))]
        assert order == OS.schedule(d, policy), policy
        M, pp, pl = c.memsim(order, 16)
        sim = OS.memsim(d, order, 16)
        assert list(M) == sim["M"] and pp == sim["peak_post"] and pl == sim["peak_live"]


def test_corr_func_shapes_reach_the_table_sizes():
    """The generators reproduce the table's tree count and leaf count exactly
    and its vertex count within 0.1 % (full size; structure only)."""
    for row in ("a0-d3", "tritium"):
        tab = CF.TABLE[row]
        wl = CF.corr_func_like(row)
        assert len(wl.graphs) == tab["trees"]
        assert len(wl.leaves) == tab["V"] - tab["E"] // 2
        c = ctx_for(wl)
        st = c.dag_stats()
        assert abs(st["n_vertices"] - tab["V"]) <= 0.001 * tab["V"], (row, st)
        assert st["n_edges"] == 2 * (st["n_vertices"] - len(wl.leaves))


def test_general_kinds_flops_and_validation():
    """Plan flops are 8 Nt M N K per exterior contraction (M = N^(rl-c),
    N^(rr-c), K = N^c) plus 8 Nt N^2 per trace; rank rules as in the oracle."""
    wl = W.rank4_mix(nvec=3, nt=2, n_graphs=30, seed=401, with_data=False)
    d = OD.build(wl.leaves, wl.graphs)
    want = 0
    for u in range(d.n_nodes):
        k = d.kind[u]
        if k < 0:
            continue
        n, nt = d.nvec[u], d.nt[u]
        if k == W.HCA:
            want += 8 * nt * n * n
            continue
        c = OD.contracted_axes(k)
        rl, rr = d.rank[d.left[u]], d.rank[d.right[u]]
        want += 8 * nt * n ** (rl - c) * n ** (rr - c) * n ** c
    assert any(d.kind[u] in (W.C1, W.C2, W.C3) for u in range(d.n_nodes))
    c = ctx_for(wl)
    c.schedule("tree")
    assert c.plan("fp64", True)["flops"] == want
    L = [_L(2), _L(3), _L(4), _L(4), _L(3)]
    for ops in ([(W.C2, 0, 1), (W.HCA, -1, 0)], [(W.C1, 2, 3), (W.HCA, -1, 0)],
                [(W.C3, 1, 4), (W.HCA, -1, 0)], [(7, 0, 1), (W.HCA, -1, 0)]):
        with pytest.raises(X.CdagError) as e:
            c.build_cdag(L, [_G(ops)])
        assert e.value.code == B.E_INVALID
    with pytest.raises(X.CdagError):
        c.build_cdag([_L(5), _L(2)], [_G([(W.HCA, 0, 1)])])


def test_mixed_precision_plans_halve_sizes():
    wl = WORKLOADS[3]
    d = OD.build(wl.leaves, wl.graphs)
    c = ctx_for(wl)
    order = [int(x) for x in c.schedule("tree")]
    live = OS.memsim(d, order, 8)["peak_live"]
    c.set_mem_budget(live // 3)
    for prec in ("fp32", "bf16x3", "bf16x6"):
        p = c.plan(prec, True)
        ref = OP.plan(d, order, elem_bytes=8, budget=live // 3, batched=True)
        assert p["h2d_bytes"] == ref["h2d_bytes"] and p["n_evict"] == ref["n_evict"]


GOLD_FULL = os.path.join(HERE, "golden", "full_configs.json")


@pytest.mark.skipif(not os.path.exists(GOLD_FULL), reason="golden file not generated")
def test_full_configs_match_stored_oracle_results():
    """Schedules and plans on the full-size workloads against values written by
    tests/golden/make_full_configs.py (which calls only the oracle)."""
    import hashlib
    gold = json.load(open(GOLD_FULL))
    for name, entry in gold.items():
        wl = W.config(name, with_data=False)
        c = ctx_for(wl)
        for policy, g in entry["policies"].items():
            order = np.asarray(c.schedule(policy), dtype=np.int64)
            assert hashlib.sha256(order.tobytes()).hexdigest() == g["order_sha256"], (name, policy)
            M, pp, pl = c.memsim(order, 16)
            assert (pp, pl) == (g["peak_post"], g["peak_live"])
            c.set_mem_budget(entry["budget"])
            for mode, ref in g["plans"].items():
                p = c.plan("fp64", mode == "waves")
                for k, v in ref.items():
                    assert p[k] == v, (name, policy, mode, k)
            c.set_mem_budget(None)


def test_kernel_variants_round_trip_and_share_decomposition():
    """Every (tile, grid, lds_stages, split_k) choice is stored and reported
    back.  Work items are output tiles of the chosen shape (times the K splits):
    with no split (K = N = 72 < 512) their count is sum over contractions of
    Nt * ceil(M / bm) * ceil(N / bn), whatever the grid policy and LDS stages."""
    wl = W.meson_ring(n_leaves=6, nvec=72, nt=5, n_graphs=20, lmin=4, lmax=6, with_data=False)
    d = OD.build(wl.leaves, wl.graphs)
    n_k22 = sum(1 for u in range(d.n_nodes) if d.kind[u] == W.K22)
    c = ctx_for(wl)
    c.schedule("tree")
    for tile, (bm, bn) in sorted(X.TILES.items()):
        want = n_k22 * 5 * (-(-72 // bm)) * (-(-72 // bn))
        for grid in (0, 1):
            for stages in (2, 1):
                for split in (1, 0):
                    for prec in ("fp64", "fp32", "bf16x3", "bf16x6"):
                        for kind in (0, 1, 2):
                            c.set_tile(prec, kind, 72, tile, grid, stages, split)
                            assert c.get_tile(prec, kind, 72) == (tile, grid, stages, split)
                        assert c.plan(prec, True)["hec_items"] == want, (tile, grid, stages, prec)
    for bad in ((6, 1, 2, 1), (-2, 1, 2, 1), (0, 2, 2, 1), (0, 1, 3, 1), (0, 1, 0, 1), (0, 1, 2, 2)):
        with pytest.raises(X.CdagError) as e:
            c.set_tile("fp64", 0, 72, *bad)
        assert e.value.code == B.E_INVALID
    c.set_tile("fp64", 0, 72, -1)          # back to the default choice
    t, g, st, sk = c.get_tile("fp64", 0, 72)
    assert t in X.TILES and (g, st, sk) == (1, 2, 1)


def test_split_k_choice_sets_the_work_items():
    """K33 at N = 40 has K = 1600: with split_k 1 and fewer than 512 output
    tiles it is cut into min(ceil(512 / tiles), K / 256) splits, rounded to
    whole k-steps; with split_k 0 each output tile is one work item."""
    wl = W.baryon_mix(n_bar=3, n_mes=3, nvec=40, nt=5, n_graphs=12, with_data=False)
    d = OD.build(wl.leaves, wl.graphs)
    n_k = {k: sum(1 for u in range(d.n_nodes) if d.kind[u] == k) for k in (W.K32, W.K33)}
    c = ctx_for(wl)
    c.schedule("tree")
    for tile, (bm, bn) in sorted(X.TILES.items()):
        for prec, kstep in (("fp64", 16), ("fp32", 32), ("bf16x3", 32), ("bf16x6", 32)):
            k32 = n_k[W.K32] * 5 * (-(-1600 // bm)) * (-(-40 // bn))   # K32: M = N^2, K = N: no split
            base33 = 5 * (-(-40 // bm)) * (-(-40 // bn))
            for kind in (1, 2):
                c.set_tile(prec, kind, 40, tile, 1, 2, 0)
            assert c.plan(prec, True)["hec_items"] == k32 + n_k[W.K33] * base33
            for kind in (1, 2):
                c.set_tile(prec, kind, 40, tile, 1, 2, 1)
            splits = max(1, min(-(-512 // base33), 1600 // 256))
            kspl = -(-(-(-1600 // splits)) // kstep) * kstep
            splits = -(-1600 // kspl)
            assert c.plan(prec, True)["hec_items"] == k32 + n_k[W.K33] * base33 * splits, (tile, prec)


def test_launch_records_empty_without_a_timed_execute():
    wl = W.fig1_dag("fgh", with_data=False)
    c = ctx_for(wl)
    assert c.launch_records() == []
    with pytest.raises(X.CdagError) as e:
        B._check(B.lib().cdag_launch_records(c.h, None, 4, None))
    assert e.value.code == B.E_INVALID


def test_errors_leave_context_usable():
    c = X.Context()
    with pytest.raises(X.CdagError) as e:
        c.schedule("tree")
    assert e.value.code == B.E_STATE
    L = [_L(2), _L(2), _L(3)]
    bad = [
        [(W.K22, 0, 0), (W.HCA, -1, 1)],
        [(W.K22, 0, 1)],
        [(W.HCA, 0, 1), (W.HCA, 0, 1)],
        [(W.K22, 0, 7), (W.HCA, -1, 1)],
        [(W.K22, 0, -1), (W.HCA, -1, 1)],
        [(W.K22, 2, 1), (W.HCA, -1, 1)],
        [(W.K22, 0, 1), (W.K22, 1, 0), (W.HCA, -1, 0)],
        [(9, 0, 1), (W.HCA, -1, 1)],
    ]
    for ops in bad:
        with pytest.raises(X.CdagError) as e:
            c.build_cdag(L, [_G(ops)])
        assert e.value.code == B.E_INVALID
    with pytest.raises(X.CdagError):
        c.build_cdag([_L(2, nvec=4), _L(2, nvec=5)], [_G([(W.HCA, 0, 1)])])
    with pytest.raises(X.CdagError):   # one correlator, two Nt
        c.build_cdag([_L(2, nt=1), _L(2, nt=1), _L(2, nt=2), _L(2, nt=2)],
                     [_G([(W.HCA, 0, 1)]), _G([(W.HCA, 2, 3)])])
    # still usable
    wl = W.fig1_dag("fgh", with_data=False)
    c.build_cdag(wl.leaves, wl.graphs)
    assert len(c.schedule("tree")) == 4
    with pytest.raises(X.CdagError) as e:          # no leaf data
        c.execute("fp64", False)
    assert e.value.code == B.E_STATE
    c.set_mem_budget(2 * 4 * 4 * 16)
    with pytest.raises(X.CdagError) as e:
        c.plan("fp64", False)
    assert e.value.code == B.E_BUDGET
    c.set_mem_budget(None)
    assert c.plan("fp64", False)["n_evict"] == 0
    with pytest.raises(X.CdagError) as e:
        B._check(B.lib().cdag_plan(c.h, 7, 0, None))
    assert e.value.code == B.E_INVALID
    with pytest.raises(X.CdagError) as e:
        B._check(B.lib().cdag_bind_device(c.h, 0, None, None))
    assert e.value.code == B.E_INVALID


def test_tree_scheduler_speed_full_meson_ring():
    wl = W.config("meson_ring", with_data=False)
    c = ctx_for(wl)
    import time
    t0 = time.perf_counter()
    c.schedule("tree")
    assert time.perf_counter() - t0 < 5.0


# ---------------------------------------------------------------- general DAGs (any number of children)
def _general_cases():
    from synth.general import random_general
    for seed in range(40):
        yield seed, random_general(seed, n_leaves=6 + seed % 10, n_trees=3 + seed % 12,
                                   max_arity=1 + seed % 5, depth=2 + seed % 3,
                                   share=(0.0, 0.2, 0.5)[seed % 3])


@pytest.mark.parametrize("seed,case", list(_general_cases()))
def test_general_dag_matches_oracle(seed, case):
    """Input order, Tree (with its incremental gains checked against M - M' at
    every pick), node gain, the memory model and the DAG statistics on general
    DAGs."""
    nl, sizes, kids = case
    d = OD.general(nl, sizes, kids)
    c = X.Context()
    c.build_general(nl, sizes, kids)
    for pol in ("input", "tree", "node"):
        got = list(c.schedule(pol, check=(pol in ("tree", "node"))))
        ref = OS.schedule(d, pol)
        assert got == ref, pol
        M, post, live = c.memsim(got)
        sim = OS.memsim(d, ref)
        assert (list(M), post, live) == (sim["M"], sim["peak_post"], sim["peak_live"])
    st, so = c.dag_stats(), OD.stats(d)
    assert (st["n_vertices"], st["n_edges"], st["n_trees"]) == (so["n_nodes"], so["n_edges"], so["n_trees"])
    assert st["f_v"] == pytest.approx(so["f_v"], abs=1e-12) and st["f_e"] == pytest.approx(so["f_e"], abs=1e-12)
    if any(len(k) != 2 for k in kids[nl:]):
        with pytest.raises(X.CdagError) as e:
            c.schedule("sibling")
        assert e.value.code == B.E_INVALID
    c.close()


def test_general_dag_of_a_contraction_dag():
    """A contraction DAG handed over as a general DAG (its FP64 node sizes) gets
    the same input, Sibling, Tree and node-gain orders and memory figures as
    the original."""
    wl = W.config("meson_ring", with_data=False)
    c = ctx_for(wl)
    kind, left, right = c.nodes()
    d = OD.build(wl.leaves, wl.graphs)
    kids = [d.children(u) for u in range(d.n_nodes)]
    g = X.Context()
    g.build_general(d.n_leaves, [d.size(u, 16) for u in range(d.n_nodes)], kids)
    for pol in ("input", "sibling", "tree", "node"):
        a, b = list(c.schedule(pol)), list(g.schedule(pol))
        assert a == b, pol
        assert [list(x) if hasattr(x, "__len__") else x for x in c.memsim(a)] == \
               [list(x) if hasattr(x, "__len__") else x for x in g.memsim(b)]
    gk, gl, gr = g.nodes()
    assert list(gl) == list(left) and list(gr) == list(right)
    assert all(k == 7 for k in gk[d.n_leaves:]) and all(k == -1 for k in gk[:d.n_leaves])
    c.close()
    g.close()


def test_general_dag_validation_and_state():
    c = X.Context()
    bad = [
        (2, [1, 1, 1], [(), (), ()]),            # non-leaf without children
        (2, [1, 1, 1], [(), (0,), (0, 1)]),      # leaf with a child
        (2, [1, 1, 1], [(), (), (0, 0)]),        # repeated child
        (2, [1, 1, 1], [(), (), (0, 2)]),        # child id not below the node
        (2, [1, 1, -1], [(), (), (0, 1)]),       # negative size
        (3, [1, 1], [(), ()]),                   # more leaves than nodes
    ]
    for nl, sizes, kids in bad:
        with pytest.raises(X.CdagError) as e:
            c.build_general(nl, sizes, kids)
        assert e.value.code == B.E_INVALID
    c.build_general(2, [4, 8, 0], [(), (), (0, 1)])
    assert list(c.schedule("tree")) == [2]
    M, post, live = c.memsim([2])
    assert (list(M), post, live) == ([0], 0, 12)
    with pytest.raises(X.CdagError) as e:
        c.plan("fp64", True)
    assert e.value.code == B.E_STATE
    c.close()


@pytest.mark.parametrize("n_leaves", [0, 3])
def test_dag_without_graphs(n_leaves):
    """No graph: every schedule is empty, the plan has no step and moves no byte,
    on both sides."""
    rng = np.random.default_rng(5)
    leaves = [W.Leaf(2, 4, 2, W._draw(rng, (2, 4, 4), 0.5)) for _ in range(n_leaves)]
    wl = W.Workload("no_graphs", leaves, [])
    c = ctx_for(wl)
    for policy in ("input", "sibling", "tree"):
        assert len(c.schedule(policy)) == 0
        d, order, res = OP_counts(wl, policy)
        assert list(order) == []
        p = c.plan("fp64")
        assert p["n_contr"] == 0 and p["n_steps"] == 0 and p["n_roots"] == 0
        for k in ("n_h2d", "h2d_bytes", "n_d2h", "n_evict", "peak_resident"):
            assert p[k] == res[k] == 0, k
        assert p["peak_live"] == p["peak_post"] == 0
    c.close()


def OP_counts(wl, policy):
    d = OD.build(wl.leaves, wl.graphs)
    order = OS.schedule(d, policy, 16)
    return d, order, OP.plan(d, order, elem_bytes=16, budget=OP.UNLIMITED, batched=False)


def test_saved_order_serves_another_n():
    """A schedule found once is installed on a DAG of the same structure built
    with another N and Nt (the paper reuses schedules across N): same plan ops,
    and memory figures that scale with the element count."""
    small = W.meson_ring(n_leaves=8, nvec=4, nt=2, n_graphs=30, lmin=4, lmax=7, seed=41, with_data=False)
    big = W.meson_ring(n_leaves=8, nvec=16, nt=3, n_graphs=30, lmin=4, lmax=7, seed=41, with_data=False)
    a, b = ctx_for(small), ctx_for(big)
    for policy in ("tree", "sibling", "node"):
        order = a.schedule(policy)
        b.set_order(order)
        assert list(b.schedule(policy)) == list(order)        # what b would find itself
        b.set_order(order)
        scale = (16 * 16 * 3) // (4 * 4 * 2)
        Ma, pa, la = a.memsim(order, 16)
        Mb, pb, lb = b.memsim(order, 16)
        assert [x * scale for x in Ma] == list(Mb) and pa * scale == pb and la * scale == lb
        for budget_frac in (None, 3):
            for c, wl in ((a, small), (b, big)):
                if budget_frac is None:
                    c.set_mem_budget(None)
                else:
                    d = OD.build(wl.leaves, wl.graphs)
                    c.set_mem_budget(OS.memsim(d, [int(x) for x in order], 16)["peak_live"] // budget_frac)
            a.plan("fp64", True)
            b.plan("fp64", True)
            assert a.plan_ops() == b.plan_ops()
        a.set_mem_budget(None)
        b.set_mem_budget(None)
    a.close()
    b.close()


def test_set_order_validation():
    wl = W.fig1_dag("fgh", with_data=False)
    c = X.Context()
    with pytest.raises(X.CdagError) as e:
        c.set_order([4, 5, 6, 7])
    assert e.value.code == B.E_STATE
    c.build_cdag(wl.leaves, wl.graphs)
    good = [int(x) for x in c.schedule("tree")]
    d = OD.build(wl.leaves, wl.graphs)
    e_id = next(u for u in d.contractions() if (d.left[u], d.right[u]) == (1, 2))
    g_id = next(u for u in d.contractions() if d.left[u] == 0 and d.right[u] == e_id)
    bad = [good[:-1],                                  # one missing
           good + [good[0]],                           # too many
           [good[0]] * len(good),                      # repeats
           [0] + good[1:],                             # a leaf
           [99] + good[1:],                            # out of range
           [g_id] + [u for u in good if u != g_id]]    # g before its child e
    for o in bad:
        with pytest.raises(X.CdagError) as e:
            c.set_order(o)
        assert e.value.code == B.E_INVALID, o
    c.set_order(good)
    assert c.plan("fp64", False)["n_contr"] == 4
    c.close()


def test_header_is_plain_c99(tmp_path):
    """include/cdag.h compiles as C99 with warnings as errors (the ABI is C)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use.c"
    src.write_text('#include "cdag.h"\n'
                   "int main(void) { cdag_ctx* c = 0; cdag_trace_rec t; cdag_launch_record l;\n"
                   "  cdag_plan_stats p; cdag_exec_stats e; (void)t; (void)l; (void)p; (void)e;\n"
                   "  return cdag_create(&c); }\n")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.dirname(HEADER), "-c", str(src), "-o", str(tmp_path / "use.o")],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("which", ["meson_ring", "baryon_mix", "a0-d3", "tritium", "general"])
def test_node_scheduler_self_check_at_full_size(which):
    """Where the oracle is too slow (quadratic in the DAG), the library's own
    check mode verifies every pick of the node scheduler: each ready gain
    recomputed equals the cached one, and the pick is the largest."""
    c = X.Context()
    if which == "general":
        from synth.general import random_general
        nl, sizes, kids = random_general(7, n_leaves=200, n_trees=4000, max_arity=4, depth=3, share=0.05)
        c.build_general(nl, sizes, kids)
    else:
        wl = CF.corr_func_like(which) if which in CF.TABLE else W.config(which, with_data=False)
        c.build_cdag(wl.leaves, wl.graphs)
    assert list(c.schedule("node", check=True)) == list(c.schedule("node"))
    c.close()


def test_index_pair_specs_build_and_validation():
    """Contractions over index pairs: node kinds, ranks and merging equal the
    oracle's (a spec equal to C1 merges with C1 nodes); every malformed spec
    or use is refused with CDAG_E_INVALID; split-BF16 plans refuse them."""
    wl = W.pairs_mix(nvec=3, nt=2, n_graphs=40, seed=9, with_data=False)
    d = OD.build(wl.leaves, wl.graphs, wl.specs)
    c = ctx_for(wl)
    kind, left, right = c.nodes()
    assert [int(k) for k in kind] == d.kind and list(left) == d.left and list(right) == d.right
    assert W.SPEC_BASE + 4 not in d.kind and W.C1 in d.kind          # the C1-shaped spec merged
    c.schedule("tree")
    assert c.plan("fp64", True)["n_contr"] == d.n_nodes - d.n_leaves
    with pytest.raises(X.CdagError) as e:
        c.plan("bf16x3", True)
    assert e.value.code == B.E_INVALID
    L = [W.Leaf(3, 3, 1), W.Leaf(3, 3, 1), W.Leaf(2, 3, 1)]
    bad = [W.Spec(3, 3, ((0, 0), (0, 1)), (0, 1)),          # an axis twice
           W.Spec(3, 3, ((3, 0),), (0, 1, 2, 3)),          # axis out of range
           W.Spec(3, 3, ((0, 0),), (0, 1, 1, 2)),          # perm not a permutation
           W.Spec(3, 2, ((0, 0),), (0, 1, 2)),             # ranks differ from the operands'
           W.Spec(3, 3, ((0, 0), (1, 1), (2, 2)), (0,))]   # output rank 0
    for sp in bad:
        g = [W.GraphSpec([(W.SPEC_BASE, 0, 1), (W.HCA, -1, 2)])] if len(sp.perm) == 2 else \
            [W.GraphSpec([(W.SPEC_BASE, 0, 1), (W.C2, -1, 0), (W.HCA, -1, 2)])]
        with pytest.raises(X.CdagError) as e:
            X.Context().build_cdag(L, g, [sp])
        assert e.value.code == B.E_INVALID, sp
        with pytest.raises(OD.InvalidGraph):
            OD.build(L, g, [sp])
    with pytest.raises(X.CdagError) as e:                  # a kind with no spec
        X.Context().build_cdag(L, [W.GraphSpec([(W.SPEC_BASE + 1, 0, 1), (W.HCA, -1, 2)])], [])
    assert e.value.code == B.E_INVALID
