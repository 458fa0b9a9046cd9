"""Executor walk without a GPU (CPU only): the eager three-stream issue order
(kernels, uploads, spills), recorded by cdag_trace_execute, checked for races.

A happens-before check with vector clocks over the three streams: every pair of
accesses to overlapping bytes of the same space (device arena, host spill
pool, a leaf's staging buffer) where one is a write must be ordered, by the
stream order or by an event the later stream waited for.  The checker is
pinned by planting mistakes in the trace (a wait taken out) and requiring that
it reports them.  Transfers must follow the plan's op list, every wait must
name an event recorded earlier, and an injected failure at any record must
leave the context usable.
"""
import pytest

import paper_2511_02257_amd as X
from paper_2511_02257_amd import binding as B
from synth import workloads as W
from oracle import dag as OD
from oracle import schedules as OS


NS = 3   # streams: compute, upload, spill


def races(trace):
    """(earlier record index, later record index) of every unordered conflicting pair."""
    clock = {s: [0] * NS for s in range(NS)}
    events = {}
    op_clock = {}
    seen = []          # (index, space key, lo, hi, write, stream, clock, seq)
    bad = []
    for i, r in enumerate(trace):
        st = r["stream"]
        if r["op"] == "record":
            events[r["event"]] = list(clock[st])
            continue
        if r["op"] == "wait":
            e = events[r["event"]]
            clock[st] = [max(a, b) for a, b in zip(clock[st], e)]
            continue
        if r["seq"] not in op_clock:
            clock[st][st] += 1
            op_clock[r["seq"]] = list(clock[st])
        vc = op_clock[r["seq"]]
        key = (r["space"], r["node"] if r["space"] == "stage" else None)
        lo, hi, w = r["off"], r["off"] + r["bytes"], r["op"] == "write"
        for j, k2, lo2, hi2, w2, st2, vc2, seq2 in seen:
            if k2 == key and seq2 != r["seq"] and (w or w2) and lo2 < hi and lo < hi2:
                if vc2[st2] > vc[st2]:
                    bad.append((j, i))
        seen.append((i, key, lo, hi, w, st, vc, r["seq"]))
    return bad


def _visit(los, segs, lo, hi, fresh):
    """Segments of one space covering [lo, hi), split at lo and hi, with gaps
    filled by fresh(a, b) segments; segs[k] = [lo, hi, ...], sorted, disjoint."""
    import bisect

    def split(x):
        k = bisect.bisect_right(los, x) - 1
        if k >= 0 and segs[k][0] < x < segs[k][1]:
            a = segs[k]
            b = [x, a[1]] + [list(v) if isinstance(v, list) else v for v in a[2:]]
            a[1] = x
            los.insert(k + 1, x)
            segs.insert(k + 1, b)
    split(lo)
    split(hi)
    k = bisect.bisect_left(los, lo)
    pos = lo
    while pos < hi:
        end = segs[k][0] if k < len(segs) and segs[k][0] < hi else hi
        if end > pos:                                  # a gap nothing touched yet
            los.insert(k, pos)
            segs.insert(k, fresh(pos, end))
        yield segs[k]
        pos = segs[k][1]
        k += 1


def provenance_errors(trace):
    """Reads whose bytes were last written by another tensor (or never written):
    every device range a kernel or a spill reads must hold that tensor, and
    every spill-pool range an upload reads must hold its spilled copy."""
    spaces = {}
    bad = []
    for i, r in enumerate(trace):
        if r["op"] not in ("read", "write") or r["space"] == "stage":
            continue
        los, segs = spaces.setdefault(r["space"], ([], []))
        for seg in _visit(los, segs, r["off"], r["off"] + r["bytes"], lambda a, b: [a, b, None]):
            if r["op"] == "write":
                seg[2] = r["node"]
            elif seg[2] != r["node"]:
                bad.append((i, r["node"], seg[2]))
    return bad


def races_by_segment(trace):
    """The same happens-before check, kept per byte segment: each segment holds
    its last write and the reads since, so a new access is compared with those
    only (an earlier write is ordered before the last one, or that pair was
    already reported).  Finds a race exactly when races() does; fast enough
    for full-size walks.  Returns the number of unordered pairs it saw."""
    clock = {s: [0] * NS for s in range(NS)}
    events = {}
    op_clock = {}
    spaces = {}        # key -> (los, segs); segs[k] = [lo, hi, last write, reads since]
    n_bad = 0
    for i, r in enumerate(trace):
        st = r["stream"]
        if r["op"] == "record":
            events[r["event"]] = list(clock[st])
            continue
        if r["op"] == "wait":
            clock[st] = [max(a, b) for a, b in zip(clock[st], events[r["event"]])]
            continue
        if r["seq"] not in op_clock:
            clock[st][st] += 1
            op_clock[r["seq"]] = list(clock[st])
        cur = (st, op_clock[r["seq"]], r["seq"])
        key = (r["space"], r["node"] if r["space"] == "stage" else None)
        los, segs = spaces.setdefault(key, ([], []))
        w = r["op"] == "write"
        for seg in _visit(los, segs, r["off"], r["off"] + r["bytes"], lambda a, b: [a, b, None, []]):
            prior = ([seg[2]] if seg[2] is not None else []) + (seg[3] if w else [])
            for p_st, p_vc, p_seq in prior:
                if p_seq != cur[2] and p_vc[p_st] > cur[1][p_st]:
                    n_bad += 1
            if w:
                seg[2], seg[3] = cur, []
            else:
                seg[3].append(cur)
    return n_bad


def _ctx(wl):
    c = X.Context()
    c.build_cdag(wl.leaves, wl.graphs)
    return c


def _cases():
    yield "meson", W.meson_ring(n_leaves=8, nvec=8, nt=2, n_graphs=24, lmin=4, lmax=7, seed=31,
                                with_data=False)
    yield "baryon", W.baryon_mix(n_bar=4, n_mes=4, nvec=4, nt=2, n_graphs=10, seed=32, with_data=False)
    yield "rank4", W.rank4_mix(nvec=3, nt=2, n_graphs=12, seed=33, with_data=False)


CASES = list(_cases())


def _budget(wl, frac):
    d = OD.build(wl.leaves, wl.graphs)
    return OS.memsim(d, OS.input_order(d), 16)["peak_live"] // frac


@pytest.mark.parametrize("name,wl", CASES, ids=[n for n, _ in CASES])
@pytest.mark.parametrize("policy", ["input", "tree", "node"])
def test_eager_walk_has_no_races(name, wl, policy):
    c = _ctx(wl)
    c.schedule(policy)
    checked = 0
    for frac in (None, 3, 5):
        budget = None if frac is None else _budget(wl, frac)
        c.set_mem_budget(budget)
        for batched, look, resident in ((False, 0, False), (True, 0, False), (True, 16, False),
                                        (True, B.LOOKAHEAD_ALL, True)):
            c.set_options(leaves_resident=resident, wave_lookahead=look)
            for prec in ("fp64", "fp32"):
                try:
                    p = c.plan(prec, batched)
                except X.CdagError as e:
                    assert e.code == B.E_BUDGET
                    continue
                t = c.trace_execute(prec, batched)
                assert races(t) == [], (name, policy, frac, batched, look, resident, prec)
                # transfers in the plan's order, one per H2D / D2H record; the
                # spill stream moves D2H, the upload stream H2D
                moves = [(r["node"], r["step"]) for r in t if r["op"] == "write" and r["stream"] in (1, 2)]
                plan = [(node, step) for op, node, step in c.plan_ops() if op in ("H2D", "D2H")]
                assert moves == plan
                assert all(r["stream"] == (2 if r["space"] == "spill" else 1)
                           for r in t if r["op"] == "write" and r["stream"] != 0)
                assert p["n_h2d"] + p["n_d2h"] == len(plan)
                recorded = set()
                for r in t:
                    if r["op"] == "record":
                        recorded.add(r["event"])
                    elif r["op"] == "wait":
                        assert r["event"] in recorded
                checked += 1
    assert checked >= 10
    c.close()


def test_checker_finds_planted_missing_waits():
    """Waits taken out of a budgeted walk: of a sample of single waits, at
    least one leaves a conflicting pair unordered; taking all out leaves many."""
    name, wl = CASES[0]
    c = _ctx(wl)
    c.schedule("tree")
    c.set_mem_budget(_budget(wl, 4))
    c.set_options(leaves_resident=False, wave_lookahead=0)
    t = c.trace_execute("fp64", False)
    c.close()
    assert races(t) == []
    waits = [i for i, r in enumerate(t) if r["op"] == "wait"]
    assert len(waits) > 10
    found = 0
    for i in waits[::max(1, len(waits) // 12)]:
        found += bool(races(t[:i] + t[i + 1:]))
    assert found >= 1
    assert len(races([r for r in t if r["op"] != "wait"])) > 10
    # the upload stream's first wait guards an upload into memory that a kernel
    # of an earlier step still reads; without it that pair is unordered
    k = next(i for i, r in enumerate(t) if r["op"] == "wait" and r["stream"] == 1)
    assert races(t[:k] + t[k + 1:])
    # every stream's waits matter: without all the waits of one stream, some
    # pair it takes part in is unordered
    for st in range(NS):
        assert races([r for r in t if not (r["op"] == "wait" and r["stream"] == st)]), st


def _chunk_cases():
    yield "meson", W.meson_ring(n_leaves=8, nvec=8, nt=4, n_graphs=24, lmin=4, lmax=7, seed=34,
                                with_data=False)
    yield "baryon", W.baryon_mix(n_bar=4, n_mes=4, nvec=4, nt=8, n_graphs=10, seed=35, with_data=False)


@pytest.mark.parametrize("name,wl", list(_chunk_cases()), ids=["meson", "baryon"])
@pytest.mark.parametrize("chunks", [2, 4])
def test_time_slice_passes_have_no_races(name, wl, chunks):
    """Passes over slices of the time axis alternate between two halves of the
    arena and of the spill pool: no race across passes (a pass waits for the
    one two before it), every read finds its tensor, and the transfers are
    the plan's, once per pass, each moving the pass's slices."""
    c = _ctx(wl)
    d = OD.build(wl.leaves, wl.graphs)
    checked = planted = 0
    for policy in ("input", "tree"):
        c.schedule(policy)
        for frac in (None, 3, 5):
            budget = None if frac is None else 2 * _budget(wl, frac) // chunks
            c.set_mem_budget(budget)
            c.set_time_chunks(chunks)
            for batched, look, resident in ((False, 0, False), (True, 16, False), (True, 16, True)):
                c.set_options(leaves_resident=resident, wave_lookahead=look)
                try:
                    p = c.plan("fp64", batched)
                except X.CdagError as e:
                    assert e.code == B.E_BUDGET
                    continue
                t = c.trace_execute("fp64", batched)
                assert races_by_segment(t) == 0, (policy, frac, batched, look, resident)
                u = [r for r in t if not (resident and r["op"] == "read" and r["node"] < len(wl.leaves))]
                assert provenance_errors(u) == []
                moves = [(r["node"], r["step"] % (p["n_steps"] // chunks)) for r in t
                         if r["op"] == "write" and r["stream"] in (1, 2)]
                plan = [(node, step) for op, node, step in c.plan_ops() if op in ("H2D", "D2H")]
                assert moves == plan * chunks
                assert p["n_h2d"] + p["n_d2h"] == chunks * len(plan)
                for r in t:
                    if r["op"] in ("read", "write") and r["space"] != "stage":
                        assert r["bytes"] == d.size(r["node"], 16) // chunks
                if chunks > 2 and p["n_h2d"]:
                    # without the pass-end waits, pass k and pass k - 2 (same
                    # half) are unordered unless other waits happen to order them
                    nw = [r for r in t if not (r["op"] == "wait" and r["event"] >= 3 * p["n_steps"])]
                    planted += races_by_segment(nw) > 0
                checked += 1
            c.set_time_chunks(1)
    assert checked >= 8
    # on the meson DAG some upload of pass k is ordered against pass k - 2
    # only by the pass-end waits (on the baryon DAG other waits also do)
    assert chunks == 2 or name != "meson" or planted >= 1
    c.close()


def test_trace_fusion_leaves_plan_and_walk_unchanged():
    """Trace fusion changes only how a step's kernels are grouped into
    launches: the plan and the executor's walk (transfers, waits, the ranges
    each step's kernels read and write) are the same with it on."""
    for name, wl in CASES:
        c = _ctx(wl)
        c.schedule("tree")
        c.set_mem_budget(_budget(wl, 2))
        c.set_options(leaves_resident=False, wave_lookahead=16)
        c.set_trace_fusion(False)
        p0, t0 = c.plan("fp64", True), c.trace_execute("fp64", True)
        assert p0["n_h2d"] > 0
        c.set_trace_fusion(True)
        p1, t1 = c.plan("fp64", True), c.trace_execute("fp64", True)
        c.close()
        assert {k: v for k, v in p0.items() if not k.startswith("t_")} == \
            {k: v for k, v in p1.items() if not k.startswith("t_")}, name
        assert t0 == t1, name


def test_injected_failures_leave_the_context_usable():
    name, wl = CASES[0]
    c = _ctx(wl)
    c.schedule("tree")
    c.set_mem_budget(_budget(wl, 4))
    full = c.trace_execute("fp64", False)
    for k in (0, 1, len(full) // 2, len(full) - 1):
        with pytest.raises(X.CdagError) as e:
            c.trace_execute("fp64", False, fail_at=k)
        assert e.value.code == B.E_HIP
        assert "injected" in str(e.value)
        assert c.trace_execute("fp64", False) == full
    assert c.trace_execute("fp64", False, fail_at=len(full)) == full      # past the end: no failure
    c.close()


def test_trace_needs_a_schedule_and_shapes():
    c = X.Context()
    with pytest.raises(X.CdagError) as e:
        c.trace_execute()
    assert e.value.code == B.E_STATE
    c.build_general(2, [1, 1, 0], [(), (), (0, 1)])
    c.schedule("tree")
    with pytest.raises(X.CdagError) as e:
        c.trace_execute()
    assert e.value.code == B.E_STATE
    c.close()


def test_segment_checker_agrees_with_the_pairwise_one():
    """On clean walks and on walks with planted missing waits, both checkers
    agree on whether there is a race."""
    name, wl = CASES[0]
    c = _ctx(wl)
    for policy in ("tree", "input"):
        c.schedule(policy)
        c.set_mem_budget(_budget(wl, 4))
        t = c.trace_execute("fp64", False)
        assert races(t) == [] and races_by_segment(t) == 0
        waits = [i for i, r in enumerate(t) if r["op"] == "wait"]
        for i in waits[::max(1, len(waits) // 15)]:
            u = t[:i] + t[i + 1:]
            assert bool(races(u)) == (races_by_segment(u) > 0), i
        u = [r for r in t if r["op"] != "wait"]
        assert races_by_segment(u) > 0
    c.close()


@pytest.mark.parametrize("policy,look,prec", [("input", 0, "fp64"), ("tree", 0, "fp64"), ("tree", 16, "fp64"),
                                              ("node", 16, "fp64"), ("tree", 16, "fp32"), ("input", 0, "fp32")])
def test_full_meson_budgeted_walk_has_no_races(policy, look, prec):
    """The bench's budgeted meson configuration at full size (2000 graphs,
    leaves on the host, a quarter of the input-order live peak of the
    precision): no race, and every read finds its tensor."""
    wl = W.config("meson_ring", with_data=False)
    c = _ctx(wl)
    c.schedule("input")
    budget = c.plan(prec, False)["peak_live"] // 4
    c.schedule(policy)
    c.set_mem_budget(budget)
    c.set_options(leaves_resident=False, wave_lookahead=look)
    p = c.plan(prec, True)
    t = c.trace_execute(prec, True)
    c.close()
    assert p["n_evict"] > 0 and p["n_d2h"] > 0
    assert races_by_segment(t) == 0
    assert provenance_errors(t) == []


@pytest.mark.parametrize("name,wl", CASES, ids=[n for n, _ in CASES])
def test_every_read_finds_its_tensor(name, wl):
    """Placement (arena and spill-pool offsets): every range read holds the
    tensor that is read, across budgets, waves and resident leaves."""
    c = _ctx(wl)
    for policy in ("input", "tree"):
        c.schedule(policy)
        for frac in (None, 3, 5):
            c.set_mem_budget(None if frac is None else _budget(wl, frac))
            for batched, look, resident in ((False, 0, False), (True, 16, False), (True, 0, True)):
                c.set_options(leaves_resident=resident, wave_lookahead=look)
                try:
                    c.plan("fp64", batched)
                except X.CdagError:
                    continue
                t = c.trace_execute("fp64", batched)
                if resident:   # resident leaves are uploaded once, outside the walk
                    t = [r for r in t if not (r["op"] == "read" and r["node"] < len(wl.leaves))]
                assert provenance_errors(t) == [], (policy, frac, batched, look, resident)
    c.close()


def test_provenance_check_finds_a_planted_overlap():
    """Moving one upload's destination onto another live tensor is reported."""
    name, wl = CASES[0]
    c = _ctx(wl)
    c.schedule("tree")
    c.set_mem_budget(_budget(wl, 4))
    t = c.trace_execute("fp64", False)
    c.close()
    assert provenance_errors(t) == []
    ups = [i for i, r in enumerate(t) if r["op"] == "write" and r["stream"] == 1 and r["space"] == "arena"]
    k1, k2 = ups[0], ups[1]
    u = [dict(r) for r in t]
    u[k2]["off"] = u[k1]["off"]             # second upload lands on the first
    assert provenance_errors(u)


@pytest.mark.parametrize("name,prec", [("batched", "fp32"), ("baryon_mix", "fp64")])
@pytest.mark.parametrize("policy", ["input", "tree"])
def test_full_configuration_walks_under_their_budgets(name, prec, policy):
    """The batched (20,301 contractions; input order evicts 2,967 times there)
    and baryon configurations at full size under their own budgets, waves with
    lookahead 16: no race, every read finds its tensor."""
    wl = W.config(name, with_data=False)
    c = _ctx(wl)
    c.schedule(policy)
    c.set_mem_budget(wl.budget_bytes)
    c.set_options(leaves_resident=False, wave_lookahead=16)
    p = c.plan(prec, True)
    t = c.trace_execute(prec, True)
    c.close()
    if name == "batched" and policy == "input":
        assert p["n_evict"] > 0 and p["n_d2h"] > 0
    assert races_by_segment(t) == 0
    assert provenance_errors(t) == []


@pytest.mark.parametrize("name,prec,policy,chunks,look", [
    ("meson_ring", "fp64", "tree", 16, 384), ("meson_ring", "fp64", "input", 16, 384),
    ("baryon_mix", "fp64", "tree", 8, None), ("batched", "fp32", "tree", 8, None)])
def test_full_configurations_in_passes_have_no_races(name, prec, policy, chunks, look):
    """The bench's pass configurations at full size: the meson DAG in 16 passes
    with lookahead 384 under a quarter of the input-order live peak, the
    headline and batched DAGs in 8 passes with every ready contraction in a
    wave under their budgets.  No race between the three streams, and every
    read finds its tensor."""
    wl = W.config(name, with_data=False)
    c = _ctx(wl)
    if name == "meson_ring":
        c.schedule("input")
        budget = c.plan(prec, False)["peak_live"] // 4
    else:
        budget = wl.budget_bytes
    c.schedule(policy)
    c.set_mem_budget(budget)
    c.set_time_chunks(chunks)
    c.set_options(leaves_resident=False, wave_lookahead=X.binding.LOOKAHEAD_ALL if look is None else look)
    p = c.plan(prec, True)
    t = c.trace_execute(prec, True)
    c.close()
    assert p["peak_resident"] <= budget
    assert races_by_segment(t) == 0
    assert provenance_errors(t) == []
