"""GPU parity: the HIP path through the C ABI against the oracle (marked gpu).

Bars: FP64 correlators within 1e-12 (norm-wise relative over t per graph);
FP32 within 1e-5; split-BF16 with three pieces (six products) within 1e-5;
split-BF16 with two pieces (three products) within 4e-5 on these small
rings of up to 7 contractions (each operand keeps 16 of its 24 significand
bits, so a product carries up to ~3 * 2^-16 relative error; the mode meets
1e-5 on the baryon and batched configurations, not on long meson rings);
cross sums within the same bound of the condition scale sum_g |w_g C_g|;
plan counters equal to the oracle's; identical bits across schedules,
budgets and batching within one precision.
"""
import numpy as np
import pytest

from synth import workloads as W
from oracle import values as OV

from gpu_util import run, rel_errors, sum_errors, oracle_plan_counts

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 4e-5, "bf16x6": 1e-5}


def _wl_meson_small():
    # N = 72: two 64-wide tiles per dimension with a ragged tail of 8
    return W.meson_ring(n_leaves=8, nvec=72, nt=5, n_graphs=40, lmin=4, lmax=7, sigma=1 / 8,
                        n_corr=3, seed=11, name="meson_small")


def _wl_baryon_small():
    # N = 40: ragged tiles; K33 has K = 1600 and runs split-K
    return W.baryon_mix(n_bar=4, n_mes=4, nvec=40, nt=3, n_graphs=12, sigma=1 / 16, n_corr=2,
                        seed=12, name="baryon_small")


def _wl_rank4_small():
    # N = 10: rank-4 intermediates (C1 on two baryons, GEMM 100 x 100 x 10),
    # C2 of rank 4 x 3 (100 x 10 x 100) and C3 of rank 4 x 4 (10 x 10 x 1000,
    # split-K with a ragged tail); ragged tiles everywhere
    return W.rank4_mix(n_bar=5, n_mes=4, n_r4=2, nvec=10, nt=3, n_graphs=24, seed=14, name="rank4_small")


@pytest.fixture(scope="module")
def rank4_small():
    wl = _wl_rank4_small()
    return wl, OV.correlators(wl)


@pytest.fixture(scope="module")
def tiny():
    wl = W.config("tiny")
    return wl, OV.correlators(wl)


@pytest.fixture(scope="module")
def meson_small():
    wl = _wl_meson_small()
    return wl, OV.correlators(wl)


@pytest.fixture(scope="module")
def baryon_small():
    wl = _wl_baryon_small()
    return wl, OV.correlators(wl)


def test_tiny_fp64_all_modes(tiny):
    wl, ref = tiny
    base = None
    for policy in ("input", "sibling", "tree", "node"):
        for batched in (False, True):
            r = run(wl, policy, "fp64", batched)
            err = rel_errors(r["corr"], ref)
            print(f"tiny {policy} batched={batched} max rel {err.max():.3e}")
            assert err.max() <= TOL["fp64"]
            assert sum_errors(wl, r["sums"], ref) <= 1e-12
            bits = np.concatenate(r["corr"]).view(np.uint64)
            if base is None:
                base = bits
            assert np.array_equal(bits, base), "correlators differ across schedules/batching"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_meson_ragged_with_evictions(meson_small, prec):
    wl, ref = meson_small
    eb = 16 if prec == "fp64" else 8
    # a quarter of the input-order live peak: forces spills and re-uploads
    from oracle import dag as OD, schedules as OS
    d = OD.build(wl.leaves, wl.graphs)
    budget = OS.memsim(d, OS.input_order(d), eb)["peak_live"] // 4
    results = []
    for policy, batched, look, graphs in (
            ("input", False, 0, True), ("input", False, 0, False), ("input", True, 0, True),
            ("tree", False, 0, False), ("tree", True, 0, True), ("tree", True, 0, False),
            ("tree", True, 5, True), ("tree", True, 1 << 62, False),
            ("node", False, 0, True), ("node", True, 0, False)):
        r = run(wl, policy, prec, batched, budget=budget, wave_lookahead=look, use_graphs=graphs)
        _, _, o = oracle_plan_counts(wl, policy, eb, budget, batched, lookahead=look)
        p = r["stats"]["plan"]
        for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes"):
            assert p[k] == o[k], (policy, batched, k)
        assert p["n_evict"] > 0
        err = rel_errors(r["corr"], ref)
        print(f"meson_small {prec} {policy} batched={batched} lookahead={look} graphs={graphs} "
              f"waves={p['n_steps']} evict={p['n_evict']} "
              f"max rel {err.max():.3e} median {np.median(err):.3e}")
        assert err.max() <= TOL[prec]
        results.append(np.concatenate(r["corr"]).view(np.uint64))
    for b in results[1:]:
        assert np.array_equal(b, results[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_baryon_ragged_splitk(baryon_small, prec):
    wl, ref = baryon_small
    results = []
    for policy, batched in (("tree", False), ("tree", True), ("sibling", True)):
        r = run(wl, policy, prec, batched)
        err = rel_errors(r["corr"], ref)
        print(f"baryon_small {prec} {policy} batched={batched} max rel {err.max():.3e} "
              f"median {np.median(err):.3e}")
        assert err.max() <= TOL[prec]
        assert sum_errors(wl, r["sums"], ref) <= TOL[prec]
        results.append(np.concatenate(r["corr"]).view(np.uint64))
    for b in results[1:]:
        assert np.array_equal(b, results[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("grid", [0, 1])
@pytest.mark.parametrize("stages", [2, 1])
def test_every_tile_shape(meson_small, baryon_small, prec, tile, grid, stages):
    for name, (wl, ref) in (("meson_small", meson_small), ("baryon_small", baryon_small)):
        r = run(wl, "tree", prec, True, tile=tile, grid=grid, lds_stages=stages)
        err = rel_errors(r["corr"], ref)
        print(f"{name} {prec} tile {tile} grid {grid} stages {stages}: max rel {err.max():.3e}")
        assert err.max() <= TOL[prec]


def _wl_interior():
    # N = 64 and 48: contractions that are a whole number of tiles for the tile
    # shapes dividing their GEMM, whose launches run the kernel form without
    # bounds tests (K33 at N = 64 runs split-K with K = 4096)
    return [W.meson_ring(n_leaves=6, nvec=64, nt=2, n_graphs=16, lmin=4, lmax=6, sigma=1 / 8, n_corr=2,
                         seed=61, name="meson_n64"),
            W.baryon_mix(n_bar=3, n_mes=3, nvec=64, nt=2, n_graphs=8, sigma=1 / 16, n_corr=2, seed=62,
                         name="baryon_n64"),
            W.baryon_mix(n_bar=3, n_mes=3, nvec=48, nt=2, n_graphs=8, sigma=1 / 16, n_corr=2, seed=63,
                         name="baryon_n48")]


@pytest.fixture(scope="module")
def interior_workloads():
    return [(wl, OV.correlators(wl)) for wl in _wl_interior()]


def _interior_expected(name, tile, prec):
    """Which exterior-contraction launches are interior: 'all', 'some' or
    'none', from the GEMM shapes (K22 64 x 64 x 64; K32 N^2 x N x N; K33
    N x N x N^2) against the tile and the k-step (FP64 16, FP32 and split
    BF16 32)."""
    bm, bn = {0: (64, 64), 1: (32, 32), 2: (48, 48), 3: (128, 64), 4: (64, 32), 5: (64, 64)}[tile]
    n = 64 if name.endswith("n64") else 48
    bk = 16 if prec == "fp64" else 32
    shapes = [(n, n, n)] if name.startswith("meson") else [(n * n, n, n), (n, n, n * n)]
    ok = [m % bm == 0 and nn % bn == 0 and k % bk == 0 for m, nn, k in shapes]
    return "all" if all(ok) else "some" if any(ok) else "none"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("grid", [0, 1])
@pytest.mark.parametrize("stages", [2, 1])
def test_every_tile_shape_interior(interior_workloads, prec, tile, grid, stages):
    """Whole tiles: every variant in its interior form (unpredicated vector
    loads, stores without bounds tests) against the oracle, and the launch
    records say which launches ran it."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    for wl, ref in interior_workloads:
        ctx = X.Context()
        ctx.build_cdag(wl.leaves, wl.graphs)
        ctx.schedule("tree")
        ctx.set_options(wave_lookahead=X.binding.LOOKAHEAD_ALL)
        for kind in (0, 1, 2):
            ctx.set_tile(prec, kind, wl.leaves[0].nvec, tile, grid, stages, 1)
        runner = DeviceRunner(ctx, 0)
        ctx.set_timing(True)
        runner.run(prec, True)
        hec = [r for r in ctx.launch_records() if r["type"] == "hec"]
        corr = ctx.fetch_correlators()
        ctx.close()
        err = rel_errors(corr, ref)
        inner = [r["interior"] for r in hec]
        expect = _interior_expected(wl.name, tile, prec)
        print(f"{wl.name} {prec} tile {tile} grid {grid} stages {stages}: interior {sum(inner)}/{len(inner)} "
              f"(expected {expect}), max rel {err.max():.3e}")
        assert err.max() <= TOL[prec]
        if expect == "all":
            assert all(inner)
        elif expect == "some":
            assert any(inner)
        else:
            assert not any(inner)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_without_split_k(baryon_small, prec):
    """split_k 0: K33 (K = 1600) runs as one work item per output tile with the
    whole K in one accumulator; the result matches the oracle and does not
    depend on grouping (waves vs one launch per contraction)."""
    wl, ref = baryon_small
    a = run(wl, "tree", prec, True, tile=0, grid=1, split_k=0)
    b = run(wl, "tree", prec, False, tile=0, grid=1, split_k=0)
    c = run(wl, "tree", prec, True, tile=0, grid=1, split_k=1)
    assert a["stats"]["plan"]["hec_items"] < c["stats"]["plan"]["hec_items"]
    for r in (a, b):
        err = rel_errors(r["corr"], ref)
        print(f"baryon_small {prec} no split-K: max rel {err.max():.3e}")
        assert err.max() <= TOL[prec]
    assert np.array_equal(np.concatenate(a["corr"]).view(np.uint64),
                          np.concatenate(b["corr"]).view(np.uint64))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_rank4_general_contractions(rank4_small, prec):
    """General contractions through rank-4 intermediates: every schedule and
    batching mode, with and without split-K, against the oracle."""
    wl, ref = rank4_small
    from oracle import dag as OD
    d = OD.build(wl.leaves, wl.graphs)
    assert {W.C1, W.C2, W.C3} <= set(d.kind)
    base = None
    for policy, batched in (("input", False), ("tree", True), ("sibling", True)):
        r = run(wl, policy, prec, batched)
        err = rel_errors(r["corr"], ref)
        print(f"rank4_small {prec} {policy} batched={batched}: max rel {err.max():.3e}")
        assert err.max() <= TOL[prec]
        assert sum_errors(wl, r["sums"], ref) <= TOL[prec]
        bits = np.concatenate(r["corr"]).view(np.uint64)
        if base is None:
            base = bits
        assert np.array_equal(bits, base)
    r = run(wl, "tree", prec, True, tile=1, grid=0, lds_stages=1, split_k=0)
    err = rel_errors(r["corr"], ref)
    print(f"rank4_small {prec} 32x32 persistent, no split-K: max rel {err.max():.3e}")
    assert err.max() <= TOL[prec]


@pytest.mark.parametrize("in_situ", [False, True])
def test_autotune_then_parity(baryon_small, in_situ):
    wl, ref = baryon_small
    for prec in ("fp64", "fp32"):
        r = run(wl, "tree", prec, True, autotune=True, in_situ=in_situ)
        print(f"autotuned {prec} in_situ={in_situ}: {r['tuned']}")
        assert rel_errors(r["corr"], ref).max() <= TOL[prec]


def test_timed_execute_records_every_launch(baryon_small):
    """Timing mode: one record per kernel launch, carrying the plan's flops and
    bytes, and one per host transfer (the leaves start on the host here), in
    step order with the cross sum last; results unchanged."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    wl, ref = baryon_small
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    ctx.set_options(wave_lookahead=X.binding.LOOKAHEAD_ALL)
    runner = DeviceRunner(ctx, 0)
    ctx.set_timing(True)
    st = runner.run("fp64", True)
    records = ctx.launch_records()
    corr = ctx.fetch_correlators()
    ctx.close()
    moves = [r for r in records if r["type"] in ("h2d", "d2h")]
    recs = [r for r in records if r["type"] not in ("h2d", "d2h")]
    assert len(recs) == st["n_launches"]
    p = st["plan"]
    assert sum(r["type"] == "h2d" for r in moves) == p["n_h2d"] > 0
    assert sum(r["type"] == "d2h" for r in moves) == p["n_d2h"]
    assert sum(r["bytes"] for r in moves if r["type"] == "h2d") == p["h2d_bytes"]
    assert all(r["ms"] > 0 and r["flops"] == 0 and r["n_items"] == 1 for r in moves)
    assert [r["step"] for r in records[:-1]] == sorted(r["step"] for r in records[:-1])
    hec = [r for r in recs if r["type"] == "hec"]
    assert len(hec) == st["n_hec_launches"]
    assert sum(r["flops"] for r in hec) == st["hec_flops"]
    assert sum(r["bytes"] for r in hec) == st["hec_bytes"]
    hca = [r for r in recs if r["type"] == "hca"]
    # traces in launches of their own or carried by a contraction launch
    assert sum(r["flops"] + r["trace_flops"] for r in hec + hca) == pytest.approx(st["plan"]["flops"], rel=1e-12)
    assert sum(r["n_items"] for r in hca) + sum(r["trace_items"] for r in hec) == 3 * st["plan"]["n_roots"]
    assert any(r["type"] == "reduce" and r["kinds"] == [2] for r in recs)   # K33 split-K
    assert recs[-1]["type"] == "xsum" and recs[-1]["step"] == -1
    steps = [r["step"] for r in recs[:-1]]
    assert steps == sorted(steps)
    assert all(r["ms"] > 0 for r in recs)
    assert abs(sum(r["ms"] for r in hec) * 1e-3 - st["t_hec_s"]) <= 1e-9 * max(1, len(hec))
    assert rel_errors(corr, ref).max() <= TOL["fp64"]


def test_resident_leaves_and_graph_replay(baryon_small):
    wl, ref = baryon_small
    a = run(wl, "tree", "fp64", True, leaves_resident=True, use_graphs=True)
    b = run(wl, "tree", "fp64", True, leaves_resident=True, use_graphs=False)
    assert a["stats"]["n_graph_segments"] == 1 and b["stats"]["n_graph_segments"] == 0
    assert a["stats"]["plan"]["n_h2d"] == 0
    assert rel_errors(a["corr"], ref).max() <= TOL["fp64"]
    assert np.array_equal(np.concatenate(a["corr"]).view(np.uint64),
                          np.concatenate(b["corr"]).view(np.uint64))


@pytest.mark.parametrize("resident,budget_frac", [(True, None), (False, 4)])
def test_graph_replays_match_eager(meson_small, resident, budget_frac):
    """Captured segments replayed several times, with eager executes and host
    synchronisation in between; every replay must equal the eager result bit for bit."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    from oracle import dag as OD, schedules as OS
    wl, ref = meson_small
    d = OD.build(wl.leaves, wl.graphs)
    budget = None if budget_frac is None else OS.memsim(d, OS.input_order(d))["peak_live"] // budget_frac
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    ctx.set_mem_budget(budget)
    runner = DeviceRunner(ctx, 0)
    ctx.set_options(leaves_resident=resident, use_graphs=False)
    runner.run("fp64", True)
    eager = np.concatenate(ctx.fetch_correlators()).view(np.uint64).copy()
    assert rel_errors(ctx.fetch_correlators(), ref).max() <= TOL["fp64"]
    for rep in range(3):
        ctx.set_options(leaves_resident=resident, use_graphs=True)
        st = runner.run("fp64", True)
        assert st["n_graph_segments"] >= 1
        got = np.concatenate(ctx.fetch_correlators()).view(np.uint64)
        assert np.array_equal(got, eager), f"replay {rep}"
        runner.torch.cuda.synchronize()
        ctx.set_options(leaves_resident=resident, use_graphs=False)
        runner.run("fp64", True)            # eager work between replays
        assert np.array_equal(np.concatenate(ctx.fetch_correlators()).view(np.uint64), eager)
    ctx.close()


def _identity(nt, n):
    return np.broadcast_to(np.eye(n, dtype=np.complex128), (nt, n, n)).copy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_identity_trace_exact(prec):
    nt, n = 4, 48
    leaves = [W.Leaf(2, n, nt, _identity(nt, n)) for _ in range(4)]
    graphs = [W.GraphSpec([(W.K22, 0, 1), (W.K22, -1, 2), (W.HCA, -2, 3)], 0, 1.0),
              W.GraphSpec([(W.K22, 1, 2), (W.HCA, -1, 3)], 0, 1.0)]
    wl = W.Workload("identity", leaves, graphs)
    r = run(wl, "input", prec, False)
    for c in r["corr"]:
        assert np.array_equal(c, np.full(nt, n, dtype=np.complex128))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tile", [0, 1, 5])
def test_times_identity_and_selector(prec, tile):
    """X I and a selector tensor against the direct trace.  Tile 0 (64 x 64,
    four real products per complex one) reproduces the direct trace bit for
    bit: every product is by 0 or 1 and every sum adds zeros.  Tiles 1 and 5
    (Gauss's three products; tile 5 is the one the autotuner picks at N = 64)
    round Ar + Ai and then cancel Ar against it, so there the two agree only
    to rounding."""
    rng = np.random.default_rng(3)
    nt, n = 3, 24
    X2 = W._draw(rng, (nt, n, n), 0.5)
    Y2 = W._draw(rng, (nt, n, n), 0.5)
    X3 = W._draw(rng, (nt, n, n, n), 0.5)
    E = np.zeros((nt, n, n, n), dtype=np.complex128)
    for m in range(n):
        E[:, m, 0, m] = 1.0
    X3sel = np.ascontiguousarray(X3[:, :, :, 0])
    leaves = [W.Leaf(2, n, nt, X2), W.Leaf(2, n, nt, _identity(nt, n)), W.Leaf(2, n, nt, Y2),
              W.Leaf(3, n, nt, X3), W.Leaf(3, n, nt, E), W.Leaf(2, n, nt, X3sel)]
    graphs = [W.GraphSpec([(W.K22, 0, 1), (W.HCA, -1, 2)]),      # tr((X I) Y)
              W.GraphSpec([(W.HCA, 0, 2)]),                       # tr(X Y)
              W.GraphSpec([(W.K33, 3, 4), (W.HCA, -1, 2)]),      # tr(K33(X3, E) Y)
              W.GraphSpec([(W.HCA, 5, 2)])]                       # tr(X3[..,0] Y)
    wl = W.Workload("exact", leaves, graphs)
    r = run(wl, "input", prec, False, tile=tile)
    c = r["corr"]
    if tile == 0:
        assert np.array_equal(c[0], c[1])
        assert np.array_equal(c[2], c[3])
    else:
        bound = 1e-13 if prec == "fp64" else TOL[prec]
        assert rel_errors(c, {0: c[1], 2: c[3]}).max() <= bound
    if prec == "fp64":
        ref = OV.correlators(wl)
        assert rel_errors(c, ref).max() <= 1e-13


def test_deterministic_rerun(baryon_small):
    wl, _ = baryon_small
    a = run(wl, "tree", "fp32", True)
    b = run(wl, "tree", "fp32", True)
    assert np.array_equal(np.concatenate(a["corr"]).view(np.uint64),
                          np.concatenate(b["corr"]).view(np.uint64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_traces_with_mixed_n_in_one_launch(prec):
    """Roots with N = 10 (partial 4 x 4 blocks, masked loads) and N = 12 and 16
    (whole blocks, vector loads) in the same trace launch, and a DAG whose roots
    all have N a multiple of 4; both match the oracle."""
    rng = np.random.default_rng(21)
    nt = 3
    leaves, graphs = [], []
    for n in (10, 12, 16):
        base = len(leaves)
        leaves += [W.Leaf(2, n, nt, W._draw(rng, (nt, n, n), 0.5)) for _ in range(3)]
        graphs.append(W.GraphSpec([(W.K22, base, base + 1), (W.HCA, -1, base + 2)]))
        graphs.append(W.GraphSpec([(W.HCA, base + 2, base)]))
    for wl in (W.Workload("mixed_n", leaves, graphs),
               W.Workload("whole_n", leaves[3:], [W.GraphSpec([(k, l - 3 if l >= 0 else l, r - 3 if r >= 0 else r)
                                                               for k, l, r in g.ops]) for g in graphs[2:]])):
        ref = OV.correlators(wl)
        # every ready contraction joins the first wave, so the leaf-only roots
        # of all three N share one trace launch
        r = run(wl, "tree", prec, True, wave_lookahead=(1 << 63) - 1)
        assert r["stats"]["plan"]["n_steps"] == 2
        err = rel_errors(r["corr"], ref)
        print(f"{wl.name} {prec}: max rel {err.max():.3e}")
        assert err.max() <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("tile", [0, 1, 3, 5])
def test_xcd_item_order_with_nt_multiple_of_8(prec, tile):
    """Nt = 8 and 16 put contractions whose items start on a multiple of 8 on
    the XCD-aware item order (all tiles of a time slice on one XCD), ragged
    multi-tile contractions included (N = 40, K32 with 50 row tiles, K33 with
    K = 1600 split or not).  Results match the oracle and do not depend on
    grouping, whether or not the order applies to a contraction."""
    cases = [W.baryon_mix(n_bar=3, n_mes=3, nvec=40, nt=nt, n_graphs=8, sigma=1 / 16, n_corr=2,
                          seed=30 + nt, name=f"baryon_nt{nt}") for nt in (8, 16)]
    # general kinds C1..C3 through rank-4 intermediates (C3: K = 1000, split-K)
    cases.append(W.rank4_mix(n_bar=4, n_mes=3, n_r4=2, nvec=10, nt=8, n_graphs=16, seed=41, name="rank4_nt8"))
    for wl in cases:
        nt = wl.leaves[0].nt
        ref = OV.correlators(wl)
        for split_k in (1, 0):
            a = run(wl, "tree", prec, True, tile=tile, grid=1, split_k=split_k)
            b = run(wl, "tree", prec, False, tile=tile, grid=0, split_k=split_k)
            for r in (a, b):
                err = rel_errors(r["corr"], ref)
                assert err.max() <= TOL[prec], (nt, split_k, err.max())
            print(f"{wl.name} {prec} tile {tile} split_k {split_k}: max rel {err.max():.3e}")
            assert np.array_equal(np.concatenate(a["corr"]).view(np.uint64),
                                  np.concatenate(b["corr"]).view(np.uint64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("policy,look", [("input", 0), ("tree", 0), ("tree", 16)])
@pytest.mark.parametrize("mode", [1, 2])
def test_captured_transfer_segments_replay(meson_small, prec, policy, look, mode):
    """Captured graphs with spills and re-uploads (a quarter of the input-order
    live peak; mode 1: segments on one stream, mode 2: one graph over the
    compute, upload and spill streams), replayed five times with eager
    executes between replays: every replay equals the eager result bit for bit."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    from oracle import dag as OD, schedules as OS
    wl, ref = meson_small
    eb = 16 if prec == "fp64" else 8
    d = OD.build(wl.leaves, wl.graphs)
    budget = OS.memsim(d, OS.input_order(d), eb)["peak_live"] // 4
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule(policy)
    ctx.set_mem_budget(budget)
    runner = DeviceRunner(ctx, 0)
    ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=False)
    st = runner.run(prec, True)
    assert st["plan"]["n_d2h"] > 0 and st["plan"]["n_h2d"] > 0
    eager = np.concatenate(ctx.fetch_correlators()).view(np.uint64).copy()
    assert rel_errors(ctx.fetch_correlators(), ref).max() <= TOL[prec]
    for rep in range(5):
        ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=mode)
        st = runner.run(prec, True)
        assert st["n_graph_segments"] >= 1
        assert np.array_equal(np.concatenate(ctx.fetch_correlators()).view(np.uint64), eager), f"replay {rep}"
        ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=False)
        runner.run(prec, True)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nvec", [7, 12])
def test_trace_layouts(prec, nvec):
    """The root trace in both of its layouts: launches of at least 1024 traces
    (one wave per trace) and of fewer (one workgroup per trace), with N a
    multiple of 4 (vector loads) and not (masked loads): against the oracle,
    and the same bits from both layouts (waves of every ready contraction
    against one launch per contraction, on the same DAG)."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    for nt, many in ((64, True), (3, False)):
        wl = W.meson_ring(n_leaves=10, nvec=nvec, nt=nt, n_graphs=60, lmin=2, lmax=3, sigma=1 / 4, n_corr=3,
                          seed=41, name="trace_layouts")
        ref = OV.correlators(wl)
        ctx = X.Context()
        ctx.build_cdag(wl.leaves, wl.graphs)
        ctx.schedule("tree")
        ctx.set_trace_fusion(False)     # the trace kernel's own launches
        runner = DeviceRunner(ctx, 0)
        bits = []
        for batched in (True, False):
            ctx.set_options(leaves_resident=True, wave_lookahead=X.binding.LOOKAHEAD_ALL, use_graphs=0)
            ctx.set_timing(True)
            runner.run(prec, batched)
            items = [r["n_items"] for r in ctx.launch_records() if r["type"] == "hca"]
            assert (max(items) >= 1024) == (many and batched), items
            err = rel_errors(ctx.fetch_correlators(), ref)
            print(f"N={nvec} nt={nt} {prec} batched={batched}: trace launches of at most {max(items)}, "
                  f"max rel {err.max():.3e}")
            assert err.max() <= TOL[prec]
            bits.append(np.concatenate(ctx.fetch_correlators()).view(np.uint64).copy())
        assert np.array_equal(bits[0], bits[1])
        ctx.close()


def test_resident_leaves_after_a_host_leaf_execute(meson_small):
    """A plan with the leaves on the host uses the memory where a resident
    plan keeps them; the resident execute that follows uploads them again and
    gives the same bits as before."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    from oracle import dag as OD, schedules as OS
    wl, ref = meson_small
    d = OD.build(wl.leaves, wl.graphs)
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    runner = DeviceRunner(ctx, 0)
    ctx.set_options(leaves_resident=True, wave_lookahead=16, use_graphs=0)
    runner.run("fp64", True)
    first = np.concatenate(ctx.fetch_correlators()).view(np.uint64).copy()
    ctx.set_mem_budget(OS.memsim(d, OS.input_order(d), 16)["peak_live"] // 4)
    ctx.set_options(leaves_resident=False, wave_lookahead=16, use_graphs=0)
    runner.run("fp64", True)
    assert rel_errors(ctx.fetch_correlators(), ref).max() <= TOL["fp64"]
    ctx.set_options(leaves_resident=True, wave_lookahead=16, use_graphs=0)
    runner.run("fp64", True)
    again = np.concatenate(ctx.fetch_correlators()).view(np.uint64)
    ctx.close()
    assert np.array_equal(first, again)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_trace_fusion(meson_small, rank4_small, prec):
    """Trace fusion (a step's root traces ride in one of its contraction
    launches): the same bits as separate trace launches for every tile shape
    (a 64-thread workgroup carries one trace as one wave, a 256-thread one one
    trace, a 512-thread one two, with an idle group when the count is odd),
    with leaves resident and under a budget that forces spills, in each issue
    mode; the launch records carry every trace exactly once."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    from oracle import dag as OD, schedules as OS
    ALL = X.binding.LOOKAHEAD_ALL
    eb = 16 if prec == "fp64" else 8
    for wl, ref in (meson_small, rank4_small):
        d = OD.build(wl.leaves, wl.graphs)
        budget = OS.memsim(d, OS.input_order(d), eb)["peak_live"] // 4 if wl.name == "meson_small" else None
        ctx = X.Context()
        ctx.build_cdag(wl.leaves, wl.graphs)
        ctx.schedule("tree")
        runner = DeviceRunner(ctx, 0)
        nt = wl.leaves[0].nt
        for tile in (0, 1, 2, 4, 5):
            for n in {lf.nvec for lf in wl.leaves}:
                for kind in (0, 1, 2, 4, 5, 6):
                    ctx.set_tile(prec, kind, n, tile, 1, 1, 1)
            for resident, bud, look, mode in ((True, None, ALL, 0), (False, budget, 16, 1), (False, budget, 16, 2)):
                bits = []
                for fuse in (False, True):
                    ctx.set_trace_fusion(fuse)
                    ctx.set_mem_budget(bud)
                    ctx.set_options(leaves_resident=resident, wave_lookahead=look, use_graphs=mode)
                    runner.run(prec, True)
                    corr = ctx.fetch_correlators()
                    assert rel_errors(corr, ref).max() <= TOL[prec], (wl.name, tile, resident, mode, fuse)
                    bits.append(np.concatenate(corr).view(np.uint64).copy())
                assert np.array_equal(bits[0], bits[1]), (wl.name, prec, tile, resident, mode)
            ctx.set_trace_fusion(True)
            ctx.set_mem_budget(None)
            ctx.set_options(leaves_resident=True, wave_lookahead=ALL, use_graphs=0)
            ctx.set_timing(True)
            st = runner.run(prec, True)
            recs = [r for r in ctx.launch_records() if r["type"] not in ("h2d", "d2h")]
            ctx.set_timing(False)
            carried = sum(r["trace_items"] for r in recs if r["type"] == "hec")
            alone = sum(r["n_items"] for r in recs if r["type"] == "hca")
            print(f"{wl.name} {prec} tile {tile}: {carried} traces carried, {alone} in trace launches, "
                  f"{len(recs)} launches")
            assert carried > 0 and carried + alone == st["plan"]["n_roots"] * nt
            assert all(3 in r["kinds"] for r in recs if r["trace_items"] > 0)
            assert all(r["trace_items"] == 0 for r in recs if r["type"] != "hec")
            total = sum(r["flops"] + r["trace_flops"] for r in recs)
            assert abs(total - st["plan"]["flops"]) <= 1e-9 * st["plan"]["flops"]
        ctx.set_trace_fusion(False)
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_degenerate_dags(prec):
    """Edge cases of the method: a DAG of leaves with no graph; roots that
    trace two leaves directly (no contraction); N = 1 and Nt = 1 (every tile
    ragged, K = 1); N = 3 (partial trace blocks); a graph given twice (one
    shared root, two outputs) and the same leaves traced in both orders."""
    rng = np.random.default_rng(21)
    empty = W.Workload("leaves_only", [W.Leaf(2, 4, 2, W._draw(rng, (2, 4, 4), 0.5))], [])
    r = run(empty, "tree", prec, False)
    assert r["corr"] == [] and r["sums"] == []
    assert r["stats"]["plan"]["n_contr"] == 0

    for n, nt in ((1, 1), (3, 2)):
        m = [W.Leaf(2, n, nt, W._draw(rng, (nt, n, n), 0.5)) for _ in range(3)]
        b = [W.Leaf(3, n, nt, W._draw(rng, (nt, n, n, n), 0.5)) for _ in range(2)]
        leaves = m + b
        ring = [(W.K22, 0, 1), (W.K22, -1, 2), (W.HCA, -2, 0)]
        chain = [(W.K32, 3, 0), (W.K33, -1, 4), (W.HCA, -2, 1)]
        graphs = [W.GraphSpec([(W.HCA, 0, 1)], 0, 1.0),
                  W.GraphSpec([(W.HCA, 1, 0)], 0, -1.0),
                  W.GraphSpec(ring, 1, 1.0),
                  W.GraphSpec(list(ring), 1, 0.5),
                  W.GraphSpec(chain, 2, 1.0)]
        wl = W.Workload(f"degenerate_n{n}", leaves, graphs)
        ref = OV.correlators(wl)
        for policy in ("input", "tree"):
            r = run(wl, policy, prec, False)
            err = rel_errors(r["corr"], ref)
            print(f"degenerate N={n} Nt={nt} {prec} {policy}: max rel {err.max():.3e}")
            assert err.max() <= TOL[prec]
            assert np.array_equal(r["corr"][2], r["corr"][3])
            assert sum_errors(wl, r["sums"], ref) <= TOL[prec]
            assert r["stats"]["plan"]["n_contr"] == 2 + 3 + 3    # two traces, one shared ring, chain


def test_recorded_walk_is_the_executed_walk(meson_small):
    """The eager execute issues its transfers and kernels in the order that
    cdag_trace_execute records without a GPU (the walk the CPU race check
    covers): same transfers (direction, step, bytes) in the same order, and
    kernels in the same steps."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    from oracle import dag as OD, schedules as OS
    wl, ref = meson_small
    d = OD.build(wl.leaves, wl.graphs)
    budget = OS.memsim(d, OS.input_order(d), 16)["peak_live"] // 4
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    ctx.set_mem_budget(budget)
    ctx.set_options(leaves_resident=False, wave_lookahead=0, use_graphs=False)
    runner = DeviceRunner(ctx, 0)
    for batched in (False, True):
        trace = ctx.trace_execute("fp64", batched)
        ctx.set_timing(True)
        runner.run("fp64", batched)
        recs = ctx.launch_records()
        ctx.set_timing(False)
        corr = ctx.fetch_correlators()
        assert rel_errors(corr, ref).max() <= TOL["fp64"]
        want = [("d2h" if r["space"] == "spill" else "h2d", r["step"], r["bytes"])
                for r in trace if r["op"] == "write" and r["stream"] in (1, 2)]
        got = [(r["type"], r["step"], int(r["bytes"])) for r in recs if r["type"] in ("h2d", "d2h")]
        assert got == want and len(got) > 0
        assert sorted({r["step"] for r in trace if r["stream"] == 0 and r["op"] == "read"}) == \
            sorted({r["step"] for r in recs if r["type"] in ("hec", "hca", "reduce")})
    ctx.close()


def _wl_meson_nt4():
    # N = 72 (ragged tiles), Nt = 4 (two or four passes over the time slices)
    return W.meson_ring(n_leaves=8, nvec=72, nt=4, n_graphs=30, lmin=4, lmax=7, sigma=1 / 8,
                        n_corr=2, seed=15, name="meson_nt4")


def _wl_baryon_nt4():
    # N = 40: ragged tiles, split-K K33 (K = 1600)
    return W.baryon_mix(n_bar=4, n_mes=4, nvec=40, nt=4, n_graphs=12, sigma=1 / 16, n_corr=2,
                        seed=16, name="baryon_nt4")


@pytest.fixture(scope="module")
def nt4_workloads():
    out = []
    for wl in (_wl_meson_nt4(), _wl_baryon_nt4()):
        out.append((wl, OV.correlators(wl)))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_time_slice_passes_and_stream_modes(nt4_workloads, prec, mode):
    """Passes over slices of the time axis (2 and 4 passes, alternating halves
    of the arena and of the spill pool) under a budget that forces spills, in
    an issue mode (0: eager on three streams, 1: one-stream captured segments,
    2: one graph over the three streams' work with explicit edges), per
    contraction and in waves: correlators equal the single-pass run bit for
    bit, plan counters equal the oracle's."""
    from oracle import dag as OD, schedules as OS
    eb = 16 if prec == "fp64" else 8
    for wl, ref in nt4_workloads:
        d = OD.build(wl.leaves, wl.graphs)
        live = OS.memsim(d, OS.input_order(d), eb)["peak_live"]
        base = run(wl, "tree", prec, True)
        assert rel_errors(base["corr"], ref).max() <= TOL[prec]
        want = np.concatenate(base["corr"]).view(np.uint64)
        # a fraction of the input-order live peak (per pass: of its slices)
        fracs = (4, 4, 3) if wl.name == "meson_nt4" else (2, 2, 2)
        for chunks, frac in zip((1, 2, 4), fracs):
            budget = 2 * live // (frac * chunks) if chunks > 1 else live // frac
            for batched, look in ((False, 0), (True, 0), (True, 16)):
                _, _, o = oracle_plan_counts(wl, "tree", eb, budget, batched, lookahead=look, t_chunks=chunks)
                print(f"{wl.name} {prec} passes={chunks} batched={batched} look={look} mode={mode}", flush=True)
                r = run(wl, "tree", prec, batched, budget=budget, wave_lookahead=look, use_graphs=mode,
                        t_chunks=chunks)
                p = r["stats"]["plan"]
                for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "n_steps"):
                    assert p[k] == o[k], (wl.name, chunks, batched, look, mode, k)
                got = np.concatenate(r["corr"]).view(np.uint64)
                print(f"  steps={p['n_steps']} evict={p['n_evict']} d2h={p['n_d2h']}")
                assert np.array_equal(got, want), (wl.name, chunks, batched, look, mode)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_index_pair_contractions(prec):
    """Contractions over other index pairs and output orders (the general
    kernel: index-mapped loads and stores), beside named and general kinds,
    N = 7 (ragged tiles) and N = 16, in every schedule, waves and one launch
    per contraction, under a budget that forces spills: against the oracle,
    identical bits across schedules and batching."""
    from oracle import dag as OD, schedules as OS
    for nvec, nt in ((7, 3), (16, 2)):
        wl = W.pairs_mix(nvec=nvec, nt=nt, n_graphs=40, seed=50 + nvec)
        ref = OV.correlators(wl)
        d = OD.build(wl.leaves, wl.graphs, wl.specs)
        assert any(k >= W.SPEC_BASE for k in d.kind)
        eb = 16 if prec == "fp64" else 8
        budget = OS.memsim(d, OS.input_order(d), eb)["peak_live"] // 2
        base = None
        for policy, batched, look, bud in (("input", False, 0, None), ("tree", True, 0, None),
                                           ("tree", True, 1 << 62, None), ("sibling", True, 16, budget),
                                           ("node", False, 0, budget)):
            r = run(wl, policy, prec, batched, budget=bud, wave_lookahead=look)
            err = rel_errors(r["corr"], ref)
            print(f"pairs N={nvec} {prec} {policy} batched={batched} look={look} budget={bud}: "
                  f"max rel {err.max():.3e}")
            assert err.max() <= TOL[prec]
            assert sum_errors(wl, r["sums"], ref) <= TOL[prec]
            bits = np.concatenate(r["corr"]).view(np.uint64)
            if base is None:
                base = bits
            assert np.array_equal(bits, base)


def test_index_pair_contractions_refused_in_split_bf16():
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd import binding as B
    wl = W.pairs_mix(nvec=5, nt=2, n_graphs=10, seed=3)
    with pytest.raises(X.CdagError) as e:
        run(wl, "tree", "bf16x3", True)
    assert e.value.code == B.E_INVALID
