"""GPU parity at full size (marked gpu): the meson and baryon workloads in the
launch configurations bench.py times, against the oracle.

The meson workload's 2000 correlators are all computed by the oracle (a few
seconds); the baryon workload's by sampling graphs the oracle evaluates one by
one.  Plan counters must equal the stored oracle values
(tests/golden/full_configs.json, written by make_full_configs.py).
"""
import json
import os

import numpy as np
import pytest

from synth import workloads as W
from oracle import values as OV

from gpu_util import run, rel_errors, sum_errors, oracle_plan_counts

pytestmark = pytest.mark.gpu

ALL = (1 << 63) - 1
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_configs.json")))


@pytest.fixture(scope="module")
def meson():
    wl = W.config("meson_ring")
    return wl, OV.correlators(wl)


def test_meson_ring_full_fp64_bench_configuration(meson):
    wl, ref = meson
    r = run(wl, "tree", "fp64", True, leaves_resident=True, wave_lookahead=ALL, use_graphs=True)
    err = rel_errors(r["corr"], ref)
    print(f"meson_ring fp64 resident waves={r['stats']['plan']['n_steps']} max rel {err.max():.3e}")
    assert err.max() <= 1e-12
    assert sum_errors(wl, r["sums"], ref) <= 1e-12
    # the budgeted run (leaves on the host, a quarter of the input-order live peak)
    gold = GOLD["meson_ring"]
    b = run(wl, "tree", "fp64", True, budget=gold["budget"], wave_lookahead=0)
    p = b["stats"]["plan"]
    for k, v in gold["policies"]["tree"]["plans"]["waves"].items():
        assert p[k] == v, k
    assert np.array_equal(np.concatenate(b["corr"]).view(np.uint64),
                          np.concatenate(r["corr"]).view(np.uint64))
    # the node-gain order under the same budget, waves with lookahead 16 and
    # captured segments: same bits
    n = run(wl, "node", "fp64", True, budget=gold["budget"], wave_lookahead=16)
    assert n["stats"]["plan"]["n_evict"] > 0
    assert np.array_equal(np.concatenate(n["corr"]).view(np.uint64),
                          np.concatenate(r["corr"]).view(np.uint64))
    # the bench's fastest budgeted form: 16 passes over the time slices with
    # lookahead 384, captured segments; plan counters equal the oracle's
    _, _, o = oracle_plan_counts(wl, "tree", 16, gold["budget"], True, lookahead=384, t_chunks=16)
    c = run(wl, "tree", "fp64", True, budget=gold["budget"], wave_lookahead=384, t_chunks=16)
    p = c["stats"]["plan"]
    for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "n_steps"):
        assert p[k] == o[k], k
    assert np.array_equal(np.concatenate(c["corr"]).view(np.uint64),
                          np.concatenate(r["corr"]).view(np.uint64))


# Split-BF16 with two pieces misses 1e-5 on the longest meson rings (about
# 1.6e-5 measured): its bound here is 4e-5; three pieces meet 1e-5.
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 4e-5), ("bf16x6", 1e-5)])
def test_meson_ring_full_mixed(meson, prec, tol):
    wl, ref = meson
    r = run(wl, "tree", prec, True, leaves_resident=True, wave_lookahead=ALL, use_graphs=True)
    err = rel_errors(r["corr"], ref)
    print(f"meson_ring {prec}: max rel {err.max():.3e} median {np.median(err):.3e} "
          f"p99 {np.quantile(err, 0.99):.3e}")
    assert err.max() <= tol
    assert sum_errors(wl, r["sums"], ref) <= tol


@pytest.fixture(scope="module")
def baryon():
    """Sample: for every distinct K32 output X = K32(B_a, M_b) of the DAG the
    first graph that uses it, so that each is compared at least once, plus ten
    seeded graphs."""
    wl = W.config("baryon_mix")
    first = {}
    for g, spec in enumerate(wl.graphs):
        first.setdefault(tuple(spec.ops[0]), g)
    rng = np.random.default_rng(77)
    sample = sorted(set(first.values()) | {int(g) for g in rng.choice(len(wl.graphs), size=10, replace=False)})
    return wl, sample, OV.correlators(wl, sample)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-5), ("bf16x6", 1e-5)])
def test_baryon_mix_full_sampled(baryon, prec, tol):
    wl, sample, ref = baryon
    budget = 32 * 10**9 if prec == "fp64" else 16 * 10**9
    r = run(wl, "tree", prec, True, budget=budget, wave_lookahead=0)
    p = r["stats"]["plan"]
    if prec == "fp64":
        for k, v in GOLD["baryon_mix"]["policies"]["tree"]["plans"]["waves"].items():
            assert p[k] == v, k
    err = np.array([np.linalg.norm(r["corr"][g] - ref[g]) / np.linalg.norm(ref[g]) for g in sample])
    print(f"baryon_mix {prec}: waves={p['n_steps']} max rel {err.max():.3e} median {np.median(err):.3e} "
          f"device {r['stats']['t_device_s'] * 1e3:.1f} ms, {p['flops'] / r['stats']['t_device_s'] / 1e12:.1f} TFLOP/s")
    assert err.max() <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-5), ("bf16x6", 1e-5)])
def test_baryon_mix_headline_configuration(baryon, prec, tol):
    """The launch configuration of the bench's headline and precision-form
    rows: 8 passes over the time slices, every ready contraction in a wave,
    a 32e9 B budget, leaves in pinned host memory, eager issue on three
    streams, the bench's kernel choices (FP64: 64x64 tiles of 512 threads, one
    LDS stage, K33 without split-K; the other modes tuned in situ).  Plan
    counters equal the oracle's; the sampled correlators are within the bound."""
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    wl, sample, ref = baryon
    budget = 32 * 10**9
    _, _, o = oracle_plan_counts(wl, "tree", 16 if prec == "fp64" else 8, budget, True, lookahead=ALL, t_chunks=8)
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    ctx.set_mem_budget(budget)
    ctx.set_time_chunks(8)
    ctx.set_options(leaves_resident=False, wave_lookahead=ALL, use_graphs=0)
    runner = DeviceRunner(ctx, 0)
    if prec == "fp64":
        ctx.set_tile("fp64", W.K32, 64, 5, 1, 1, 1)
        ctx.set_tile("fp64", W.K33, 64, 5, 1, 1, 0)
    else:
        runner.autotune(prec, True, reps=1, in_situ=True)
    st = runner.run(prec, True)
    p = st["plan"]
    for k in ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "n_steps"):
        assert p[k] == o[k], k
    corr = ctx.fetch_correlators()
    ctx.close()
    err = np.array([np.linalg.norm(corr[g] - ref[g]) / np.linalg.norm(ref[g]) for g in sample])
    print(f"baryon_mix headline configuration {prec}: steps={p['n_steps']} h2d={p['h2d_bytes'] / 1e9:.2f} GB "
          f"max rel {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= tol


@pytest.fixture(scope="module")
def batched():
    wl = W.config("batched")
    # one ring and one chain from each N family (graphs alternate by family round-robin)
    nf = len(W.BATCHED_NVECS)
    sample = []
    for f in range(nf):
        fam = [g for g in range(f, len(wl.graphs), nf)]
        ring = next(g for g in fam if wl.graphs[g].ops[0][0] == W.K22)
        chain = next(g for g in fam if wl.graphs[g].ops[0][0] == W.K32)
        sample += [ring, chain]
    return wl, sorted(sample), OV.correlators(wl, sorted(sample))


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-5), ("bf16x6", 1e-5)])
def test_batched_full_sampled(batched, prec, tol):
    """Five N families, just over 20,000 merged contractions, complex64 storage,
    64 GB budget: waves of every ready contraction, captured segments, autotuned tiles."""
    wl, sample, ref = batched
    r = run(wl, "tree", prec, True, budget=64 * 10**9, wave_lookahead=ALL, autotune=True)
    p = r["stats"]["plan"]
    assert p["n_contr"] >= 20000
    err = np.array([np.linalg.norm(r["corr"][g] - ref[g]) / np.linalg.norm(ref[g]) for g in sample])
    fams = [wl.leaves[wl.graphs[g].ops[0][1]].nvec for g in sample]
    print(f"batched {prec}: contractions={p['n_contr']} waves={p['n_steps']} evict={p['n_evict']} "
          f"h2d={p['h2d_bytes'] / 1e9:.2f} GB peak={p['peak_resident'] / 1e9:.2f} GB "
          f"device {r['stats']['t_device_s'] * 1e3:.1f} ms total {r['stats']['t_total_s'] * 1e3:.1f} ms "
          f"{p['flops'] / r['stats']['t_device_s'] / 1e12:.1f} TFLOP/s tiles {r['tuned']}")
    for n, e in zip(fams, err):
        print(f"   N={n}: rel {e:.3e}")
    assert err.max() <= tol


def test_batched_per_contraction_matches_waves(batched):
    wl, sample, ref = batched
    a = run(wl, "tree", "fp32", False, budget=64 * 10**9)
    b = run(wl, "tree", "fp32", True, budget=64 * 10**9, wave_lookahead=ALL)
    # the bench's passes form: 8 passes over the time slices, every ready
    # contraction in a wave, eager issue
    c = run(wl, "tree", "fp32", True, budget=64 * 10**9, wave_lookahead=ALL, use_graphs=False, t_chunks=8)
    assert c["stats"]["plan"]["n_evict"] == 0
    for g in sample:
        assert np.array_equal(a["corr"][g].view(np.uint64), b["corr"][g].view(np.uint64))
        assert np.array_equal(c["corr"][g].view(np.uint64), b["corr"][g].view(np.uint64))
    ta, tb = a["stats"]["t_total_s"], b["stats"]["t_total_s"]
    print(f"batched fp32: per-contraction {ta * 1e3:.1f} ms ({a['stats']['n_launches']} launches), "
          f"waves {tb * 1e3:.1f} ms ({b['stats']['n_launches']} launches)")


@pytest.fixture(scope="module")
def tritium():
    """The Table corr-func tritium-shaped DAG (BxBxB, N = 32, 6085 graphs merged
    into 7588 contractions through rank-4 intermediates: C1 of two baryons,
    the O(N^5) step, then C2 and K33) with seeded entries and Nt = 2.  Sample:
    graphs that together use every distinct C1 -> C2 pair of the DAG, plus ten
    seeded ones."""
    from synth import corr_func as CF
    wl = CF.with_data(CF.corr_func_like("tritium", nt=2))
    keys, sample = set(), []
    for g, spec in enumerate(wl.graphs):
        ops = spec.ops
        mine = set()
        for i, (k, l, r) in enumerate(ops):
            if k == W.C2 and r >= 0 and ops[-l - 1][0] == W.C1:
                mine.add((ops[-l - 1][1], ops[-l - 1][2], r))
        if mine - keys:
            keys |= mine
            sample.append(g)
    rng = np.random.default_rng(78)
    sample = sorted(set(sample) | {int(g) for g in rng.choice(len(wl.graphs), size=10, replace=False)})
    return wl, sample, OV.correlators(wl, sample)


# Split-BF16 with two pieces carries up to ~3 * 2^-16 relative error per
# product; the tritium-shaped chains run six to seven contractions deep on both
# sides of the trace (measured 5.5e-5), so its bound here is 1e-4.
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-4), ("bf16x6", 1e-5)])
def test_tritium_shaped_full(tritium, prec, tol):
    wl, sample, ref = tritium
    r = run(wl, "tree", prec, True, wave_lookahead=ALL, autotune=True)
    p = r["stats"]["plan"]
    assert p["n_contr"] == 7588
    err = np.array([np.linalg.norm(r["corr"][g] - ref[g]) / np.linalg.norm(ref[g]) for g in sample])
    print(f"tritium-shaped {prec}: {p['n_contr']} contractions, waves={p['n_steps']}, sample {len(sample)} graphs, "
          f"max rel {err.max():.3e} median {np.median(err):.3e}, device {r['stats']['t_device_s'] * 1e3:.1f} ms")
    assert err.max() <= tol
    if prec == "fp64":
        # default kernel choices: waves and one contraction per step give the
        # same bits (split counts do not depend on grouping)
        a = run(wl, "tree", prec, True, wave_lookahead=ALL)
        b = run(wl, "input", prec, False)
        for g in sample:
            assert np.array_equal(a["corr"][g].view(np.uint64), b["corr"][g].view(np.uint64))
            assert np.linalg.norm(a["corr"][g] - ref[g]) / np.linalg.norm(ref[g]) <= tol
