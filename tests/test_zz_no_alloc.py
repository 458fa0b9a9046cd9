"""The entry point that allocates nothing (cdag_execute_static) against
execute on the GPU: the same plan gives the same correlators bit for bit, on
two calls in a row, the second with a smaller DAG (the static scratch keeps the
first call's contents)."""
import numpy as np
import pytest

from synth import workloads as W
from oracle import values as OV

from gpu_util import rel_errors

pytestmark = pytest.mark.gpu


def _run_both(wl, prec, batched, policy="tree", budget=None, look=0, resident=False):
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule(policy)
    ctx.set_mem_budget(budget)
    ctx.set_options(leaves_resident=resident, wave_lookahead=look, use_graphs=0)
    runner = DeviceRunner(ctx, 0)
    a = runner.run(prec, batched)
    want = [c.copy() for c in ctx.fetch_correlators()]
    want_sums = [c.copy() for c in ctx.fetch_sums()]
    ctx.plan(prec, batched)
    b = ctx.execute_static(prec, batched)
    got = ctx.fetch_correlators()
    got_sums = ctx.fetch_sums()
    ctx.close()
    return a, b, want, want_sums, got, got_sums


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_static_execute_matches_execute_twice(prec):
    import paper_2511_02257_amd as X
    # first call: ragged baryon chains with split-K K33 (the workspace is scratch)
    big = W.baryon_mix(n_bar=4, n_mes=4, nvec=40, nt=3, n_graphs=12, sigma=1 / 16, n_corr=2, seed=12,
                       name="baryon_small")
    # second call, smaller: meson rings with ragged tiles and waves
    small = W.meson_ring(n_leaves=6, nvec=24, nt=2, n_graphs=10, lmin=3, lmax=6, sigma=1 / 8, n_corr=2,
                         seed=13, name="meson_smaller")
    sizes = []
    for wl, batched, resident in ((big, True, False), (small, False, True)):
        a, b, want, want_sums, got, got_sums = _run_both(wl, prec, batched, resident=resident)
        sizes.append(b["arena_highwater"])
        assert b["arena_highwater"] <= X.binding.STATIC_SCRATCH_BYTES
        for x, y in zip(want, got):
            assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
        for x, y in zip(want_sums, got_sums):
            assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
        assert b["plan"]["n_h2d"] == a["plan"]["n_h2d"] and b["n_launches"] == a["n_launches"]
        ref = OV.correlators(wl)
        tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 4e-5}[prec]
        assert rel_errors(got, ref).max() <= tol
    assert sizes[1] < sizes[0]


def test_static_execute_refuses_what_it_cannot_hold():
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd import binding as B
    from paper_2511_02257_amd.device import DeviceRunner
    wl = W.meson_ring(n_leaves=6, nvec=24, nt=2, n_graphs=10, lmin=3, lmax=6, seed=13)
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    ctx.schedule("tree")
    runner = DeviceRunner(ctx, 0)  # noqa: F841  (keeps the streams alive)
    with pytest.raises(X.CdagError) as e:        # no plan made for it yet
        ctx.execute_static("fp64", True)
    assert e.value.code == B.E_STATE
    big = W.baryon_mix(n_bar=4, n_mes=4, nvec=64, nt=8, n_graphs=6, seed=14)   # 128 MiB leaves
    ctx.build_cdag(big.leaves, big.graphs)
    ctx.schedule("tree")
    ctx.plan("fp64", True)
    with pytest.raises(X.CdagError) as e:
        ctx.execute_static("fp64", True)
    assert e.value.code == B.E_NOMEM and "static scratch" in str(e.value)
    ctx.close()
