"""Helpers for the GPU parity tests: run a workload through the C ABI on cuda:0
and measure errors against the oracle."""
from __future__ import annotations

import numpy as np

from oracle import dag as OD
from oracle import schedules as OS
from oracle import values as OV


def run(wl, policy="tree", prec="fp64", batched=False, budget=None, leaves_resident=False,
        use_graphs=True, wave_max=4096, wave_lookahead=0, device=0, tile=None, grid=1,
        lds_stages=2, split_k=1, autotune=False, in_situ=False, t_chunks=1):
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs, getattr(wl, "specs", ()))
    order = ctx.schedule(policy)
    ctx.set_mem_budget(budget)
    ctx.set_options(leaves_resident=leaves_resident, wave_max=wave_max,
                    wave_lookahead=wave_lookahead, use_graphs=use_graphs)
    ctx.set_time_chunks(t_chunks)
    if tile is not None:
        for lf_n in {lf.nvec for lf in wl.leaves}:
            for kind in (0, 1, 2, 4, 5, 6):
                ctx.set_tile(prec, kind, lf_n, tile, grid, lds_stages, split_k)
    runner = DeviceRunner(ctx, device)
    tuned = None
    if autotune:
        runner.autotune(prec, batched, reps=2, in_situ=in_situ)
        tuned = {(k, n): ctx.get_tile(prec, k, n) for n in {lf.nvec for lf in wl.leaves} for k in (0, 1, 2, 4, 5, 6)}
    st = runner.run(prec, batched)
    corr = ctx.fetch_correlators()
    sums = ctx.fetch_sums()
    ctx.close()
    return dict(order=order, stats=st, corr=corr, sums=sums, tuned=tuned)


def rel_errors(corr, ref):
    """Per graph ||C - C_ref||_2 / ||C_ref||_2 over t."""
    out = []
    for g, r in ref.items():
        out.append(np.linalg.norm(corr[g] - r) / np.linalg.norm(r))
    return np.array(out)


def sum_errors(wl, sums, ref_vals):
    """Cross-diagram sums: |S - S_ref| / sum_g |w_g C_g| per t (condition-aware)."""
    ref = OV.cross_sums(wl, ref_vals)
    scale = OV.cross_sum_scale(wl, ref_vals)
    worst = 0.0
    for c, s in ref.items():
        worst = max(worst, float(np.max(np.abs(sums[c] - s) / scale[c])))
    return worst


def oracle_plan_counts(wl, policy, elem_bytes, budget, batched, leaves_resident=False, lookahead=0,
                       t_chunks=1):
    from oracle import planner as OP
    d = OD.build(wl.leaves, wl.graphs, getattr(wl, "specs", ()))
    order = OS.schedule(d, policy, elem_bytes)
    res = OP.plan(d, order, elem_bytes=elem_bytes,
                  budget=OP.UNLIMITED if budget is None else budget,
                  batched=batched, leaves_resident=leaves_resident, lookahead=lookahead,
                  t_chunks=t_chunks)
    return d, order, res
