"""Benchmark: contraction-DAG execution on one MI355X.

Workload (the memory-bound meson configuration): 16 meson leaves, complex128
[Nt=32][64][64], entries N(0,1)/8; 2000 seeded ring traces of 4..8 distinct
leaves contracted as random binary trees, common sub-products merged.

One step = one execute() of the whole scheduled DAG: every exterior
contraction (grouped per wave), every root trace, the FP64 cross-diagram sums
and the copy of all correlators to the host.  The DAG is built, scheduled
(Tree) and planned once; the schedule is reused by every step, as the paper
reuses a schedule across runs.  `value` is algorithmic complex TFLOP/s (8 flops
per complex multiply-add) with the leaves already resident in HBM.

The same line also reports: the budgeted runs (HBM budget = a quarter of the
input-order schedule's live peak, leaves starting in pinned host memory,
spills and re-uploads over PCIe) for the input-order, Sibling, Tree and node-gain
schedules: time-to-solution, H2D/D2H GB, evictions, peak resident bytes; the
host-transfer rates beside a pinned-copy link reference; the memory of the
headline run (arena, live peak, H2D per step); the FP32 and split-BF16 modes;
per-contraction launches vs waves; the roofline of the exterior-contraction
kernel; and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CDAG time-to-solution, complex TFLOP/s, H2D GB, peak HBM (FP64 vs mixed)"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}   # TFLOP/s per algorithmic flop
HBM_PEAK = 8000.0   # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(ctx, runner, prec, batched, steps, warmup):
    for _ in range(warmup):
        runner.run(prec, batched)
    torch = runner.torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        st = runner.run(prec, batched)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, st


def measured_traffic(variant):
    """HBM bytes per launch of the exterior-contraction kernel from the committed
    counter summary, or None when the kernel source or variant differs from the
    one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", "hec_traffic_meson_ring.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_2511_02257_amd.profiling import kernel_source_sha256
    if rec.get("kernel_sha256") != kernel_source_sha256():
        return None
    entry = rec.get("variants", {}).get(str(variant))
    return None if entry is None else entry.get("traffic_bytes_per_launch")


KIND_NAMES = {0: "K22", 1: "K32", 2: "K33", 3: "HCA", 4: "C1", 5: "C2", 6: "C3"}


def kernel_table(records, prec):
    """Launch records of one timed execute, summed per (launch type, kinds):
    time, algorithmic flops and bytes, and the rates against the MI355X peaks.
    A split-K contraction kind also gets an entry that charges its reduction
    kernels to it ("hec+reduce")."""
    agg = {}
    for r in records:
        if r["type"] in ("h2d", "d2h"):
            continue
        key = r["type"] if r["type"] == "xsum" else r["type"] + ":" + "+".join(KIND_NAMES[k] for k in r["kinds"])
        a = agg.setdefault(key, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
        a["launches"] += 1
        a["ms"] += r["ms"]
        a["flops"] += r["flops"]
        a["bytes"] += r["bytes"]
    for key in [k for k in agg if k.startswith("reduce:")]:
        hk = "hec:" + key.split(":", 1)[1]
        if hk in agg:
            agg["hec+reduce:" + key.split(":", 1)[1]] = {
                "launches": agg[hk]["launches"] + agg[key]["launches"],
                "ms": agg[hk]["ms"] + agg[key]["ms"], "flops": agg[hk]["flops"],
                "bytes": agg[hk]["bytes"]}
    for key, a in agg.items():
        sec = a["ms"] * 1e-3
        if sec <= 0:
            continue
        a["TFLOP/s"] = round(a["flops"] / sec / 1e12, 3)
        a["GB/s"] = round(a["bytes"] / sec / 1e9, 1)
        if key.startswith("hec"):
            a["frac_mfma"] = round(a["flops"] / sec / 1e12 / PEAK[prec], 4)
        if not key.startswith("reduce"):
            a["frac_hbm"] = round(a["bytes"] / sec / 1e9 / HBM_PEAK, 4)
        a["ms"] = round(a["ms"], 4)
    return agg


def link_reference(torch, sizes=(2 << 20, 8 << 20, 1 << 30), total=4 << 30):
    """Plain pinned-host <-> device copies through torch on one stream, timed
    with events: the host link's practical rate per direction, for copies of
    one tensor's size (2 MiB: a meson tensor) and for large ones."""
    out = {}
    for nbytes in sizes:
        reps = max(4, total // nbytes)
        host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        dev = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        for name, dst, src in (("h2d", dev, host), ("d2h", host, dev)):
            dst.copy_(src, non_blocking=True)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                dst.copy_(src, non_blocking=True)
            b.record()
            b.synchronize()
            out[f"{name}_{nbytes >> 20}MiB_GBps"] = round(nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9, 2)
        del host, dev
    return out


def transfer_rates(records, tts_s):
    """Per direction: transfers, bytes and summed copy time of one timed
    execute, the achieved rate while copying, and the copy stream's busy
    share of the time-to-solution."""
    out = {}
    for kind in ("h2d", "d2h"):
        rs = [r for r in records if r["type"] == kind]
        ms = sum(r["ms"] for r in rs)
        nbytes = sum(r["bytes"] for r in rs)
        out[kind] = {"n": len(rs), "GB": round(nbytes / 1e9, 4), "copy_ms": round(ms, 3),
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 2) if ms > 0 else None}
    busy = sum(out[k]["copy_ms"] for k in out)
    out["copy_busy_frac_of_tts"] = round(busy * 1e-3 / tts_s, 3) if tts_s else None
    return out


def transfer_study(ctx, runner, budget, reps=1, link=True):
    """The host-transfer step on its own: per-copy events on the copy stream in
    timed (eager) executes of the budgeted FP64 Tree order with lookahead 16,
    beside the pinned-copy link reference.  An event pair around a copy that
    waits for the compute stream can include part of that wait."""
    ctx.set_mem_budget(budget)
    ctx.schedule("tree")
    ctx.set_options(leaves_resident=False, wave_lookahead=16, use_graphs=False)
    ctx.set_timing(True)
    runner.run("fp64", True)                     # plans and warms up
    runner.torch.cuda.synchronize()
    runs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        runner.run("fp64", True)
        runner.torch.cuda.synchronize()
        runs.append(transfer_rates(ctx.launch_records(), time.perf_counter() - t0))
    ctx.set_timing(False)
    out = {"fp64_tree_lookahead16": runs[-1]}
    if link:
        out["link_reference"] = link_reference(runner.torch)
    log("transfers", out)
    return out


def budgeted_schedules(ctx, runner, prec, budget, X):
    """Time-to-solution under the configuration's HBM budget with the leaves
    starting in pinned host memory (every transfer inside the time): input
    order, Sibling, Tree and node gain cut into waves with lookahead 16 and replayed from
    captured segments, Tree without lookahead, and Tree with one eager launch
    per contraction.  One warm-up and one timed execute each.  Every run's
    correlators are compared bit for bit with those of the resident run that
    precedes this call."""
    import numpy as np
    ref = np.concatenate(ctx.fetch_correlators()).view(np.uint64)
    out = {}
    ctx.set_mem_budget(budget)
    for policy, look, batched in (("input", 16, True), ("sibling", 16, True), ("tree", 16, True),
                                  ("node", 16, True), ("tree", 0, True), ("tree", 16, False)):
        ctx.schedule(policy)
        ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=batched)
        key = policy + (f"_lookahead{look}" if look and batched else "") + ("" if batched else "_per_contraction")
        try:
            dt, st = timed_steps(ctx, runner, prec, batched, 1, 1)
            p = st["plan"]
            same = bool(np.array_equal(np.concatenate(ctx.fetch_correlators()).view(np.uint64), ref))
            timing = {"tts_s": round(dt, 4), "tflops": round(p["flops"] / dt / 1e12, 3),
                      "bits_equal_resident": same}
        except X.CdagError as e:
            # e.g. pinned host memory for the spilled intermediates not available:
            # the plan's counts are still exact, the time is not measured
            p = ctx.plan(prec, batched)
            timing = {"tts_s": None, "error": str(e)[:160],
                      "host_spill_GB": round(p["host_spill_bytes"] / 1e9, 3)}
        out[key] = {**timing,
                    "h2d_GB": round(p["h2d_bytes"] / 1e9, 3), "d2h_GB": round(p["d2h_bytes"] / 1e9, 3),
                    "n_evict": p["n_evict"], "peak_resident_GB": round(p["peak_resident"] / 1e9, 3),
                    "peak_post_GB": round(p["peak_post"] / 1e9, 3), "n_steps": p["n_steps"],
                    "budget_GB": round(budget / 1e9, 3)}
        log(prec, key, out[key])
    ctx.set_mem_budget(None)
    ctx.schedule("tree")
    ctx.set_options(leaves_resident=True, wave_lookahead=X.binding.LOOKAHEAD_ALL, use_graphs=True)
    return out


def workload_rooflines(name, precs, steps, X, W, DeviceRunner, in_situ=True, fixed=None, budgeted=False):
    """One config at its full size, Tree schedule, waves of every ready
    contraction, leaves resident, graph replay: autotuned variants, time per
    execute, and per-kernel rates from a timed execute.  budgeted: also the
    schedules under the configuration's HBM budget (budgeted_schedules)."""
    import torch
    wl = W.config(name)
    budget = wl.budget_bytes
    log(f"{name}: workload built")
    shapes = set()
    for g in wl.graphs:
        n = next(wl.leaves[o].nvec for op in g.ops for o in op[1:] if o >= 0)
        shapes.update((kind, n) for kind, _, _ in g.ops if kind != 3)
    shapes = sorted(shapes)
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    del wl
    ctx.schedule("tree")
    ctx.set_mem_budget(None)
    ctx.set_options(leaves_resident=True, wave_lookahead=X.binding.LOOKAHEAD_ALL, use_graphs=True)
    runner = DeviceRunner(ctx, 0)
    res = {}
    inv = {v: k for k, v in KIND_NAMES.items()}
    for prec in precs:
        if fixed and prec in fixed:
            for key, choice in fixed[prec].items():
                kname, n = key.split("_N")
                ctx.set_tile(prec, inv[kname], int(n), *choice)
            runner.ensure_arena(ctx.plan(prec, True)["arena_bytes"])
        else:
            runner.autotune(prec, True, reps=2 if in_situ else 1, in_situ=in_situ)
        dt, st = timed_steps(ctx, runner, prec, True, steps, 1)
        p = st["plan"]
        ctx.set_timing(True)
        runner.run(prec, True)
        recs = ctx.launch_records()
        ctx.set_timing(False)
        res[prec] = {
            "tflops": round(p["flops"] * steps / dt / 1e12, 3),
            "ms_per_step": round(dt / steps * 1e3, 3), "n_waves": p["n_steps"],
            "n_contractions": p["n_contr"], "flops_per_step": p["flops"],
            "arena_GB": round(p["arena_bytes"] / 1e9, 2),
            "variants": {f"{KIND_NAMES[k]}_N{n}": list(ctx.get_tile(prec, k, n)) for k, n in shapes},
            "kernels": kernel_table(recs, prec)}
        if budgeted and budget:
            res[prec]["budgeted"] = budgeted_schedules(ctx, runner, prec, budget, X)
        log(name, prec, res[prec])
    ctx.close()
    runner.arena = None
    del runner
    torch.cuda.empty_cache()
    return res


def corr_func_study(rows=None):
    """Host-only: the peak-memory study (Sec. IV-B), the scheduler-time study
    (Table sch-time) and the data-movement counts (evictions, transfers and
    their size, Sec. IV-C) on the Table corr-func-shaped DAGs.  Per row: DAG
    size and F_v / F_e, then for the input order, Sibling, Tree and node gain
    the wall time of the schedule call, the peak memory (after-release M_i peak and
    live peak during an op) and the budgeted plan's counts, sizes in units of
    the greatest common divisor of the distinct tensor sizes as the paper
    plots them."""
    import math
    from synth import corr_func as CF
    import paper_2511_02257_amd as X
    out = {}
    for row in rows or list(CF.TABLE):
        wl = CF.corr_func_like(row)
        ctx = X.Context()
        t0 = time.perf_counter()
        ctx.build_cdag(wl.leaves, wl.graphs)
        t_build = time.perf_counter() - t0
        st = ctx.dag_stats()
        kind, _, _ = ctx.nodes()
        sizes = set()
        for lf in wl.leaves:
            sizes.add(lf.nt * lf.nvec ** lf.rank * 16)
        rank_of = {0: 2, 1: 3, 2: 2}
        n = wl.leaves[0].nvec
        for k in set(int(x) for x in kind[len(wl.leaves):]):
            if k in rank_of:
                sizes.add(wl.leaves[0].nt * n ** rank_of[k] * 16)
        unit = 0
        for z in sizes:
            unit = math.gcd(unit, z)
        res = {"system": CF.TABLE[row]["system"], "graphs": len(wl.graphs), "leaves": len(wl.leaves),
               "N": n, "build_ms": round(t_build * 1e3, 1), **{k: (round(v, 3) if isinstance(v, float) else v)
                                                           for k, v in st.items()}}
        for policy in ("input", "sibling", "tree", "node"):
            t0 = time.perf_counter()
            order = ctx.schedule(policy)
            dt = time.perf_counter() - t0
            _, pp, pl = ctx.memsim(order, 16)
            res[policy] = {"ms": round(dt * 1e3, 2), "peak_post_units": int(pp // unit),
                           "peak_live_units": int(pl // unit)}
        best = min(res["sibling"]["peak_post_units"], res["tree"]["peak_post_units"])
        res["input_over_best"] = round(res["input"]["peak_post_units"] / max(1, best), 3)
        # Budgeted plans (the data-movement study): a budget of half the lower
        # live peak of Sibling and Tree, so every schedule must evict;
        # per-contraction steps in schedule order.
        # (raised by quarters while one contraction alone does not fit)
        b_units = max(min(res["sibling"]["peak_live_units"], res["tree"]["peak_live_units"]) // 2, 1)
        while True:
            ctx.set_mem_budget(b_units * unit)
            try:
                plans = {}
                for policy in ("input", "sibling", "tree", "node"):
                    ctx.schedule(policy)
                    plans[policy] = ctx.plan("fp64", False)
                break
            except X.CdagError:
                b_units += max(1, b_units // 4)
        res["budget_units"] = b_units
        for policy, p in plans.items():
            res[policy]["plan"] = {"n_evict": p["n_evict"], "n_transfers": p["n_h2d"] + p["n_d2h"],
                                   "h2d_units": int(p["h2d_bytes"] // unit),
                                   "d2h_units": int(p["d2h_bytes"] // unit)}
        ctx.set_mem_budget(None)
        out[row] = res
        log(row, res)
        ctx.close()
    return out


def general_study(shares=(0.02, 0.05, 0.1), n_trees=40000):
    """Host-only: input order, Tree and node gain on general DAGs whose nodes have one to
    four children (synth/general.py: 400 leaves, trees of depth 3, an inner slot
    reusing an existing node with probability `share`).  Per DAG: size, F_v and
    F_e, the wall time of each schedule call and its peak memory (node sizes in
    bytes, 1..1000 per node, roots 0)."""
    from synth.general import random_general
    import paper_2511_02257_amd as X
    out = []
    for share in shares:
        nl, sizes, kids = random_general(7, n_leaves=400, n_trees=n_trees, max_arity=4, depth=3,
                                         share=share)
        ctx = X.Context()
        ctx.build_general(nl, sizes, kids)
        res = {"share": share, **{k: (round(v, 3) if isinstance(v, float) else v)
                                  for k, v in ctx.dag_stats().items()}}
        for policy in ("input", "tree", "node"):
            t0 = time.perf_counter()
            order = ctx.schedule(policy)
            dt = time.perf_counter() - t0
            _, pp, pl = ctx.memsim(order)
            res[policy] = {"ms": round(dt * 1e3, 1), "peak_post": int(pp), "peak_live": int(pl)}
        res["input_over_tree"] = round(res["input"]["peak_post"] / max(1, res["tree"]["peak_post"]), 3)
        log("general", res)
        out.append(res)
        ctx.close()
    return out


def cpu_baseline(wl, seconds=12.0):
    """The oracle (numpy complex128, each graph on its own) on a bounded sample."""
    from oracle import values as OV
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    data = [lf.data for lf in wl.leaves]
    flops = 0.0
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < len(wl.graphs):
        ops = wl.graphs[n].ops
        OV.evaluate_graph(data, ops)
        for kind, l, r in ops:
            N, T = wl.leaves[0].nvec, wl.leaves[0].nt
            flops += 8.0 * T * N ** 3 if kind == 0 else 8.0 * T * N * N
        n += 1
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": flops / dt / 1e12, "unit": "complex TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"first {n} of {len(wl.graphs)} graphs, each evaluated on its own with "
                      f"numpy complex128 matmul (no DAG sharing), {dt:.1f} s",
            "cpu": cpu, "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-extras", action="store_true", help="only the headline value")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--fp64-variant", default=None, metavar="TILE,GRID,STAGES",
                    help="fix the FP64 K22 kernel variant instead of autotuning it "
                         "(so that counter runs profile the variant a timed run chose)")
    ap.add_argument("--workload", default="meson_ring",
                    choices=("meson_ring", "baryon_mix", "batched"),
                    help="meson_ring: the headline line (default). baryon_mix, batched: that config "
                         "alone at full size, resident, with per-kernel rates (for profiling)")
    ap.add_argument("--variants-from", default=None, metavar="JSON",
                    help="with --workload baryon_mix or batched: take the kernel choices from the "
                         "JSON line of an earlier run of the same workload instead of autotuning")
    ap.add_argument("--budgeted", action="store_true",
                    help="with --workload: also time input order, Sibling and Tree under the "
                         "configuration's HBM budget with the leaves starting on the host")
    ap.add_argument("--study", default=None, choices=("corr_func", "general"),
                    help="host-only: peak memory and scheduler time on the Table corr-func-shaped "
                         "DAGs (no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (counter calibration)")
    ap.add_argument("--transfers", action="store_true",
                    help="only the budgeted meson transfers: --steps timed eager FP64 executes "
                         "(Tree, lookahead 16, leaves on the host) with per-copy events, no other "
                         "copies (for a memory-copy trace)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n, "copy_calibration_bytes_written": n,
                          "launches": 3}))
        return
    if args.study == "corr_func":
        print(json.dumps({"study": "corr_func", "rows": corr_func_study()}), flush=True)
        return
    if args.study == "general":
        print(json.dumps({"study": "general", "dags": general_study()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is not "
              f"sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    from synth import workloads as W
    import paper_2511_02257_amd as X
    from paper_2511_02257_amd.device import DeviceRunner

    if args.workload != "meson_ring":
        precs = ("fp64", "fp32", "bf16x3") if args.workload == "baryon_mix" else ("fp32", "bf16x3")
        fixed = None
        if args.variants_from:
            with open(args.variants_from) as f:
                prev = json.loads(f.read().strip().splitlines()[-1])
            fixed = {p: r["variants"] for p, r in prev["per_precision"].items()}
        res = workload_rooflines(args.workload, precs, args.steps, X, W, DeviceRunner,
                                 in_situ=args.workload == "baryon_mix", fixed=fixed, budgeted=args.budgeted)
        head = res[precs[0]]
        print(json.dumps({
            "metric": METRIC, "value": head["tflops"], "unit": "complex TFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": head["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if precs[0] == "fp64" else "c64 storage, f32 accumulate",
            "data": "synthetic",
            "config": {"workload": args.workload + " (full size, leaves resident, no budget)"},
            "per_precision": res}), flush=True)
        return

    wl = W.config("meson_ring")
    log("workload built")
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    # budget: a quarter of the input-order schedule's live peak
    ctx.schedule("input")
    live = {p: ctx.plan(p, False)["peak_live"] for p in ("fp64", "fp32")}
    budgets = {"fp64": live["fp64"] // 4, "fp32": live["fp32"] // 4, "bf16x3": live["fp32"] // 4}
    t0 = time.perf_counter()
    ctx.schedule("tree")
    t_sched = time.perf_counter() - t0
    ctx.set_mem_budget(None)
    ALL = X.binding.LOOKAHEAD_ALL
    ctx.set_options(leaves_resident=True, wave_lookahead=ALL, use_graphs=True)
    runner = DeviceRunner(ctx, 0)
    if args.transfers:
        print(json.dumps({"transfers": transfer_study(ctx, runner, budgets["fp64"], reps=args.steps,
                                                      link=False),
                          "budget_bytes": budgets["fp64"]}), flush=True)
        return
    tiles = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        if prec == "fp64" and args.fp64_variant:
            ctx.set_tile("fp64", 0, 64, *(int(x) for x in args.fp64_variant.split(",")))
            runner.ensure_arena(ctx.plan("fp64", True)["arena_bytes"])
        elif prec == "fp64" or not args.skip_extras:
            runner.autotune(prec, True, reps=3, in_situ=True)
        t, g, st, _ = ctx.get_tile(prec, 0, 64)
        tiles[prec] = {"K22_N64": {"tile": list(X.TILES[t]), "threads": X.binding.TILE_THREADS[t],
                                   "grid": X.binding.GRIDS[g], "lds_stages": st}}
    log("autotuned tiles", tiles)

    # ---- headline: FP64, Tree, waves, leaves resident, graph replay
    dt, st = timed_steps(ctx, runner, "fp64", True, args.steps, args.warmup)
    flops = st["plan"]["flops"]
    value = flops * args.steps / dt / 1e12
    log(f"fp64 waves: {dt / args.steps * 1e3:.3f} ms/step, {value:.2f} TFLOP/s")
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "complex TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "meson_ring: 16 mesons complex128 [32][64][64], 2000 ring traces "
                               "of 4-8 leaves, merged DAG",
                   "n_contractions": st["plan"]["n_contr"], "n_waves": st["plan"]["n_steps"],
                   "schedule": "tree",
                   "mode": "waves of every ready contraction, one hipGraph replay",
                   "leaves": "resident in HBM", "flops_per_step": flops,
                   "t_schedule_tree_s": round(t_sched, 4), "autotuned_tiles": tiles},
        # memory of the timed run: HBM held by the arena (leaves, tensor pool,
        # split-K workspace, descriptors, results), the plan's resident peak, and
        # host-to-device bytes per step (0: the leaves stay resident after the
        # first upload).  The budgeted runs under extras carry the same figures.
        "memory": {"arena_GB": round(st["plan"]["arena_bytes"] / 1e9, 4),
                   "tensor_highwater_GB": round(st["plan"]["tensor_highwater"] / 1e9, 4),
                   "peak_live_GB": round(st["plan"]["peak_live"] / 1e9, 4),
                   "h2d_GB_per_step": round(st["plan"]["h2d_bytes"] / 1e9, 4)},
    }

    # ---- roofline of the exterior-contraction kernel (HIP events per launch)
    ctx.set_timing(True)
    hec_t, hec_f, hec_b, hec_n = 0.0, 0.0, 0.0, 0
    for _ in range(max(1, args.steps // 5)):
        s2 = runner.run("fp64", True)
        hec_t += s2["t_hec_s"]
        hec_f += s2["hec_flops"]
        hec_b += s2["hec_bytes"]
        hec_n += s2["n_hec_launches"]
    kernels = kernel_table(ctx.launch_records(), "fp64")
    ctx.set_timing(False)
    achieved = hec_f / hec_t / 1e12
    t64, g64, st64, _ = ctx.get_tile("fp64", 0, 64)
    variant = X.binding.variant_index(t64, g64, st64)
    out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["fp64"],
                       "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp64"], 4),
                       "traffic": measured_traffic(variant), "tile": list(X.TILES[t64]),
                       "threads": X.binding.TILE_THREADS[t64],
                       "grid": X.binding.GRIDS[g64], "lds_stages": st64,
                       "variant": [t64, g64, st64],
                       "kernel": "hec_mfma<double> (grouped K22 waves)",
                       "avg_launch_us": round(hec_t / hec_n * 1e6, 3),
                       "flops_per_launch": hec_f / hec_n,
                       "alg_bytes_per_launch": hec_b / hec_n,
                       "achieved_GBps": round(hec_b / hec_t / 1e9, 1),
                       "all_kernels_last_execute": kernels}
    log("roofline", out["roofline"])

    if not args.skip_extras:
        extras = {}
        # mixed precision, same resident mode
        for prec in ("fp32", "bf16x3"):
            d2, s3 = timed_steps(ctx, runner, prec, True, max(5, args.steps // 2), 2)
            extras[f"{prec}_value"] = round(s3["plan"]["flops"] * max(5, args.steps // 2) / d2 / 1e12, 4)
            extras[f"{prec}_ms_per_step"] = round(d2 / max(5, args.steps // 2) * 1e3, 4)
        # waves that keep the schedule order exactly (no lookahead)
        ctx.set_options(leaves_resident=True, wave_lookahead=0, use_graphs=True)
        d2, s3 = timed_steps(ctx, runner, "fp64", True, max(3, args.steps // 5), 1)
        extras["fp64_ordered_waves_value"] = round(s3["plan"]["flops"] * max(3, args.steps // 5) / d2 / 1e12, 4)
        extras["fp64_ordered_waves_n_waves"] = s3["plan"]["n_steps"]
        # per-contraction launches instead of waves
        ctx.set_options(leaves_resident=True, use_graphs=False)
        d2, s3 = timed_steps(ctx, runner, "fp64", False, max(3, args.steps // 10), 1)
        extras["fp64_per_contraction_value"] = round(s3["plan"]["flops"] * max(3, args.steps // 10) / d2 / 1e12, 4)
        # budgeted, leaves start on the host (PCIe-inclusive time-to-solution)
        # Each schedule runs with eager launches on two streams (copies overlap
        # kernels) and with captured segments on one stream (fewer launches);
        # the faster is reported, with the other's time beside it.  The Tree
        # schedule is also cut into waves with growing lookahead.
        budgeted = {}
        for prec in ("fp64", "fp32"):
            ctx.set_mem_budget(budgets[prec])
            for policy, look in (("input", 0), ("sibling", 0), ("tree", 0), ("tree", 4), ("tree", 16),
                                 ("tree", ALL), ("node", 0), ("node", 16)):
                ctx.schedule(policy)
                reps = 3
                tts = {}
                for graphs in (False, True):
                    ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=graphs)
                    d2, s3 = timed_steps(ctx, runner, prec, True, reps, 1)
                    tts["graphs" if graphs else "eager"] = d2 / reps
                d2 = min(tts.values()) * reps
                p = s3["plan"]
                key = f"{prec}_{policy}" + ("" if not look else ("_lookahead_all" if look == ALL
                                                                   else f"_lookahead{look}"))
                budgeted[key] = {
                    "tts_eager_s": round(tts["eager"], 5), "tts_graphs_s": round(tts["graphs"], 5),
                    "tts_s": round(d2 / reps, 5), "h2d_GB": round(p["h2d_bytes"] / 1e9, 4),
                    "d2h_GB": round(p["d2h_bytes"] / 1e9, 4), "n_evict": p["n_evict"],
                    "n_h2d": p["n_h2d"], "peak_resident_bytes": p["peak_resident"],
                    "peak_post_bytes": p["peak_post"], "budget_bytes": p["budget"],
                    "n_waves": p["n_steps"],
                    "tflops": round(p["flops"] / (d2 / reps) / 1e12, 3)}
                log(key, budgeted[key])
        extras["budgeted"] = budgeted
        extras["transfers"] = transfer_study(ctx, runner, budgets["fp64"])
        ctx.set_mem_budget(None)
        # the baryon configuration (FP64) and its precision form, per-kernel rates
        extras["baryon_mix"] = workload_rooflines("baryon_mix", ("fp64", "fp32", "bf16x3"),
                                                  max(3, args.steps // 10), X, W, DeviceRunner)
        out["extras"] = extras

    out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
