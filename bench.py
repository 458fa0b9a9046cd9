"""Benchmark: contraction-DAG execution on one MI355X.

Headline workload (the baryon configuration as stated): 12 baryon leaves
complex128 [Nt=32][64][64][64] and 12 meson leaves [32][64][64], entries
N(0,1)/64; 500 seeded chains X = K32(B_a, M_b), Y = K33(X, B_c),
C(t) = tr(Y M_d) merged into one DAG (139 K32, 440 K33, 500 traces); FP64;
HBM budget 32e9 bytes; Tree schedule; the leaves start in pinned host memory.

One step = one execute() of the whole DAG with every leaf upload inside it:
uploads, exterior contractions, root traces, the FP64 cross-diagram sums and
the copy of every correlator to the host.  The execute runs in passes over
slices of the time axis (uploads of one pass overlap the contractions of the
previous one) and picks its issue mode (eager on three streams, or one graph
over them) by a short trial.  `value` is the algorithmic complex TFLOP/s of the
time-to-solution (8 flops per complex multiply-add; DAG-shared work counted
once).

The same JSON line also carries: the same DAG with every leaf resident (the
kernel-only reference) and in one pass (whole tensors, the paper's memory
model); its precision form (complex FP32, split-BF16 with two and with three
pieces) with each correlator's error against the FP64 oracle on the sample the
CPU baseline evaluates; the memory-bound meson configuration under a quarter of
the input-order live peak (input order vs Tree, issue modes, host-transfer
rates beside a pinned-copy link reference); the batched configuration under
64e9 bytes (waves vs one launch per contraction); the roofline of the dominant
kernel (FP64 K33); and the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --only headline|precision|meson|batched   (one part)
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
# Peaks per algorithmic flop (8 per complex multiply-add): FP64 and FP32
# matrix cores; split-BF16 runs 3 (two pieces) or 6 (three pieces) bf16
# products per real product on the 2.5 PFLOP/s dense BF16 matrix cores.
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0, "bf16x6": 2500.0 / 6.0}
HBM_PEAK = 8000.0   # GB/s
KIND_NAMES = {0: "K22", 1: "K32", 2: "K33", 3: "HCA", 4: "C1", 5: "C2", 6: "C3", 7: "pairs"}
GAUSS_TILES = {1, 4, 5}   # FP64/FP32 tiles forming a complex product from three real ones
ALL = (1 << 63) - 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(runner, prec, batched, steps, warmup):
    for _ in range(warmup):
        runner.run(prec, batched)
    torch = runner.torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for _ in range(steps):
        st = runner.run(prec, batched)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def kernel_table(records, prec):
    """Launch records of one timed execute, summed per (launch type, kinds):
    time, algorithmic flops and bytes, and the rates against the MI355X peaks.
    frac_mfma counts algorithmic flops; frac_pipe the flops the matrix cores
    execute (three real products per complex one in the Gauss tiles: 3/4 of
    the algorithmic count).  A split-K contraction kind also gets an entry
    that charges its reduction kernels to it ("hec+reduce").  A contraction
    launch that carries its step's root traces ("hec:...+HCA") counts their
    flops and bytes in its totals; frac_mfma and frac_pipe count only the
    contractions' flops."""
    agg = {}
    for r in records:
        if r["type"] in ("h2d", "d2h"):
            continue
        key = r["type"] if r["type"] == "xsum" else r["type"] + ":" + "+".join(KIND_NAMES[k] for k in r["kinds"])
        a = agg.setdefault(key, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0, "mfma_flops": 0.0,
                                 "pipe_flops": 0.0})
        a["launches"] += 1
        a["ms"] += r["ms"]
        a["flops"] += r["flops"] + r.get("trace_flops", 0.0)
        a["bytes"] += r["bytes"] + r.get("trace_bytes", 0.0)
        a["mfma_flops"] += r["flops"]
        gauss = r["type"] == "hec" and prec in ("fp64", "fp32") and (r["variant"] % 6 in GAUSS_TILES or r["variant"] == 24)
        a["pipe_flops"] += r["flops"] * (0.75 if gauss else 1.0)
    for key in [k for k in agg if k.startswith("reduce:")]:
        hk = "hec:" + key.split(":", 1)[1]
        if hk in agg:
            agg["hec+reduce:" + key.split(":", 1)[1]] = {
                "launches": agg[hk]["launches"] + agg[key]["launches"],
                "ms": agg[hk]["ms"] + agg[key]["ms"], "flops": agg[hk]["flops"],
                "bytes": agg[hk]["bytes"], "mfma_flops": agg[hk]["mfma_flops"],
                "pipe_flops": agg[hk]["pipe_flops"]}
    for key, a in agg.items():
        sec = a["ms"] * 1e-3
        if sec <= 0:
            continue
        a["TFLOP/s"] = round(a["flops"] / sec / 1e12, 3)
        a["GB/s"] = round(a["bytes"] / sec / 1e9, 1)
        if key.startswith("hec"):
            a["frac_mfma"] = round(a["mfma_flops"] / sec / 1e12 / PEAK[prec], 4)
            a["frac_pipe"] = round(a["pipe_flops"] / sec / 1e12 / PEAK[prec], 4)
        if not key.startswith("reduce"):
            a["frac_hbm"] = round(a["bytes"] / sec / 1e9 / HBM_PEAK, 4)
        a["ms"] = round(a["ms"], 4)
        del a["pipe_flops"], a["mfma_flops"]
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
    execute, the achieved rate while copying, and each stream's busy share of
    the time-to-solution."""
    out = {}
    for kind in ("h2d", "d2h"):
        rs = [r for r in records if r["type"] == kind]
        ms = sum(r["ms"] for r in rs)
        nbytes = sum(r["bytes"] for r in rs)
        out[kind] = {"n": len(rs), "GB": round(nbytes / 1e9, 4), "copy_ms": round(ms, 3),
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 2) if ms > 0 else None,
                     "busy_frac_of_tts": round(ms * 1e-3 / tts_s, 3) if tts_s else None}
    return out


def plan_summary(p):
    return {"h2d_GB": round(p["h2d_bytes"] / 1e9, 4), "d2h_GB": round(p["d2h_bytes"] / 1e9, 4),
            "n_evict": p["n_evict"], "n_h2d": p["n_h2d"], "n_d2h": p["n_d2h"],
            "peak_resident_GB": round(p["peak_resident"] / 1e9, 4),
            "arena_GB": round(p["arena_bytes"] / 1e9, 4), "budget_GB": round(p["budget"] / 1e9, 4)
            if p["budget"] < (1 << 62) else None, "n_steps": p["n_steps"]}


def best_mode(runner, ctx, prec, batched, modes=(0, 2), reps=2, **opts):
    """Issue mode by trial: one warm-up and `reps` timed executes per mode;
    returns (mode, {mode: seconds per execute})."""
    times = {}
    for m in modes:
        ctx.set_options(use_graphs=m, **opts)
        dt, _ = timed_steps(runner, prec, batched, reps, 1)
        times[m] = dt / reps
    m = min(times, key=times.get)
    ctx.set_options(use_graphs=m, **opts)
    return m, times


def sample_bits(ctx, sample):
    corr = ctx.fetch_correlators()
    return {g: corr[g].copy() for g in sample}


# ---------------------------------------------------------------- headline
def given_tiles(args):
    """Kernel choices from --tiles-from or --tiles: {prec: {"K32_N64": [tile, grid, stages,
    split_k], ...}}, or {} when neither is given."""
    tiles = {}
    if args.tiles_from:
        with open(args.tiles_from) as f:
            prev = json.loads(f.read().strip().splitlines()[-1])
        tiles = prev["config"]["kernel_choices"]
    elif args.tiles:
        for part in args.tiles.split(";"):
            prec, rest = part.split(":")
            tiles[prec] = {k: [int(x) for x in v.split(".")] for k, v in
                           (item.split("=") for item in rest.split(","))}
    return tiles


def set_tiles(ctx, tiles, precs=None):
    for prec, table in tiles.items():
        if precs is not None and prec not in precs:
            continue
        for key, choice in table.items():
            kname, n = key.split("_N")
            ctx.set_tile(prec, {v: k for k, v in KIND_NAMES.items()}[kname], int(n), *choice)


def k64_kernels(args, X, W, DeviceRunner):
    """Kernel-only references of the K = 64 exterior contractions, for profiling: the
    meson DAG (K22) in FP64 and FP32 and the baryon DAG (K32, K33) in FP32, every leaf
    resident, Tree order, every ready contraction in a wave, eager issue.  Kernel choices
    from --tiles (else the in-situ autotuner); root traces in launches of their own, so
    that the contraction launches time the contractions alone.  Per part: the time per
    execute and the kernel table of one timed execute."""
    tiles = given_tiles(args)
    out = {}
    for name, prec in (("meson_ring", "fp64"), ("meson_ring", "fp32"), ("baryon_mix", "fp32")):
        wl = W.config(name)
        ctx = X.Context()
        ctx.build_cdag(wl.leaves, wl.graphs)
        del wl
        ctx.schedule("tree")
        ctx.set_trace_fusion(False)
        ctx.set_options(leaves_resident=True, wave_lookahead=ALL, use_graphs=0)
        runner = DeviceRunner(ctx, 0)
        if prec in tiles:
            set_tiles(ctx, tiles, (prec,))
            runner.ensure_arena(ctx.plan(prec, True)["arena_bytes"])
        else:
            runner.autotune(prec, True, reps=2, in_situ=True)
        choices = {f"{KIND_NAMES[k]}_N64": list(ctx.get_tile(prec, k, 64)) for k in (0, 1, 2)}
        dt, st = timed_steps(runner, prec, True, args.steps, args.warmup)
        ctx.set_timing(True)
        runner.run(prec, True)
        kt = kernel_table(ctx.launch_records(), prec)
        ctx.set_timing(False)
        ctx.close()
        log(f"k64 {name} {prec}: {dt / args.steps * 1e3:.3f} ms", {k: v.get("frac_mfma") for k, v in kt.items()})
        out[f"{name}_{prec}"] = {"ms_per_step": round(dt / args.steps * 1e3, 4), "kernel_choices": choices,
                                 "kernels": kt}
    return out


def headline(args, X, W, DeviceRunner, sample):
    """The baryon configuration as stated, FP64, plus its references: every
    leaf resident (kernel time), one pass (whole tensors), the precision
    forms.  Returns (line fields, extras, correlators of the sample per
    precision)."""
    torch = __import__("torch")
    wl = W.config("baryon_mix")
    budget = wl.budget_bytes
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    del wl
    t0 = time.perf_counter()
    ctx.schedule("tree")
    t_sched = time.perf_counter() - t0
    runner = DeviceRunner(ctx, 0)
    ctx.set_mem_budget(budget)
    ctx.set_time_chunks(args.chunks)
    opts = dict(leaves_resident=False, wave_lookahead=ALL)
    ctx.set_options(use_graphs=0, **opts)
    tiles = given_tiles(args)
    if tiles:
        set_tiles(ctx, tiles)
        runner.ensure_arena(ctx.plan("fp64", True)["arena_bytes"])
    else:
        runner.autotune("fp64", True, reps=2, in_situ=True)
        tiles["fp64"] = {f"{KIND_NAMES[k]}_N64": list(ctx.get_tile("fp64", k, 64)) for k in (1, 2)}
    log("fp64 kernel choices", tiles["fp64"])
    mode, mode_times = best_mode(runner, ctx, "fp64", True, **opts)
    dt, st = timed_steps(runner, "fp64", True, args.steps, args.warmup)
    p = st["plan"]
    corr = {"fp64": sample_bits(ctx, sample)}
    tts = dt / args.steps
    value = p["flops"] / tts / 1e12
    log(f"headline: {tts * 1e3:.2f} ms/step, {value:.2f} TFLOP/s, mode {mode} {mode_times}")
    fields = {
        "value": round(value, 4), "ms_per_step": round(tts * 1e3, 4),
        "config": {
            "workload": "baryon_mix as stated: 12 baryons complex128 [32][64][64][64] + 12 mesons "
                        "[32][64][64], N(0,1)/64, 500 chains K32 -> K33 -> trace merged "
                        f"({p['n_contr']} nodes), HBM budget 32e9 B, leaves start in pinned host "
                        "memory (every upload timed), Tree schedule",
            "schedule": "tree", "t_schedule_s": round(t_sched, 4), "precision": "fp64",
            "time_slice_passes": args.chunks, "wave_lookahead": "all ready",
            "issue_mode": X.binding.GRAPH_MODES[mode],
            "issue_mode_trial_ms": {X.binding.GRAPH_MODES[m]: round(t * 1e3, 3) for m, t in mode_times.items()},
            "flops_per_step": p["flops"], **plan_summary(p), "kernel_choices": tiles},
    }
    # roofline of the dominant kernel: FP64 K33 launches, HIP events per launch
    ctx.set_options(use_graphs=0, **opts)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    runner.run("fp64", True)
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t0
    recs = ctx.launch_records()
    ctx.set_timing(False)
    k33 = [r for r in recs if r["type"] == "hec" and r["kinds"] == [2]]
    ms = sum(r["ms"] for r in k33) / len(k33)
    fl = sum(r["flops"] for r in k33) / len(k33)
    by = sum(r["bytes"] for r in k33) / len(k33)
    variant = k33[0]["variant"]
    gauss = variant % 6 in GAUSS_TILES
    achieved = fl / (ms * 1e-3) / 1e12
    fields["roofline"] = {
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["fp64"], "unit": "TFLOP/s",
        "frac": round(achieved / PEAK["fp64"], 4),
        "traffic": measured_traffic("baryon_mix", variant),
        "kernel": "hec_mfma<double> (grouped K33 launches of the headline execute)",
        "variant": variant, "launches_per_step": len(k33), "avg_launch_us": round(ms * 1e3, 3),
        "flops_per_launch": fl, "alg_bytes_per_launch": by,
        "achieved_GBps": round(by / (ms * 1e-3) / 1e9, 1),
        "executed_flops_per_launch": fl * (0.75 if gauss else 1.0),
        "frac_pipe": round(achieved * (0.75 if gauss else 1.0) / PEAK["fp64"], 4),
        "all_kernels_timed_execute": kernel_table(recs, "fp64"),
        "transfers_timed_execute": transfer_rates(recs, t_timed)}
    extras = {}
    if args.only == "headline-fp64":
        ctx.close()
        return fields, extras, corr
    # references on the same DAG: one pass (whole tensors), and every leaf resident
    for name, chunks, resident in (("one_pass", 1, False), ("resident", 1, True)):
        ctx.set_time_chunks(chunks)
        o = dict(leaves_resident=resident, wave_lookahead=ALL)
        m, mt = best_mode(runner, ctx, "fp64", True, modes=(0, 2) if not resident else (1,), **o)
        d2, s2 = timed_steps(runner, "fp64", True, max(3, args.steps // 4), 1)
        extras[f"fp64_{name}"] = {"ms_per_step": round(d2 / max(3, args.steps // 4) * 1e3, 3),
                                  "issue_mode": X.binding.GRAPH_MODES[m], **plan_summary(s2["plan"])}
        log(name, extras[f"fp64_{name}"])
    res_ms = extras["fp64_resident"]["ms_per_step"]
    h2d_floor_ms = p["h2d_bytes"] / 1e9 / args.link_GBps * 1e3
    extras["fp64_overlap"] = {
        "tts_over_max_kernel_or_link": round(tts * 1e3 / max(res_ms, h2d_floor_ms), 3),
        "resident_ms": res_ms, "h2d_floor_ms": round(h2d_floor_ms, 3), "link_GBps_assumed": args.link_GBps}
    # the precision form: same DAG, budget and passes, complex64 storage
    ctx.set_time_chunks(args.chunks)
    for prec in ("fp32", "bf16x3", "bf16x6"):
        if prec not in tiles:
            ctx.set_options(use_graphs=0, **opts)
            runner.autotune(prec, True, reps=1, in_situ=True)
            tiles[prec] = {f"{KIND_NAMES[k]}_N64": list(ctx.get_tile(prec, k, 64)) for k in (1, 2)}
        m, mt = best_mode(runner, ctx, prec, True, **opts)
        n = max(3, args.steps // 2)
        d2, s2 = timed_steps(runner, prec, True, n, 1)
        corr[prec] = sample_bits(ctx, sample)
        extras[prec] = {"ms_per_step": round(d2 / n * 1e3, 3),
                        "tflops": round(s2["plan"]["flops"] / (d2 / n) / 1e12, 3),
                        "speedup_vs_fp64": round(tts / (d2 / n), 3),
                        "issue_mode": X.binding.GRAPH_MODES[m], "kernel_choices": tiles[prec],
                        **plan_summary(s2["plan"])}
        log(prec, extras[prec])
    # the schedules on the same configuration (FP64, budget, passes, kernel
    # choices, eager issue) with waves of lookahead 16, where the order decides
    # the resident peak (with every ready contraction in a wave all orders give
    # the same three waves)
    sched = {}
    ctx.set_options(use_graphs=0, leaves_resident=False, wave_lookahead=16)
    for policy in ("input", "sibling", "node", "tree"):
        ctx.schedule(policy)
        n = max(3, args.steps // 4)
        d2, s2 = timed_steps(runner, "fp64", True, n, 1)
        sched[policy] = {"ms_per_step": round(d2 / n * 1e3, 3),
                         "tflops": round(s2["plan"]["flops"] / (d2 / n) / 1e12, 3), **plan_summary(s2["plan"])}
        log("schedule", policy, sched[policy])
    extras["fp64_schedules"] = sched
    ctx.close()
    runner.arena = None
    del runner
    torch.cuda.empty_cache()
    return fields, extras, corr


def measured_traffic(workload, variant):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source or variant differs from the one the
    counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"hec_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_2511_02257_amd.profiling import kernel_source_sha256
    if rec.get("kernel_sha256") != kernel_source_sha256():
        return None
    entry = rec.get("variants", {}).get(str(variant))
    return None if entry is None else entry.get("traffic_bytes_per_launch")


# ---------------------------------------------------------------- meson
def meson_budgeted(args, X, W, DeviceRunner):
    """The memory-bound meson configuration: 16 mesons complex128 [32][64][64],
    2000 ring traces; budget a quarter of the input-order live peak; leaves in
    pinned host memory.  Input order, Tree and node order on whole tensors
    (waves with lookahead 16, and Tree without lookahead), then passes over the
    time slices, each in every issue mode; host-transfer rates of the eager
    Tree run beside a pinned-copy link reference."""
    torch = __import__("torch")
    wl = W.config("meson_ring")
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    del wl
    ctx.schedule("input")
    budget = ctx.plan("fp64", False)["peak_live"] // 4
    runner = DeviceRunner(ctx, 0)
    ctx.schedule("tree")
    ctx.set_options(leaves_resident=True, wave_lookahead=ALL, use_graphs=1)
    runner.autotune("fp64", True, reps=1, in_situ=False)
    ref = None
    out = {"budget_bytes": budget}
    d2, s2 = timed_steps(runner, "fp64", True, 10, 2)
    out["resident_tree_ms"] = round(d2 / 10 * 1e3, 3)
    ref = np.concatenate(ctx.fetch_correlators()).view(np.uint64).copy()
    ctx.set_mem_budget(budget)
    # whole tensors (the memory model of Sec. II-C), then passes over the time
    # slices under the same budget: a pass holds slices of every tensor in half
    # the budget, so the budget binds less, the plan moves less, and larger
    # waves fit (16 passes with lookahead 384 is the fastest of a sweep over
    # 1-32 passes and lookahead 16-768; every leaf is uploaded once)
    for policy, look, chunks in (("input", 16, 1), ("tree", 16, 1), ("tree", 0, 1), ("node", 16, 1),
                                 ("tree", 16, 4), ("tree", 384, 16), ("input", 384, 16)):
        ctx.schedule(policy)
        ctx.set_time_chunks(chunks)
        row = {}
        for mode in (0, 1, 2):
            ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=mode)
            d2, s2 = timed_steps(runner, "fp64", True, 3, 1)
            row[X.binding.GRAPH_MODES[mode] + "_ms"] = round(d2 / 3 * 1e3, 3)
        row["bits_equal_resident"] = bool(np.array_equal(np.concatenate(ctx.fetch_correlators()).view(np.uint64), ref))
        row.update(plan_summary(s2["plan"]))
        row["tflops_best"] = round(s2["plan"]["flops"] / (min(v for k, v in row.items() if k.endswith("_ms")) * 1e-3) / 1e12, 3)
        if (policy, look, chunks) == ("tree", 384, 16):
            # the same with every step's root traces in a launch of their own
            ctx.set_trace_fusion(False)
            ctx.set_options(leaves_resident=False, wave_lookahead=look, use_graphs=1)
            d2, _ = timed_steps(runner, "fp64", True, 3, 1)
            row["one-stream segments_traces_unfused_ms"] = round(d2 / 3 * 1e3, 3)
            ctx.set_trace_fusion(True)
        key = f"{policy}_lookahead{look}" + (f"_{chunks}passes" if chunks > 1 else "")
        out[key] = row
        log("meson", key, row)
    ctx.set_time_chunks(1)
    ctx.schedule("tree")
    ctx.set_options(leaves_resident=False, wave_lookahead=16, use_graphs=0)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    runner.run("fp64", True)
    torch.cuda.synchronize()
    out["transfers_tree_lookahead16_eager"] = transfer_rates(ctx.launch_records(), time.perf_counter() - t0)
    ctx.set_timing(False)
    out["link_reference"] = link_reference(torch)
    link = out["link_reference"].get("h2d_2MiB_GBps")
    best = min(v for k, v in out["tree_lookahead16"].items() if k.endswith("_ms"))
    if link:
        floor = out["tree_lookahead16"]["h2d_GB"] / link * 1e3
        out["tree_lookahead16_over_link_floor"] = round(best / floor, 3)
    ctx.close()
    runner.arena = None
    del runner
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- batched
def batched_budgeted(args, X, W, DeviceRunner):
    """The batched configuration: five N families (32..128), Nt = 64, complex64
    storage, just over 20,000 contractions; HBM budget 64e9 bytes; leaves in
    pinned host memory; Tree order; synthetic autotuner.  Waves with the kernel
    choice tuned per (kind, N) (one grouped launch per choice and wave) and
    with one choice for all shapes (one grouped launch per wave), every ready
    contraction in a wave over 8 passes of the time slices, against one launch
    per contraction; FP32 and split-BF16 with two pieces."""
    torch = __import__("torch")
    wl = W.config("batched")
    ctx = X.Context()
    ctx.build_cdag(wl.leaves, wl.graphs)
    budget = wl.budget_bytes
    del wl
    ctx.schedule("tree")
    ctx.set_mem_budget(budget)
    runner = DeviceRunner(ctx, 0)
    out = {}
    for prec in ("fp32", "bf16x3"):
        for uniform in (False, True):
            ctx.set_options(leaves_resident=False, wave_lookahead=16, use_graphs=0)
            runner.autotune(prec, True, reps=1, in_situ=False, uniform=uniform)
            ref = None
            # waves of lookahead 16 on whole tensors; every ready contraction in a
            # wave over 8 passes of the time slices (the fastest of a sweep over
            # 1-64 passes and lookahead 16 to all; no eviction under the budget);
            # one launch per contraction
            rows = (("waves_lookahead16", True, 16, 1),)
            if not uniform:
                rows += (("waves_all_8passes", True, ALL, 8),)
                if prec == "fp32":
                    rows += (("per_contraction", False, 0, 1),)
            for name, batched, look, chunks in rows:
                ctx.set_time_chunks(chunks)
                m, mt = best_mode(runner, ctx, prec, batched, modes=(0, 2) if batched else (0,), reps=1,
                                  leaves_resident=False, wave_lookahead=look)
                d2, s2 = timed_steps(runner, prec, batched, 1, 0)
                bits = np.concatenate(ctx.fetch_correlators()).view(np.uint64)
                if ref is None:
                    ref = bits.copy()
                row = {"tts_s": round(d2, 4), "tflops": round(s2["plan"]["flops"] / d2 / 1e12, 3),
                       "issue_mode": X.binding.GRAPH_MODES[m], "n_hec_launches": s2["n_hec_launches"],
                       "n_launches": s2["n_launches"], "bits_equal_first": bool(np.array_equal(bits, ref)),
                       "n_contractions": s2["plan"]["n_contr"], **plan_summary(s2["plan"])}
                key = f"{prec}_{name}" + ("_one_choice" if uniform else "")
                if uniform:
                    t, g, st_, sk = ctx.get_tile(prec, 2, 128)
                    row["choice"] = {"tile": list(X.TILES[t]), "grid": X.binding.GRIDS[g], "lds_stages": st_,
                                     "split_k": sk}
                out[key] = row
                log("batched", key, row)
            ctx.set_time_chunks(1)
        for kind in (0, 1, 2):            # back to the per-shape default before the next precision
            for n in (32, 48, 64, 96, 128):
                ctx.set_tile(prec, kind, n, -1)
    ctx.close()
    runner.arena = None
    del runner
    torch.cuda.empty_cache()
    return out


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


def cpu_baseline(seconds):
    """The oracle (numpy complex128, each graph evaluated on its own) on the
    first graphs of the headline workload, for about `seconds`; returns the
    baseline record and the oracle's correlators of the sample."""
    from oracle import values as OV
    from synth import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    wl = W.config("baryon_mix")
    data = [lf.data for lf in wl.leaves]
    ref = {}
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < len(wl.graphs):
        ref[n] = OV.evaluate_graph(data, wl.graphs[n].ops)
        n += 1
    dt = time.perf_counter() - t0
    N, T = 64, 32
    per_graph_flops = 2 * 8.0 * T * N ** 4 + 8.0 * T * N * N       # K32 + K33 + trace, no sharing
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    tts_all = dt / n * len(wl.graphs)
    return {"value": round(per_graph_flops * n / dt / 1e12, 5), "unit": "complex TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"first {n} of {len(wl.graphs)} graphs of the headline workload, each evaluated on its "
                      f"own with numpy complex128 tensordot (no DAG sharing, no memory budget), {dt:.1f} s",
            "time_to_solution_extrapolated_s": round(tts_all, 2),
            "cpu": cpu, "host_cpus": os.cpu_count()}, ref


def errors_vs_oracle(corr, ref):
    """Per correlator of the sample: ||C - C_ref|| / ||C_ref|| over t."""
    errs = np.array([np.linalg.norm(corr[g] - ref[g]) / np.linalg.norm(ref[g]) for g in ref])
    return {"graphs": len(errs), "max": float(errs.max()), "median": float(np.median(errs))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunks", type=int, default=8, help="time-slice passes of the headline execute")
    ap.add_argument("--link-GBps", type=float, default=55.0,
                    help="host-link rate for the upload floor of the headline (large pinned copies)")
    ap.add_argument("--only", default=None, choices=("headline", "headline-fp64", "meson", "batched", "k64"),
                    help="one part: the headline (with its references and precision form), the headline "
                         "FP64 execute alone (for profiling), the budgeted meson configuration, the "
                         "batched configuration, or the K = 64 contraction kernels on resident DAGs "
                         "(for profiling)")
    ap.add_argument("--tiles-from", default=None, metavar="JSON",
                    help="take the headline's kernel choices from the JSON line of an earlier run "
                         "instead of autotuning (so that profiled runs use the same kernels)")
    ap.add_argument("--tiles", default=None, metavar="PREC:KIND_N=T.G.S.K,...",
                    help="the headline's kernel choices written out, e.g. "
                         "fp64:K32_N64=5.1.1.1,K33_N64=5.1.1.0 (tile, grid, LDS stages, split_k)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--study", default=None, choices=("corr_func", "general"),
                    help="host-only: peak memory and scheduler time on the Table corr-func-shaped "
                         "DAGs, or on general DAGs (no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (counter calibration)")
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

    out = {"metric": METRIC, "unit": "complex TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic"}
    if args.only == "meson":
        print(json.dumps({"meson_ring_budgeted": meson_budgeted(args, X, W, DeviceRunner)}), flush=True)
        return
    if args.only == "batched":
        print(json.dumps({"batched_budgeted": batched_budgeted(args, X, W, DeviceRunner)}), flush=True)
        return
    if args.only == "k64":
        print(json.dumps({"k64_kernels": k64_kernels(args, X, W, DeviceRunner)}), flush=True)
        return
    # the oracle's sample first (its correlators also give the precision errors)
    base, ref = cpu_baseline(args.cpu_seconds if args.only is None else min(args.cpu_seconds, 2.0))
    fields, extras, corr = headline(args, X, W, DeviceRunner, sorted(ref))
    out.update(fields)
    errs = {p: errors_vs_oracle(c, ref) for p, c in corr.items()}
    out["config"]["correlator_error_vs_fp64_oracle"] = errs["fp64"]
    for p in ("fp32", "bf16x3", "bf16x6"):
        if p in extras:
            extras[p]["correlator_error_vs_fp64_oracle"] = errs[p]
    out["extras"] = {"baryon_mix": extras}
    if args.only is None:
        out["extras"]["meson_ring_budgeted"] = meson_budgeted(args, X, W, DeviceRunner)
        out["extras"]["batched_budgeted"] = batched_budgeted(args, X, W, DeviceRunner)
    out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
