"""Benchmark of the CBAA hot path on one MI355X.

One step = one window of the core-edge workload through every stage:
  local servers: take every router's packets into its source-keyed and
  destination-keyed cubes, which start the window empty (one read of each
  pair; all routers in one batched launch sequence flagged fresh, so the
  update stores whole row blocks instead of zeroing the cubes first);
  global server: OR-merge the routers' cubes, restore the super hosts of
  both global cubes, copy both sorted lists and counters to pinned host
  memory.
The step is captured once in a HIP graph and replayed (``--eager`` launches it
directly instead).

Workload: 64 x 2^20 synthetic packets (8M Zipf(1.1) sources, 1000 planted
hosts of 1k-200k peers, half fan-out and half fan-in, 10% duplicates), split
at random over the edge routers; paper dimensions r=4, |RA|=3, |VA|=1,
g=c=2^12 (128 MiB per cube); theta = 1024. Inputs are resident in HBM before
timing starts.

Besides the headline throughput the JSON line carries per-phase times, the
roofline of the update, a serving run (Poisson chunk arrivals from 16
routers, continuous batching; p50/p99 chunk-to-result latency), the learned
estimator against linear counting, and the CPU oracle's throughput.

Only one GPU is used: --gpus above 1 exits.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes of one update call on the default workload (2 routers, default
# tuning), from FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy's counters;
# valid only while the update kernels' sources are the ones measured
# (profiles/update_core_edge_64M_traffic.txt).
UPDATE_TRAFFIC = {"bytes": 3485792106, "sources": {
    "paper_1901_06207_amd/csrc/cbaa_partition.hip":
        "6b0e18e633405e019f80713effa66c493443e9cbd0939c55824acc37c38e820c",
    "paper_1901_06207_amd/csrc/cbaa_internal.hpp":
        "04742cfdeb7a9049a49c18455a2a890d340d8c3e9ea9799752d7d5507db85aca"}}


def measured_traffic(record, default_workload):
    """The recorded counter bytes if the measured sources are unchanged."""
    if not default_workload:
        return None
    for rel, digest in record["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return record["bytes"]
METRIC = "Gpkt/s cube update, ms/window restore, p99 latency; learned vs linear-count err"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--routers", type=int, default=2)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = 64Mi packets)")
    ap.add_argument("--theta", type=float, default=1024.0)
    ap.add_argument("--eager", action="store_true", help="launch the step without a HIP graph")
    ap.add_argument("--tune", action="store_true", help="autotune the update's shapes first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-streams summary in the default line")
    ap.add_argument("--pipeline", action="store_true",
                    help="also time windows back to back, each window end overlapping the next "
                         "window's update (off by default)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="packets of the window the CPU oracle step is timed on (0 = all)")
    ap.add_argument("--workload", choices=["core-edge", "batched", "sweep"], default="core-edge",
                    help="batched: 32 router streams of 1M-64M packets in one graph replay; "
                         "sweep: accuracy of the restored lists over r, g and the threshold rule")
    ap.add_argument("--sweep-windows", default="small:1,2,3;core-edge:11,12,13",
                    help="windows of the sweep: kind:seeds;kind:seeds")
    ap.add_argument("--streams", type=int, default=32)
    ap.add_argument("--update-streams", choices=["one", "per-router"], default="one",
                    help="one: all routers' packets in one batched update call; per-router: "
                         "each router's batch on its own stream, overlapping on the device")
    ap.add_argument("--window-end-streams", choices=["one", "per-side"], default="per-side",
                    help="per-side: the two global cubes' merge and restore run on two streams "
                         "and overlap (one side's scan with the other's tuple check)")
    ap.add_argument("--store-merged", action="store_true",
                    help="the window end also stores each side's merged (global) cube")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in the design notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import tracegen
    from paper_1901_06207_amd import autotune, cbaa

    cbaa.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = cbaa.cbaa_config_default()
    cube_bytes = cbaa.cbaa_cube_bytes(cfg)
    if args.calibrate_copy:
        calibrate_copy(dev)
    if args.workload == "batched":
        return bench_batched(cfg, dev, args)
    if args.workload == "sweep":
        return bench_sweep(dev, args)

    t0 = time.time()
    trace = tracegen.window_core_edge(args.seed, scale=args.scale)
    parts = tracegen.split_routers(trace.pairs, args.routers, seed=args.seed)
    log(f"generated {trace.n} packets in {time.time() - t0:.1f}s; routers "
        f"{[len(q) for q in parts]}")
    d_parts = [cbaa.pairs_to_device(q, dev) for q in parts]
    local = [(cbaa.new_cube(cfg, dev), cbaa.new_cube(cfg, dev)) for _ in parts]
    table = [(q, a, b, cbaa.SIDE_SRC, cbaa.BATCH_FRESH) for q, (a, b) in zip(d_parts, local)]
    tuning = None
    tune_info = None
    if args.tune:
        tune_info = autotune.tune_update(cfg, table)
        tuning = tune_info["best"]
        log(f"autotuned: {tune_info['best']} {tune_info['best_ms']:.3f} ms "
            f"(default {tune_info['default_ms']:.3f} ms)")
    per_router = args.update_streams == "per-router" and len(parts) > 1
    if per_router:
        # each local server updates its own cubes on its own stream: the
        # routers' launch sequences overlap on the device
        tables = [[t] for t in table]
        scratch_us = [cbaa.scratch_tensor(cbaa.cbaa_update_batch_scratch_bytes(cfg, t, tuning), dev)
                      for t in tables]
        ustreams = [torch.cuda.Stream(device=dev) for _ in tables]
    else:
        scratch_u = cbaa.scratch_tensor(cbaa.cbaa_update_batch_scratch_bytes(cfg, table, tuning), dev)

    g_src = cbaa.new_cube(cfg, dev, init=False)
    g_dst = cbaa.new_cube(cfg, dev, init=False)
    capacity = 1 << 14
    rs_bytes = cbaa.cbaa_restore_scratch_bytes(cfg, capacity)
    scratch_r = [cbaa.scratch_tensor(rs_bytes, dev) for _ in range(2)]
    # each side's list and counters contiguous in one device buffer,
    # [list 0 | stats 0 | list 1 | stats 1], so that a side's results come
    # back with one copy (both sides' with one when the sides run in order)
    lb = capacity * cbaa.HOST_BYTES
    sb = cbaa.STATS_BYTES
    pb = (lb + sb + 255) // 256 * 256
    d_res = torch.empty(2 * pb, dtype=torch.uint8, device=dev)
    h_res = torch.empty(2 * pb, dtype=torch.uint8, pin_memory=True)
    outs = [d_res[i * pb: i * pb + lb] for i in range(2)]
    stats = [d_res[i * pb + lb: i * pb + lb + sb].view(torch.int64) for i in range(2)]
    h_outs = [h_res[i * pb: i * pb + lb] for i in range(2)]
    h_stats = [h_res[i * pb + lb: i * pb + lb + sb].view(torch.int64) for i in range(2)]
    d_sides = [d_res[i * pb: (i + 1) * pb] for i in range(2)]
    h_sides = [h_res[i * pb: (i + 1) * pb] for i in range(2)]

    ev = {}

    def mark(name, stream):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev.setdefault(name, []).append(e)

    def step(stream, timed=False):
        # the phase pass (timed) runs the two sides one after the other, so
        # that its per-side figures are latencies; the step overlaps them
        overlap = per_side and not timed
        if timed:
            mark("update", stream)
        if per_router:
            fork = torch.cuda.Event()
            fork.record(stream)
            joins = []
            for t, sc, us in zip(tables, scratch_us, ustreams):
                us.wait_event(fork)
                cbaa.cbaa_update_batch(cfg, t, sc, tuning, us)
                e = torch.cuda.Event()
                e.record(us)
                joins.append(e)
            for e in joins:
                stream.wait_event(e)
        else:
            cbaa.cbaa_update_batch(cfg, table, scratch_u, tuning, stream)
        if timed:
            mark("window_end", stream)
        # global server: OR-merge the routers' cubes and restore, per side.
        # The merged cube is an intermediate of the restore: unless asked to,
        # it is not stored, and the restore reads each column it needs as the
        # OR of the router cubes.
        side_args = [(cfg, cube if args.store_merged else None, [x[i] for x in local],
                      args.theta, cbaa.THR_THM2, scratch_r[i], outs[i], capacity, stats[i])
                     for i, cube in enumerate((g_src, g_dst))]
        if overlap:
            # the sides on two streams, at once: the scans stream the cubes
            # with the non-temporal hint, so one side's scan leaves the other
            # side's tuple check its hot columns in L2 (ordering the second
            # scan after the first side's hot lists no longer pays)
            fork = torch.cuda.Event()
            fork.record(stream)
            for st in wstreams:
                st.wait_event(fork)
            cbaa.cbaa_merge_scan(*side_args[0], wstreams[0])
            cbaa.cbaa_merge_scan(*side_args[1], wstreams[1])
            cbaa.cbaa_restore_scanned(*side_args[0], wstreams[0])
            cbaa.cbaa_restore_scanned(*side_args[1], wstreams[1])
            # each side's list to the host as soon as that side is done
            for i, st in enumerate(wstreams):
                with torch.cuda.stream(st):
                    h_sides[i].copy_(d_sides[i], non_blocking=True)
        else:
            for a in side_args:
                cbaa.cbaa_merge_restore(*a, stream)
        if overlap:
            for st in wstreams:
                e = torch.cuda.Event()
                e.record(st)
                stream.wait_event(e)
        if timed:
            mark("copy", stream)
        if not overlap:
            with torch.cuda.stream(stream):
                h_res.copy_(d_res, non_blocking=True)
        if timed:
            mark("end", stream)

    stream = torch.cuda.Stream(device=dev)
    # the two sides' window ends are independent (one global cube each)
    per_side = args.window_end_streams == "per-side"
    wstreams = [torch.cuda.Stream(device=dev) for _ in range(2)] if per_side else []
    for _ in range(args.warmup):
        step(stream)
    torch.cuda.synchronize(dev)
    n_found = [int(h_stats[i][0]) for i in range(2)]
    if max(n_found) > capacity:
        raise SystemExit(f"restore capacity {capacity} too small for {n_found}")
    ref_lists = [h_outs[i][: n_found[i] * 16].clone() for i in range(2)]
    log(f"super hosts found: source-keyed {n_found[0]}, destination-keyed {n_found[1]}")

    graph = None
    if not args.eager:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            step(stream)
        torch.cuda.synchronize(dev)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize(dev)
        for i in range(2):   # the replayed step reproduces the eager lists
            if int(h_stats[i][0]) != n_found[i] or not torch.equal(
                    h_outs[i][: n_found[i] * 16], ref_lists[i]):
                raise SystemExit("graph replay differs from the eager step")

    # timed region: exactly K steps
    torch.cuda.synchronize(dev)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step(stream)
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = trace.n / (elapsed / args.steps) / 1e9

    # per-phase breakdown with events on the launch stream (eager pass)
    ev.clear()
    phase_steps = max(3, min(args.steps, 10))
    for _ in range(phase_steps):
        step(stream, timed=True)
    torch.cuda.synchronize(dev)

    def span(a, b):
        return np.array([x.elapsed_time(y) for x, y in zip(ev[a], ev[b])])

    upd_ms = span("update", "window_end")
    window_end_ms = span("window_end", "copy") / 2.0   # merge + restore per global cube
    copy_ms = span("copy", "end")
    # the two halves of the window end on their own (outside the step): the
    # OR-merge of both sides, and the restore of one merged cube
    ev.clear()
    for _ in range(phase_steps):
        mark("m0", stream)
        cbaa.cbaa_merge_or(cfg, g_src, [x[0] for x in local], stream)
        cbaa.cbaa_merge_or(cfg, g_dst, [x[1] for x in local], stream)
        mark("m1", stream)
        for i, cube in enumerate((g_src, g_dst)):
            cbaa.cbaa_restore(cfg, cube, args.theta, cbaa.THR_THM2, scratch_r[i], outs[i],
                              capacity, stats[i], stream)
        mark("m2", stream)
    torch.cuda.synchronize(dev)
    merge_ms = span("m0", "m1")
    restore_ms = span("m1", "m2") / 2.0
    # the window end in the other mode (merged cube stored or not), per side
    ev.clear()
    for _ in range(phase_steps):
        mark("w0", stream)
        for i, cube in enumerate((g_src, g_dst)):
            cbaa.cbaa_merge_restore(cfg, None if args.store_merged else cube,
                                    [x[i] for x in local], args.theta, cbaa.THR_THM2,
                                    scratch_r[i], outs[i], capacity, stats[i], stream)
        mark("w1", stream)
    torch.cuda.synchronize(dev)
    window_end_other_ms = span("w0", "w1") / 2.0
    mall = mall_cold_warm(cfg, dev, args, stream, table, scratch_u, tuning, local, scratch_r,
                          outs, stats, capacity, phase_steps)
    pcie = host_fed(dev, stream, graph, parts, d_parts, trace.n, phase_steps, ms_per_step)
    upd_gpkts = trace.n / (upd_ms.mean() * 1e-3) / 1e9

    # roofline of the dominant kernel set, the batched update call: algorithmic
    # bytes = 8 B per packet read + every router cube written once
    upd_alg_bytes = 8.0 * trace.n + 2.0 * len(parts) * cube_bytes
    achieved = upd_alg_bytes / (upd_ms.mean() * 1e-3) / 1e9
    traffic = measured_traffic(UPDATE_TRAFFIC, len(parts) == 2 and tuning is None
                               and args.scale == 1.0)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                # the measured HBM bytes over the same duration: how close the
                # kernels run to the memory system on the bytes they do move
                "traffic_frac": (round(traffic / (upd_ms.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                 if traffic else None),
                "kernel": ("cbaa_update_batch (histogram, scan, scatter, apply), "
                           + ("one call per router on its own stream, overlapping; timed from "
                              "the fork to the join" if per_router else "one call for all routers")),
                "per_launch": {"packets": int(trace.n), "alg_bytes": int(upd_alg_bytes),
                               "avg_ms": round(float(upd_ms.mean()), 4)}}

    # atomic roofline: the same packets through the direct path (one
    # device-scope 32-bit atomic OR per bit-set into the cube, the paper's
    # Sec. 4.1 scheme), the rate the partitioned path is measured against
    n_arr = cfg["n_ra"] + cfg["n_va"] if isinstance(cfg, dict) else cfg.n_arrays
    bitsets = n_arr * 2 * trace.n
    d_ms = []
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for q, (a, b) in zip(d_parts, local):
            cbaa.cbaa_update2(cfg, a, b, q, None, stream)
        e1.record(stream)
        e1.synchronize()
        d_ms.append(e0.elapsed_time(e1))
    atomic = {"direct_atomic_gops": round(bitsets / (d_ms[-1] * 1e-3) / 1e9, 2),
              "partitioned_bitset_gops": round(bitsets / (upd_ms.mean() * 1e-3) / 1e9, 2),
              "bitsets_per_window": int(bitsets)}
    atomic["ratio"] = round(atomic["partitioned_bitset_gops"] / atomic["direct_atomic_gops"], 2)
    roofline["atomic"] = atomic
    # measured ceilings: the update against a streaming copy of this GPU, and
    # the bit-set rate against random atomics into as many bytes as the
    # window's router cubes (the one-thread-per-packet scheme's ceiling)
    ceil = measure_ceilings(dev, stream)
    roofline["ceilings"] = ceil
    roofline["frac_of_measured_copy"] = round(achieved / ceil["hbm_copy_gbs"], 4)
    cube_mib = 2 * len(parts) * cube_bytes / 2 ** 20
    ceil_key = "atomic_or_gops_128MiB" if cube_mib <= 192 else "atomic_or_gops_512MiB"
    atomic["ceiling_gops"] = ceil[ceil_key]
    atomic["direct_ceiling_gpkt_s"] = round(ceil[ceil_key] / (2 * n_arr), 3)
    atomic["update_over_direct_ceiling"] = round(
        atomic["partitioned_bitset_gops"] / ceil[ceil_key], 2)
    # restore's scan (per-column zeros of one 128 MiB cube) against HBM
    zb = torch.empty(cbaa.cbaa_restore_scratch_bytes(cfg, 0), dtype=torch.uint8, device=dev)
    ones_t = torch.empty(4096, dtype=torch.int32, device=dev)
    s_ms = []
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cbaa.cbaa_column_zeros(cfg, g_src, zb, ones_t, stream)
        e1.record(stream)
        e1.synchronize()
        s_ms.append(e0.elapsed_time(e1))
    scan_gbs = cube_bytes / (float(np.median(s_ms[1:])) * 1e-3) / 1e9
    scan = {"cube_bytes": int(cube_bytes), "ms": round(float(np.median(s_ms[1:])), 4),
            "achieved_gbs": round(scan_gbs, 1), "frac": round(scan_gbs / HBM_PEAK_GBS, 4)}

    # pipelined windows: a second set of router cubes, so that the window end
    # of one window (latency-bound tuple check, list copy) runs on the side
    # streams while the next window's update streams over the other set
    pipelined = None
    if per_side and graph is not None and not per_router and args.pipeline:
        pipelined = bench_pipelined(cfg, dev, args, d_parts, local, table, scratch_u, tuning,
                                    scratch_r, outs, stats, capacity, d_sides, h_sides,
                                    h_outs, h_stats, ref_lists, n_found, stream, wstreams,
                                    trace.n, ms_per_step)

    # the restored lists of the step (graph replay) against the window's exact
    # per-host counts, per side (the generator's construction counts: every
    # peer of a host is a distinct address, pinned equal to a sort-unique count)
    accuracy = {}
    for side, name in ((0, "source_keyed"), (1, "destination_keyed")):
        lst = ref_lists[side].numpy().view(cbaa.HOST_DTYPE)
        hosts, counts = tracegen.construction_truth(trace, side)
        accuracy[name] = {k: (round(v, 6) if isinstance(v, float) else v)
                          for k, v in detection_accuracy(lst["ip"], lst["est"], hosts, counts,
                                                         args.theta).items()}
        del hosts, counts
    accuracy["rule"] = "THM2"
    accuracy["note"] = ("restored lists of the timed step scored against exact per-host "
                        "distinct-peer counts (Sec. 5.2 FNR, FPR over |H|, FTR)")

    serving = None if args.no_serve else bench_serving(cfg, dev, args)
    learned = None if args.no_learned else bench_learned(cfg, trace, g_src, local, dev, args)
    cpu = None if args.no_cpu_baseline else cpu_baseline(trace.pairs, args.cpu_sample, args.theta)
    batched = None
    if not args.no_batched and args.scale == 1.0:
        batched = batched_summary(bench_batched(cfg, dev, args, emit=False))

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpkt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": (f"core-edge window: {trace.n} packets (8M Zipf(1.1) sources, 1000 planted "
                         "hosts 1k-200k peers, 10% duplicates), source- and destination-keyed "
                         f"cubes, {args.routers} edge routers OR-merged, theta {args.theta:g}, "
                         "r=4 |RA|=3 |VA|=1 g=c=4096"),
            "packets": trace.n, "routers": args.routers, "seed": args.seed,
            "launch": "eager" if graph is None else "hip-graph",
            "update_streams": args.update_streams if len(parts) > 1 else "one",
            "window_end_streams": args.window_end_streams,
            "tuning": tuning or "default",
            "merged_cube": ("stored" if args.store_merged else
                            "not stored: the restore reads columns as the OR of the router cubes"),
        },
        "phases": {
            "update_ms": round(float(upd_ms.mean()), 4),
            "update_gpkt_s": round(float(upd_gpkts), 3),
            "window_end_ms_per_side": round(float(window_end_ms.mean()), 4),
            "window_end_note": ("per-side figures come from a pass that runs the sides one after "
                                "the other; the timed step overlaps them on two streams"
                                if per_side else "the step runs the sides one after the other"),
            ("window_end_unstored_ms_per_side" if args.store_merged
             else "window_end_stored_ms_per_side"): round(float(window_end_other_ms.mean()), 4),
            "merge_ms": round(float(merge_ms.mean()), 4),
            "restore_ms_per_window": round(float(restore_ms.mean()), 4),
            "restore_ms_p99": round(float(np.percentile(restore_ms, 99)), 4),
            "lists_to_host_ms": round(float(copy_ms.mean()), 4),
            # what the step spends on both sides' window ends together: the
            # step's time less the update and the copy (timed in the phase pass)
            "window_end_ms_both_sides_in_step": round(
                ms_per_step - float(upd_ms.mean()) - float(copy_ms.mean()), 4),
            "restore_scan": scan,
            # the whole window end of one side against the HBM roofline: its
            # algorithmic bytes are the router cubes read once (plus the merged
            # cube written once when it is stored)
            "window_end_roofline": {
                "alg_bytes": int((len(parts) + (1 if args.store_merged else 0)) * cube_bytes),
                "achieved_gbs": round((len(parts) + (1 if args.store_merged else 0)) * cube_bytes
                                      / (float(window_end_ms.mean()) * 1e-3) / 1e9, 1),
                "frac": round((len(parts) + (1 if args.store_merged else 0)) * cube_bytes
                              / (float(window_end_ms.mean()) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "super_hosts": {"source_keyed": n_found[0], "destination_keyed": n_found[1]},
            "mall": mall,
            "host_fed": pcie,
        },
        "roofline": roofline,
        "pipelined": pipelined,
        "batched": batched,
        "accuracy": accuracy,
        "serving": serving,
        "learned": learned,
        "cpu_baseline": cpu,
    }
    if tune_info:
        out["autotune"] = {"best": tune_info["best"], "best_ms": round(tune_info["best_ms"], 4),
                           "default_ms": round(tune_info["default_ms"], 4)}
    print(json.dumps(out), flush=True)


def mall_cold_warm(cfg, dev, args, stream, table, scratch_u, tuning, local, scratch_r, outs,
                   stats, capacity, reps):
    """The update call and one side's window end, cold and warm in the 256 MB
    MALL (Infinity Cache): a cold run follows a 512 MiB device write that
    evicts it, a warm run repeats the same call at once."""
    import numpy as np
    import torch

    from paper_1901_06207_amd import cbaa

    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    side = (cfg, None, [x[0] for x in local], args.theta, cbaa.THR_THM2, scratch_r[0], outs[0],
            capacity, stats[0])
    calls = {"update": lambda: cbaa.cbaa_update_batch(cfg, table, scratch_u, tuning, stream),
             "window_end_source_side": lambda: cbaa.cbaa_merge_restore(*side, stream)}
    res = {}
    for name, fn in calls.items():
        cold, warm = [], []
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            with torch.cuda.stream(stream):
                flush.fill_(1)
            ev[0].record(stream)
            fn()
            ev[1].record(stream)
            fn()
            ev[2].record(stream)
            ev[2].synchronize()
            cold.append(ev[0].elapsed_time(ev[1]))
            warm.append(ev[1].elapsed_time(ev[2]))
        res[name] = {"cold_ms": round(float(np.median(cold)), 4),
                     "warm_ms": round(float(np.median(warm)), 4)}
    del flush
    res["note"] = "cold: after a 512 MiB device write; warm: the same call repeated at once; medians"
    return res


def host_fed(dev, stream, graph, parts, d_parts, n_packets, reps, step_ms):
    """The window's pairs from pinned host memory: the copy alone, and the
    step with the next window's copy running beside it on a copy stream
    (double buffering; the copy lands in a spare buffer of the same size)."""
    import numpy as np
    import torch

    h = [torch.from_numpy(np.ascontiguousarray(q, dtype=np.uint32).view(np.int32)).pin_memory()
         for q in parts]
    spare = [torch.empty_like(d) for d in d_parts]
    cstream = torch.cuda.Stream(device=dev)
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cstream)
        with torch.cuda.stream(cstream):
            for src, dst in zip(h, spare):
                dst.copy_(src, non_blocking=True)
        e1.record(cstream)
        e1.synchronize()
        t.append(e0.elapsed_time(e1))
    h2d_ms = float(np.median(t))
    nbytes = sum(int(x.numel()) * 4 for x in h)
    out = {"h2d_ms": round(h2d_ms, 4), "h2d_gbs": round(nbytes / (h2d_ms * 1e-3) / 1e9, 1),
           "serial_gpkt_s": round(n_packets / ((h2d_ms + step_ms) * 1e-3) / 1e9, 3),
           "overlapped_gpkt_s": None}
    if graph is not None:
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            with torch.cuda.stream(cstream):
                for src, dst in zip(h, spare):
                    dst.copy_(src, non_blocking=True)
            graph.replay()
            torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out["overlapped_ms_per_window"] = round(ms, 4)
        out["overlapped_gpkt_s"] = round(n_packets / (ms * 1e-3) / 1e9, 3)
    out["note"] = ("PCIe-inclusive rates: serial = copy then step (derived from the two times), "
                   "overlapped = the next window's copy beside the step (measured)")
    del spare, h
    return out


def bench_pipelined(cfg, dev, args, d_parts, local, table, scratch_u, tuning, scratch_r, outs,
                    stats, capacity, d_sides, h_sides, h_outs, h_stats, ref_lists, n_found,
                    stream, wstreams, n_packets, step_ms):
    """Windows back to back with their window ends overlapping the next
    window's update. Two sets of router cubes, A and B; one graph replay runs
    two windows: B's window end (its update was the previous replay's) on the
    side streams while A is updated, then A's window end while B is updated.
    B's update waits for B's window end, and the replay ends with A's, so no
    cube is written while it is read. Every window still runs the whole path
    (update, merge and restore per side, lists to the host)."""
    import numpy as np
    import torch

    from paper_1901_06207_amd import cbaa

    local_b = [(cbaa.new_cube(cfg, dev), cbaa.new_cube(cfg, dev)) for _ in local]
    table_b = [(q, a, b, cbaa.SIDE_SRC, cbaa.BATCH_FRESH) for q, (a, b) in zip(d_parts, local_b)]

    def window_end(cubes):
        for i, st in enumerate(wstreams):
            a = (cfg, None, [x[i] for x in cubes], args.theta, cbaa.THR_THM2, scratch_r[i],
                 outs[i], capacity, stats[i])
            cbaa.cbaa_merge_scan(*a, st)
            cbaa.cbaa_restore_scanned(*a, st)
            with torch.cuda.stream(st):
                h_sides[i].copy_(d_sides[i], non_blocking=True)

    def join_sides():
        for st in wstreams:
            e = torch.cuda.Event()
            e.record(st)
            stream.wait_event(e)

    def period():
        fork = torch.cuda.Event()
        fork.record(stream)
        for st in wstreams:
            st.wait_event(fork)
        window_end(local_b)
        cbaa.cbaa_update_batch(cfg, table, scratch_u, tuning, stream)
        a_done = torch.cuda.Event()
        a_done.record(stream)
        join_sides()                       # B is read no more: its update may start
        cbaa.cbaa_update_batch(cfg, table_b, scratch_u, tuning, stream)
        for st in wstreams:
            st.wait_event(a_done)
        window_end(local)
        join_sides()

    cbaa.cbaa_update_batch(cfg, table_b, scratch_u, tuning, stream)   # B's first window
    torch.cuda.synchronize(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        period()
    torch.cuda.synchronize(dev)
    for _ in range(max(1, args.warmup)):
        g.replay()
    torch.cuda.synchronize(dev)
    same = all(int(h_stats[i][0]) == n_found[i] and torch.equal(
        h_outs[i][: n_found[i] * 16], ref_lists[i]) for i in range(2))
    if not same:
        raise SystemExit("pipelined windows differ from the step's lists")
    replays = max(1, args.steps // 2)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize(dev)
    ms = (time.perf_counter() - t0) * 1e3 / (2 * replays)
    # the two sets take the same packets, so their cubes must be equal word for word
    same_cubes = all(torch.equal(x, y) for pa, pb in zip(local, local_b) for x, y in zip(pa, pb))
    if not same_cubes:
        raise SystemExit("pipelined windows: the two cube sets differ")
    del g, local_b
    return {"windows": 2 * replays, "ms_per_window": round(ms, 4),
            "gpkt_s": round(n_packets / (ms * 1e-3) / 1e9, 3),
            "over_step": round(step_ms / ms, 3), "lists_equal_step": bool(same),
            "cube_sets_equal": bool(same_cubes),
            "note": ("two sets of router cubes; each window's end (both sides on their own "
                     "streams, lists to the host) overlaps the next window's update; steady "
                     "state over whole graph replays of two windows each")}


def detection_accuracy(ips, est, hosts, counts, theta, hosts_sorted=False):
    """Sec. 5.2's rates of a restored list against exact per-host distinct-peer
    counts: H = hosts with at least theta peers; FNR = |H minus R| / |H|; FPR =
    |{h in R : |OP(h)| < theta}| / |H| (the paper's denominators; a restored
    address never seen as a host counts as a false positive); FTR = FNR + FPR;
    also precision and recall, and the relative error of the estimate on the
    true super hosts that were restored. `hosts_sorted`: hosts are ascending
    (sort once, score many lists)."""
    import numpy as np
    found = np.asarray(ips, np.uint32)
    found_est = np.asarray(est, np.float64)
    hosts = np.asarray(hosts, np.uint32)
    counts = np.asarray(counts, np.int64)
    if not hosts_sorted:
        order = np.argsort(hosts, kind="stable")
        hosts, counts = hosts[order], counts[order]
    n_true = int(np.count_nonzero(counts >= theta))
    # the count of every restored address (0 when it never appears as a host)
    cnt = np.zeros(found.size, np.int64)
    if found.size and hosts.size:
        pos = np.minimum(np.searchsorted(hosts, found), hosts.size - 1)
        hit = hosts[pos] == found
        cnt[hit] = counts[pos[hit]]
    tp = int(np.count_nonzero(cnt >= theta))
    fp = int(found.size - tp)
    fn = n_true - tp
    nh = max(n_true, 1)
    rel = np.abs(found_est[cnt >= theta] - cnt[cnt >= theta]) / cnt[cnt >= theta]
    return {"theta": theta, "n_true": n_true, "n_restored": int(found.size),
            "fnr": fn / nh, "fpr": fp / nh, "ftr": (fn + fp) / nh,
            "precision": tp / max(int(found.size), 1), "recall": tp / nh,
            "est_rel_err_mean": float(rel.mean()) if rel.size else None,
            "est_rel_err_p50": float(np.median(rel)) if rel.size else None,
            "est_rel_err_p99": float(np.percentile(rel, 99)) if rel.size else None}


def measure_ceilings(dev, stream, reps=5):
    """The two ceilings the update is priced against, measured on this GPU with
    the library's probes: a 1 GiB streaming copy (bytes read + written per
    second), and random no-return 32-bit atomic ORs at precomputed addresses
    into a 128 MiB buffer (one cube; fits the 256 MiB last-level cache) and a
    512 MiB one (four cubes; does not)."""
    import numpy as np
    import torch

    from paper_1901_06207_amd import cbaa

    def timed(fn):
        ms = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms[1:]))

    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    # the best of a few grid sizes, with cached and with nontemporal accesses
    copies = {}
    for blocks in (1024, 2048, 4096, 8192, 16384):
        for flags in (0, cbaa.PROBE_NONTEMPORAL):
            copies[(blocks, flags)] = timed(
                lambda: cbaa.cbaa_probe_copy(dst, src, nb, blocks, flags, stream))
    (best_blocks, best_flags), copy_ms = min(copies.items(), key=lambda kv: kv[1])

    def torch_copy():
        with torch.cuda.stream(stream):
            dst.copy_(src)
    torch_ms = timed(torch_copy)
    del src, dst
    n_ops = 1 << 26
    addr = torch.empty(n_ops, dtype=torch.int32, device=dev)
    out = {"hbm_copy_gbs": round(2 * nb / (copy_ms * 1e-3) / 1e9, 1),
           "hbm_copy_bytes": 2 * nb,
           "hbm_copy_shape": {"blocks": best_blocks, "threads": 256,
                              "nontemporal": bool(best_flags)},
           "hbm_copy_torch_gbs": round(2 * nb / (torch_ms * 1e-3) / 1e9, 1),
           "atomic_ops": n_ops}
    for mib in (128, 512):
        words = (mib << 20) // 4
        buf = torch.zeros(words, dtype=torch.int32, device=dev)
        cbaa.cbaa_probe_addresses(addr, int(words).bit_length() - 1, 0x9E3779B9, stream)
        a_ms = timed(lambda: cbaa.cbaa_probe_atomic_or(buf, addr, stream))
        out[f"atomic_or_gops_{mib}MiB"] = round(n_ops / (a_ms * 1e-3) / 1e9, 2)
        del buf
    torch.cuda.synchronize(dev)
    return out


def calibrate_copy(dev, nbytes=1 << 30):
    """A plain device-to-device copy of known size: its FETCH_SIZE/WRITE_SIZE
    counters scale the update's counters to bytes."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize(dev)
    log(f"calibration copy: {nbytes} bytes read and written per copy, 3 copies")


def bench_batched(cfg, dev, args, emit=True):
    """K edge-router streams with log-uniform 1M-64M packets (core-edge shape,
    one seed per stream), both cubes per stream, in one graph replay: zero the
    cubes, one batched update with autotuned shapes, restore every stream's
    two cubes, OR-merge all streams into the global cubes. The global cubes
    are not restored: 32 independent windows of up to 64M packets put ~7x the
    flows a 128 MiB cube is dimensioned for into it (every column saturates,
    tens of millions of "hosts" pass the threshold), so their restore measures
    nothing the method is meant for."""
    import numpy as np
    import torch

    import tracegen
    from paper_1901_06207_amd import autotune, cbaa

    rng = np.random.default_rng(args.seed)
    K = args.streams
    sizes = np.exp(rng.uniform(np.log(1 << 20), np.log(64 << 20), K)).astype(np.int64)
    t0 = time.time()
    d_pairs = []
    for i, n in enumerate(sizes):
        tr = tracegen.window_core_edge(args.seed * 1000 + i, scale=float(n) / (64 << 20))
        d_pairs.append(cbaa.pairs_to_device(tr.pairs, dev))
        del tr
    total = int(sum(int(q.shape[0]) for q in d_pairs))
    log(f"generated {K} streams, {total} packets in {time.time() - t0:.0f}s")
    cubes = [(cbaa.new_cube(cfg, dev), cbaa.new_cube(cfg, dev)) for _ in range(K)]
    table = [(q, a, b, cbaa.SIDE_SRC, cbaa.BATCH_FRESH) for q, (a, b) in zip(d_pairs, cubes)]
    tune = autotune.tune_update(cfg, table, repeats=2)
    tuning = tune["best"]
    log(f"autotuned {tuning}: {tune['best_ms']:.2f} ms (default {tune['default_ms']:.2f} ms)")
    scratch = cbaa.scratch_tensor(cbaa.cbaa_update_batch_scratch_bytes(cfg, table, tuning), dev)
    g = [cbaa.new_cube(cfg, dev, init=False) for _ in range(2)]
    cap = 1 << 14
    rs = cbaa.scratch_tensor(cbaa.cbaa_restore_scratch_bytes(cfg, cap), dev)
    outs = torch.empty((2 * K, cap * cbaa.HOST_BYTES), dtype=torch.uint8, device=dev)
    stats = torch.zeros((2 * K, len(cbaa.STATS_FIELDS)), dtype=torch.int64, device=dev)
    ev = {}

    def mark(name, st):
        e = torch.cuda.Event(enable_timing=True)
        e.record(st)
        ev.setdefault(name, []).append(e)

    def window(st, timed=False):
        if timed:
            mark("update", st)
        cbaa.cbaa_update_batch(cfg, table, scratch, tuning, st)
        if timed:
            mark("local_restore", st)
        for i, (a, b) in enumerate(cubes):
            for j, c in enumerate((a, b)):
                cbaa.cbaa_restore(cfg, c, args.theta, cbaa.THR_THM2, rs, outs[2 * i + j], cap,
                                  stats[2 * i + j], st)
        if timed:
            mark("merge", st)
        cbaa.cbaa_merge_or(cfg, g[0], [c[0] for c in cubes], st)
        cbaa.cbaa_merge_or(cfg, g[1], [c[1] for c in cubes], st)
        if timed:
            mark("end", st)

    st = torch.cuda.Stream(device=dev)
    window(st)
    torch.cuda.synchronize(dev)
    want = stats.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        window(st)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize(dev)
    if not torch.equal(stats, want):
        raise SystemExit("graph replay differs from the eager window")
    t_start = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize(dev)
    el = (time.perf_counter() - t_start) / args.steps
    ev.clear()
    for _ in range(3):
        window(st, timed=True)
    torch.cuda.synchronize(dev)

    def span(a, b):
        return float(np.mean([x.elapsed_time(y) for x, y in zip(ev[a], ev[b])]))

    upd = span("update", "local_restore")
    hosts = stats[:, 0].cpu().numpy()
    alg = 8.0 * total + 2.0 * K * cbaa.cbaa_cube_bytes(cfg)
    out = {
        "metric": METRIC, "value": round(total / el / 1e9, 3), "unit": "Gpkt/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": (f"batched: {K} router streams, log-uniform 1M-64M packets "
                                f"({total} in all, core-edge shape, seed per stream), both cubes, "
                                "per-stream restores, OR-merge of all streams into the global "
                                "cubes, one HIP-graph replay per window"),
                   "packets": total, "streams": K, "tuning": tuning,
                   "stream_packets": [int(x) for x in sizes]},
        "phases": {"update_ms": round(upd, 3), "update_gpkt_s": round(total / upd / 1e6, 3),
                   "local_restores_ms": round(span("local_restore", "merge"), 3),
                   "local_restore_ms_per_cube": round(span("local_restore", "merge") / (2 * K), 4),
                   "merge_ms": round(span("merge", "end"), 3),
                   "super_hosts_per_stream": [int(x) for x in hosts]},
        "roofline": {"bound": "hbm", "achieved": round(alg / (upd * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (upd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "cbaa_update_batch (histogram, scan, scatter, apply)"},
        "autotune": {"best": tuning, "best_ms": round(tune["best_ms"], 3),
                     "default_ms": round(tune["default_ms"], 3),
                     "candidates": len(tune["candidates"])},
        "cpu_baseline": None,
    }
    if not emit:
        del graph, cubes, table, d_pairs, scratch, g, rs, outs, stats
        torch.cuda.synchronize(dev)
        torch.cuda.empty_cache()
        return out
    print(json.dumps(out), flush=True)


def batched_summary(res):
    """The batched workload's figures carried in the default line."""
    p, r = res["phases"], res["roofline"]
    return {"workload": res["config"]["workload"], "packets": res["config"]["packets"],
            "streams": res["config"]["streams"], "gpkt_s": res["value"],
            "ms_per_window": res["ms_per_step"], "update_ms": p["update_ms"],
            "update_gpkt_s": p["update_gpkt_s"], "update_hbm_frac": r["frac"],
            "local_restore_ms_per_cube": p["local_restore_ms_per_cube"],
            "merge_ms": p["merge_ms"], "tuning": res["autotune"]["best"],
            "tuned_ms": res["autotune"]["best_ms"], "default_ms": res["autotune"]["default_ms"]}


# RA start bits per r for the sweep: |EP| = (10, 9, 10), (10, 9, 9), (9, 9, 9)
# and |CP| = (2, 3, 2), (2, 3, 3), (3, 3, 3) with 12-bit column indices
SWEEP_CL_BS = {3: [3, 13, 22], 4: [4, 14, 23], 5: [5, 14, 23]}


def sweep_config(r, log2_g):
    return dict(r=r, n_ra=3, n_va=1, log2_g=log2_g, cbn=[12, 12, 12, 12], cl_bs=SWEEP_CL_BS[r],
                seed_mangle=0x243F6A88, seed_bv=0x85A308D3, seed_va=[0x13198A2E, 0x03707344])


def bench_sweep(dev, args):
    """Accuracy of the GPU's restored lists as the dimensions vary (Sec. 3.1-3.3
    parameters; Sec. 5.2 rates): r in {3, 4, 5} (8-32 sketches), g in {2^11,
    2^12, 2^13} bits per column, c = 2^12 columns per array, |RA| = 3, |VA| = 1,
    under both threshold rules (THM2 and the printed Sec. 3.3 form), on
    1M-packet windows (source-keyed) and 64Mi-packet core-edge windows (both
    sides). Each row: array fill, the restore's counters and status, FNR, FPR,
    FTR, precision, recall and the estimate's error against exact counts."""
    import numpy as np
    import torch

    import tracegen
    from paper_1901_06207_amd import cbaa

    windows = []
    for part in args.sweep_windows.split(";"):
        kind, seeds = part.split(":")
        windows += [(kind, int(x)) for x in seeds.split(",")]
    rows = []
    t_all = time.time()
    for kind, seed in windows:
        t0 = time.time()
        tr = (tracegen.window_small(seed) if kind == "small"
              else tracegen.window_core_edge(seed, scale=args.scale))
        sides = (0,) if kind == "small" else (0, 1)
        truth = {}
        for side in sides:
            h, c = tracegen.construction_truth(tr, side)
            o = np.argsort(h, kind="stable")
            truth[side] = (h[o], c[o])
            del h, c, o
        d_pairs = cbaa.pairs_to_device(tr.pairs, dev)
        log(f"sweep window {kind}:{seed} ({tr.n} packets) ready in {time.time() - t0:.1f}s")
        for r in (3, 4, 5):
            for log2_g in (11, 12, 13):
                p = sweep_config(r, log2_g)
                cubes = [cbaa.new_cube(p, dev) for _ in sides]
                nb = cbaa.cbaa_update_scratch_bytes(p, tr.n, len(sides))
                scratch = cbaa.scratch_tensor(nb, dev) if nb else None
                torch.cuda.synchronize(dev)
                tu = time.perf_counter()
                if len(sides) == 2:
                    cbaa.cbaa_update2(p, cubes[0], cubes[1], d_pairs, scratch)
                else:
                    cbaa.cbaa_update(p, cubes[0], d_pairs, cbaa.SIDE_SRC, scratch)
                torch.cuda.synchronize(dev)
                upd_ms = (time.perf_counter() - tu) * 1e3
                del scratch
                g = 1 << log2_g
                A, S, W = 4, 1 << r, 4 * 4096
                for side, cube in zip(sides, cubes):
                    zs = cbaa.scratch_tensor(cbaa.cbaa_restore_scratch_bytes(p, 0), dev)
                    zeros = torch.empty(S * W, dtype=torch.int16, device=dev)
                    ones = torch.empty(S * A, dtype=torch.int32, device=dev)
                    cbaa.cbaa_column_zeros(p, cube, zeros, ones)
                    fill = ones.cpu().numpy().astype(np.float64).reshape(S, A) / (4096.0 * g)
                    del zs, zeros
                    for rule, rname in ((cbaa.THR_THM2, "THM2"), (cbaa.THR_PAPER, "PAPER")):
                        tr0 = time.perf_counter()
                        lst, st = cbaa.restore(p, cube, args.theta, rule, capacity=1 << 14,
                                               max_checks=1 << 26)
                        rest_ms = (time.perf_counter() - tr0) * 1e3
                        acc = detection_accuracy(lst["ip"], lst["est"], *truth[side], args.theta,
                                                 hosts_sorted=True)
                        row = {"window": f"{kind}:{seed}", "packets": int(tr.n),
                               "side": "source" if side == 0 else "destination",
                               "r": r, "g": g, "rule": rname,
                               "fill_mean": round(float(fill.mean()), 5),
                               "fill_max": round(float(fill.max()), 5),
                               "eps_max": float(np.prod(fill, axis=1).max()),
                               "update_ms": round(upd_ms, 2),
                               "path": "partitioned" if nb else "direct",
                               "restore_ms": round(rest_ms, 2),
                               "hot_columns": st["hot_columns"], "tuple_space": st["tuple_space"],
                               "status": st["status"]}
                        row.update({k: (round(v, 6) if isinstance(v, float) else v)
                                    for k, v in acc.items()})
                        rows.append(row)
                        log(f"  r={r} g={g} {row['side']} {rname}: fill {row['fill_mean']:.4f} "
                            f"FNR {row['fnr']:.4f} FPR {row['fpr']:.4f} hosts {row['n_restored']} "
                            f"status {row['status']} ({rest_ms:.1f} ms)")
                del cubes
        del d_pairs, tr, truth
        torch.cuda.empty_cache()
    # summary per (r, g, rule): mean FNR/FPR/FTR over windows and sides
    summary = []
    keys = sorted({(x["r"], x["g"], x["rule"]) for x in rows})
    for r, g, rule in keys:
        sel = [x for x in rows if (x["r"], x["g"], x["rule"]) == (r, g, rule)]
        summary.append({"r": r, "g": g, "rule": rule, "cases": len(sel),
                        "fnr": round(float(np.mean([x["fnr"] for x in sel])), 6),
                        "fpr": round(float(np.mean([x["fpr"] for x in sel])), 6),
                        "ftr": round(float(np.mean([x["ftr"] for x in sel])), 6),
                        "fill_mean": round(float(np.mean([x["fill_mean"] for x in sel])), 5),
                        "incomplete": sum(1 for x in sel if x["status"])})
    out = {"metric": METRIC, "workload": "sweep", "theta": args.theta,
           "windows": [f"{k}:{s}" for k, s in windows], "wall_s": round(time.time() - t_all, 1),
           "summary": summary, "rows": rows}
    print(json.dumps(out), flush=True)


def bench_serving(cfg, dev, args):
    """16 edge routers send Poisson-arriving chunks of 64k-4M pairs; a 60 s
    simulated window is replayed in compressed time; continuous batching
    with a 1 GiB staging budget."""
    import numpy as np
    import torch

    import tracegen
    from paper_1901_06207_amd import cbaa, serve

    n_routers, window_s, lo, hi = 16, 60.0, 65536, 4 << 20
    rate = 0.25                 # chunks per router per simulated second (~240 per window)
    events = serve.poisson_schedule(n_routers, window_s, lo, hi, rate, seed=args.seed)
    total = sum(e[2] for e in events)
    src = tracegen.window_core_edge(args.seed + 1, scale=min(1.0, total / (64 << 20)))
    pairs = src.pairs
    chunks, pos = [], 0
    for _, _, size in events:
        if pos + size > len(pairs):
            pos = 0
        q = np.ascontiguousarray(pairs[pos:pos + size]).view(np.int32)
        pos += size
        chunks.append(torch.from_numpy(q).pin_memory())
    # cubes for 12 of the 16 routers: the least recently used idle router is
    # retired into the global cubes when another one needs room
    per_router = 2 * cbaa.cbaa_cube_bytes(cfg)
    srv = serve.Server(cfg, n_routers, both_sides=True, staging_bytes=1 << 30,
                       cube_budget_bytes=12 * per_router, device=dev)
    # warm the kernels once on a few chunks
    serve.run_window(srv, events[:8], chunks[:8], time_scale=0.0)
    # saturation: every chunk arrives at once
    sat = serve.run_window(srv, events, chunks, time_scale=0.0)
    # offered load: the simulated 60 s window replayed so that packets arrive at
    # `offered` Gpkt/s on average (Poisson arrivals scaled in time)
    offered = 2.0
    time_scale = total / (offered * 1e9) / window_s
    srv.batches = 0
    res = serve.run_window(srv, events, chunks, time_scale=time_scale)
    return {"routers": n_routers, "chunks": res["chunks"], "packets": res["packets"],
            "chunk_pairs": [lo, hi], "simulated_window_s": window_s,
            "replay_window_s": round(window_s * time_scale, 4),
            "saturation_gpkt_s": round(sat["gpkt_s"], 3),
            "offered_gpkt_s": offered, "gpkt_s": round(res["gpkt_s"], 3),
            "p50_ms": round(res["p50_ms"], 3), "p99_ms": round(res["p99_ms"], 3),
            "result_p50_ms": round(res["result_p50_ms"], 3),
            "result_p99_ms": round(res["result_p99_ms"], 3),
            "cube_budget_routers": 12, "cube_peak_mib": round(res["cube_peak_bytes"] / 2 ** 20, 1),
            "retirements": res["retirements"],
            "batches": res["batches"],
            "staging_peak_mib": round(res["staging_peak_bytes"] / 2 ** 20, 1),
            "window_restore_ms": round(res["restore_ms"], 3),
            "note": ("p50/p99: a chunk's arrival to its update done on the device (its "
                     "host-to-device copy included); result_p50/p99: arrival to the restored "
                     "lists of its window on the host (the compressed window replay included)")}


def bench_learned(cfg, trace, g_src, local, dev, args):
    """The learned estimator trained on other windows and evaluated on this
    one: three core-edge training windows of other seeds (the benchmark's
    size, source-keyed cubes), at least 4M host rows drawn stratified by
    cardinality with exact counts; evaluation on up to 2M hosts of the
    benchmark's own window (its merged source-keyed cube), against the paper's
    linear count and the row-aware count at equal false-negative rate. Also
    the network's inference and training throughput on the device."""
    import numpy as np
    import torch

    import tracegen
    from paper_1901_06207_amd import cbaa, learned

    rng = np.random.default_rng(args.seed)
    t0 = time.perf_counter()
    xs, ts = [], []
    train_seeds = [args.seed + 101, args.seed + 102, args.seed + 103]
    for s in train_seeds:
        tw = tracegen.window_core_edge(s, scale=args.scale)
        cube = cbaa.new_cube(cfg, dev)
        nb = cbaa.cbaa_update_scratch_bytes(cfg, tw.n, 1)
        sc = cbaa.scratch_tensor(nb, dev)
        cbaa.cbaa_update(cfg, cube, cbaa.pairs_to_device(tw.pairs, dev), cbaa.SIDE_SRC, sc)
        del sc
        hosts, counts = tracegen.construction_truth(tw, 0)
        idx = learned.stratified_rows(counts, 1_000_000, rng)
        xs.append(learned.features(cfg, cube, hosts[idx]))
        ts.append(torch.from_numpy(np.log1p(counts[idx]).astype(np.float32)).to(dev))
        del cube, tw, hosts, counts
    x_tr = torch.cat(xs).contiguous()
    t_tr = torch.cat(ts).contiguous()
    del xs, ts
    prep_s = time.perf_counter() - t0
    model = learned.Model.new(x_tr.shape[1], seed=1)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    tl = learned.train(model, x_tr, t_tr, epochs=6, batch=65536)
    torch.cuda.synchronize(dev)
    train_s = time.perf_counter() - t0
    # evaluation on the benchmark's window
    hosts, counts = tracegen.construction_truth(trace, 0)
    te = rng.choice(hosts.size, min(hosts.size, 2_000_000), replace=False)
    x_te = learned.features(cfg, g_src, hosts[te])
    est_ml = learned.predict(model, x_te).cpu().numpy()
    est_lc = learned.linear_count(cfg, g_src, hosts[te])
    est_row = learned.row_aware_count(x_te).cpu().numpy()
    rep = learned.compare(est_lc, est_ml, counts[te], args.theta, est_row=est_row)
    # throughput: forward over the evaluation rows, one gradient over a batch
    y = torch.empty(x_te.shape[0], dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        e0.record()
        cbaa.cbaa_mlp_forward(model.n_features, model.master, model.wbf, x_te, y)
        e1.record()
        e1.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    grad = torch.empty(model.master.numel(), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    nb_ = min(x_tr.shape[0], 1 << 20)
    for _ in range(2):
        e0.record()
        cbaa.cbaa_mlp_loss_grad(model.n_features, model.master, model.wbf, x_tr[:nb_],
                                t_tr[:nb_], grad, loss)
        e1.record()
        e1.synchronize()
    grad_ms = e0.elapsed_time(e1)
    mlp_fpr, row_fpr = rep["mlp"]["fpr"], rep["row"]["fpr"]
    return {"train_windows": [f"core-edge seed {s}, {int(64 * args.scale)}Mi packets" for s in train_seeds],
            "train_rows": int(x_tr.shape[0]), "test_rows": int(te.size),
            "test_window": f"the benchmark's window (seed {args.seed})",
            "epochs": tl.epochs, "features": int(x_tr.shape[1]),
            "prep_s": round(prep_s, 2), "train_s": round(train_s, 2),
            "final_loss": round(tl.final_loss, 5),
            "forward_samples_per_s": round(x_te.shape[0] / (fwd_ms * 1e-3), 1),
            "grad_samples_per_s": round(nb_ / (grad_ms * 1e-3), 1),
            "lc": {k: round(v, 5) for k, v in rep["lc"].items()},
            "row": {k: round(v, 5) for k, v in rep["row"].items()},
            "mlp": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep["mlp"].items()},
            "mlp_vs_row_at_equal_fnr": (
                "the network is better than the row-aware count" if mlp_fpr < row_fpr else
                "the network is NOT better than the row-aware count" if mlp_fpr > row_fpr else
                "the network ties the row-aware count") + f" (FPR {mlp_fpr:.4f} vs {row_fpr:.4f})",
            "bins": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in b.items()}
                     for b in rep["bins"]]}


def host_info():
    """CPU model and core counts of the machine the oracle is timed on."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    return {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0)),
            "model": model, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(pairs, sample, theta):
    """The oracle's step (both cubes' update, both restores) on the first
    `sample` packets of the window (all by default): single-threaded (the
    reported value), and again with the update split over the host's cores
    (OpenMP, atomic ORs); the exact per-host counts (sort-unique) are timed
    beside it both ways."""
    import oracle as O
    p = O.default_params()
    s = pairs[:sample] if sample else pairs
    t0 = time.perf_counter()
    a = O.cube_of(p, s, O.SIDE_SRC)
    b = O.cube_of(p, s, O.SIDE_DST)
    t1 = time.perf_counter()
    O.restore(p, a, theta)
    O.restore(p, b, theta)
    dt = time.perf_counter() - t0
    restore_s = time.perf_counter() - t1
    t0 = time.perf_counter()
    O.exact_counts(s, O.SIDE_SRC)
    exact_1 = time.perf_counter() - t0
    threads = O.omp_threads()
    a2, b2 = O.new_cube(p), O.new_cube(p)
    t0 = time.perf_counter()
    O.update_omp(p, a2, s, O.SIDE_SRC)
    O.update_omp(p, b2, s, O.SIDE_DST)
    upd_omp = time.perf_counter() - t0
    O.restore(p, a2, theta)
    O.restore(p, b2, theta)
    dt_omp = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.exact_counts_omp(s, O.SIDE_SRC)
    exact_omp = time.perf_counter() - t0
    return {"value": round(len(s) / dt / 1e9, 6), "unit": "Gpkt/s", "cores": 1, "kind": "oracle",
            "sample": (f"{len(s)} packets of the window: oracle update of both cubes "
                       f"plus both restores, {dt:.1f}s single-threaded"),
            "update_s": round(dt - restore_s, 3), "restore_s_both": round(restore_s, 3),
            "exact_counts_s_one_side": round(exact_1, 3),
            "host": host_info(),
            "openmp": {"value": round(len(s) / dt_omp / 1e9, 6), "unit": "Gpkt/s",
                       "cores": threads, "update_s": round(upd_omp, 3),
                       "restore_s_both": round(dt_omp - upd_omp, 3),
                       "exact_counts_s_one_side": round(exact_omp, 3),
                       "note": "update over all threads with atomic ORs; the restore is the "
                               "oracle's single-threaded one"}}


if __name__ == "__main__":
    main()
