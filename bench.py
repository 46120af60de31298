"""Benchmark of the CBAA hot path on one MI355X.

One step = one window of the core-edge workload through every stage:
  per edge router: zero its two local cubes, take its packets into both
  (source-keyed and destination-keyed, one read of each pair);
  global server: OR-merge the routers' cubes; restore the super hosts of
  both global cubes; copy the two sorted lists and counters to the host.

Workload: 64 x 2^20 synthetic packets (8M Zipf(1.1) sources, 1000 planted
hosts of 1k-200k peers, half fan-out and half fan-in, 10% duplicates),
split at random over the edge routers; paper dimensions r=4, |RA|=3, |VA|=1,
g=c=2^12 (128 MiB per cube); theta = 1024. Inputs are resident in HBM
before timing starts.

Prints one JSON line (rank 0). Only one GPU is used: --gpus above 1 exits.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
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
    ap.add_argument("--update", choices=["auto", "direct", "partitioned"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="packets of the window the CPU oracle step is timed on (0 = all)")
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
    from paper_1901_06207_amd import cbaa

    cbaa.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = cbaa.cbaa_config_default()
    cube_bytes = cbaa.cbaa_cube_bytes(cfg)

    t0 = time.time()
    trace = tracegen.window_core_edge(args.seed, scale=args.scale)
    parts = tracegen.split_routers(trace.pairs, args.routers, seed=args.seed)
    log(f"generated {trace.n} packets in {time.time() - t0:.1f}s; routers "
        f"{[len(q) for q in parts]}")
    d_parts = [cbaa.pairs_to_device(q, dev) for q in parts]

    use_part = args.update != "direct"
    scratch_u = None
    if use_part:
        need = max(cbaa.cbaa_update_scratch_bytes(cfg, len(q), 2) for q in parts)
        if need > 0:
            scratch_u = cbaa.scratch_tensor(need, dev)
        elif args.update == "partitioned":
            raise SystemExit("partitioned update not available for this configuration")
    update_path = "partitioned" if scratch_u is not None else "direct"

    local = [(cbaa.new_cube(cfg, dev, init=False), cbaa.new_cube(cfg, dev, init=False))
             for _ in parts]
    g_src = cbaa.new_cube(cfg, dev, init=False)
    g_dst = cbaa.new_cube(cfg, dev, init=False)
    capacity = 1 << 14
    rs_bytes = cbaa.cbaa_restore_scratch_bytes(cfg, capacity)
    scratch_r = [cbaa.scratch_tensor(rs_bytes, dev) for _ in range(2)]
    outs = [torch.empty(capacity * cbaa.HOST_BYTES, dtype=torch.uint8, device=dev) for _ in range(2)]
    stats = [cbaa.stats_tensor(dev) for _ in range(2)]
    h_outs = [torch.empty(capacity * cbaa.HOST_BYTES, dtype=torch.uint8, pin_memory=True)
              for _ in range(2)]
    h_stats = [torch.empty(4, dtype=torch.int64, pin_memory=True) for _ in range(2)]
    stream = torch.cuda.current_stream(dev)

    ev = {}

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev.setdefault(name, []).append(e)

    def step(timed_phases=False):
        if timed_phases:
            mark("update_begin")
        for (a, b), q in zip(local, d_parts):
            cbaa.cbaa_cube_init(cfg, a, stream)
            cbaa.cbaa_cube_init(cfg, b, stream)
            if timed_phases:
                mark("u2_begin")
            cbaa.cbaa_update2(cfg, a, b, q, scratch_u, stream)
            if timed_phases:
                mark("u2_end")
        if timed_phases:
            mark("merge_begin")
        cbaa.cbaa_merge_or(cfg, g_src, [x[0] for x in local], stream)
        cbaa.cbaa_merge_or(cfg, g_dst, [x[1] for x in local], stream)
        if timed_phases:
            mark("restore_begin")
        for i, cube in enumerate((g_src, g_dst)):
            cbaa.cbaa_restore(cfg, cube, args.theta, cbaa.THR_THM2, scratch_r[i], outs[i], capacity,
                              stats[i], stream)
            h_stats[i].copy_(stats[i], non_blocking=True)
            h_outs[i].copy_(outs[i], non_blocking=True)
        if timed_phases:
            mark("restore_end")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize(dev)
    n_found = [int(h_stats[i][0]) for i in range(2)]
    if max(n_found) > capacity:
        raise SystemExit(f"restore capacity {capacity} too small for {n_found}")
    log(f"super hosts found: source-keyed {n_found[0]}, destination-keyed {n_found[1]}")

    # timed region: exactly K steps
    torch.cuda.synchronize(dev)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = trace.n / (elapsed / args.steps) / 1e9

    # per-phase breakdown with events on the launch stream (separate pass)
    ev.clear()
    phase_steps = max(3, min(args.steps, 10))
    for _ in range(phase_steps):
        step(timed_phases=True)
    torch.cuda.synchronize(dev)

    def span(a, b):
        return [x.elapsed_time(y) for x, y in zip(ev[a], ev[b])]

    upd_ms = np.array(span("u2_begin", "u2_end"))          # one per router per step
    merge_ms = np.mean(span("merge_begin", "restore_begin"))
    restore_ms = np.array(span("restore_begin", "restore_end")) / 2.0   # per window (cube)
    window_update_ms = np.mean(span("update_begin", "merge_begin"))
    pkts_per_router = np.mean([len(q) for q in parts])
    upd_gpkts = pkts_per_router / (upd_ms.mean() * 1e-3) / 1e9

    # roofline of the dominant kernel set: the update call (algorithmic bytes =
    # 8 B per packet read + both cubes written once)
    upd_alg_bytes = 8.0 * pkts_per_router + 2.0 * cube_bytes
    achieved = upd_alg_bytes / (upd_ms.mean() * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"cbaa_update2 ({update_path})",
                "per_launch": {"packets": int(pkts_per_router), "alg_bytes": int(upd_alg_bytes),
                               "avg_ms": round(float(upd_ms.mean()), 4)}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(trace.pairs, args.cpu_sample, args.theta)

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
            "packets": trace.n, "routers": args.routers, "update_path": update_path,
            "seed": args.seed,
        },
        "phases": {
            "update_gpkt_s": round(float(upd_gpkts), 3),
            "update_ms_per_window": round(float(window_update_ms), 4),
            "merge_ms": round(float(merge_ms), 4),
            "restore_ms_per_window": round(float(restore_ms.mean()), 4),
            "restore_ms_p99": round(float(np.percentile(restore_ms, 99)), 4),
            "super_hosts": {"source_keyed": n_found[0], "destination_keyed": n_found[1]},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(pairs, sample, theta):
    """The oracle's step (both cubes' update, both restores) on the first
    `sample` packets of the window, single-threaded on the host."""
    import oracle as O
    p = O.default_params()
    s = pairs[:sample] if sample else pairs
    t0 = time.perf_counter()
    a = O.cube_of(p, s, O.SIDE_SRC)
    b = O.cube_of(p, s, O.SIDE_DST)
    O.restore(p, a, theta)
    O.restore(p, b, theta)
    dt = time.perf_counter() - t0
    return {"value": round(len(s) / dt / 1e9, 6), "unit": "Gpkt/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {len(s)} packets of the window: oracle update of both cubes plus "
                       f"both restores, {dt:.1f}s single-threaded")}


if __name__ == "__main__":
    main()
