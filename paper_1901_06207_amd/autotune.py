"""Autotuner for the partitioned update's tile/partition shapes.

Times ``cbaa_update_batch`` on the caller's own streams with HIP events for a
few shapes, one parameter at a time (coordinate descent over the sample's
piece size, apply segment size, apply grid, five values each, repeated while a
sweep still moves the best shape, at most ``rounds`` sweeps), and returns the
fastest. Results are cached per (configuration, number of streams, total
packets rounded to a power of two).
"""

from __future__ import annotations

import math

import torch

from . import cbaa

CHUNKS = (4096, 8192, 16384, 32768, 65536)
SEGS = (16384, 32768, 65536, 131072, 262144)
APPLY_BLOCKS = (256, 512, 768, 1024, 2048)

_cache: dict = {}


def _key(cfg, streams):
    c = cfg if isinstance(cfg, cbaa.Config) else cbaa.Config.from_dict(cfg)
    total = sum(int(s[0].shape[0]) for s in streams)
    fresh = any(len(s) > 4 and s[4] for s in streams)
    return (c, len(streams), streams[0][2] is not None, fresh,
            1 << max(0, math.ceil(math.log2(max(total, 1)))))


def _time(cfg, streams, tuning, scratch, repeats, stream):
    ms = []
    for _ in range(repeats + 1):
        for s in streams:
            cbaa.cbaa_cube_init(cfg, s[1], stream)
            if s[2] is not None:
                cbaa.cbaa_cube_init(cfg, s[2], stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cbaa.cbaa_update_batch(cfg, streams, scratch, tuning, stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = sorted(ms[1:])
    return ms[len(ms) // 2]


def tune_update(cfg, streams, repeats: int = 3, use_cache: bool = True, stream=None,
                rounds: int = 2) -> dict:
    """Returns {"best": tuning dict, "best_ms": t, "default_ms": t0,
    "candidates": [{"tuning": ..., "ms": ...}, ...]}. The cubes of the streams
    are overwritten."""
    key = _key(cfg, streams)
    if use_cache and key in _cache:
        return _cache[key]
    stream = stream or torch.cuda.current_stream()
    need = max(cbaa.cbaa_update_batch_scratch_bytes(cfg, streams,
                                                    dict(chunk_pairs=c, seg_records=g))
               for c in CHUNKS for g in SEGS)
    scratch = cbaa.scratch_tensor(need, streams[0][1].device)
    best = dict(chunk_pairs=16384, seg_records=65536, apply_blocks=512)
    seen = {}

    def measure(t):
        k = (t["chunk_pairs"], t["seg_records"], t["apply_blocks"])
        if k not in seen:
            seen[k] = _time(cfg, streams, t, scratch, repeats, stream)
        return seen[k]

    default_ms = measure(best)
    for _ in range(max(1, rounds)):
        start = dict(best)
        for name, values in (("chunk_pairs", CHUNKS), ("seg_records", SEGS),
                             ("apply_blocks", APPLY_BLOCKS)):
            scores = {v: measure(dict(best, **{name: v})) for v in values}
            # a tie keeps the current value: the shape moves only for a gain
            best = dict(best, **{name: min(scores, key=lambda v: (scores[v], v != best[name]))})
        if best == start:
            break
    res = {"best": best, "best_ms": measure(best), "default_ms": default_ms,
           "candidates": [{"tuning": dict(chunk_pairs=k[0], seg_records=k[1], apply_blocks=k[2]),
                           "ms": v} for k, v in seen.items()]}
    _cache[key] = res
    return res
