"""Serving loop for edge-router packet streams (continuous batching).

Each router's cubes stay resident in HBM for the whole window. Packet chunks
arrive (from pinned host memory) at any time; a chunk is admitted when a
staging region of its size is free in a fixed device budget (admission by
memory), its copy to the device runs on a copy stream, and every chunk whose
copy has finished joins the next batched update (``cbaa_update_batch``) on
one of two compute streams -- so copies, and successive batches, overlap on
the device while new chunks keep arriving. A chunk's latency runs from its
arrival to the completion of the batch that took it. At window end the
routers' cubes are OR-merged into the global cubes and both are restored
(the global server of the paper's distributed model), then the routers'
cubes are zeroed for the next window.

All arithmetic is in libcbaa's kernels; this module schedules, allocates
staging space and records times.
"""

from __future__ import annotations

import collections
import dataclasses
import time
from typing import Optional

import numpy as np
import torch

from . import cbaa

ALIGN = 256


class StagingAllocator:
    """First-fit allocator over [0, size) bytes with coalescing frees."""

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]   # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, n: int) -> Optional[int]:
        n = (n + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, n: int) -> None:
        n = (n + ALIGN - 1) // ALIGN * ALIGN
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


@dataclasses.dataclass
class Chunk:
    cid: int
    router: int
    host: torch.Tensor            # pinned uint32 pairs [n, 2] (int32 storage)
    t_arrival: float
    off: int = -1
    nbytes: int = 0
    copied: Optional[torch.cuda.Event] = None
    t_done: float = 0.0


class Server:
    def __init__(self, cfg, n_routers: int, both_sides: bool = True,
                 staging_bytes: int = 512 << 20, max_batch: int = cbaa.MAX_BATCH,
                 capacity: int = 1 << 14, theta: float = 1024.0, tuning=None, device="cuda"):
        self.cfg = cfg
        self.dev = torch.device(device)
        self.nr = n_routers
        self.both = both_sides
        self.theta = theta
        self.max_batch = max_batch
        self.tuning = tuning
        self.cubes = [(cbaa.new_cube(cfg, self.dev), cbaa.new_cube(cfg, self.dev) if both_sides else None)
                      for _ in range(n_routers)]
        self.g_src = cbaa.new_cube(cfg, self.dev, init=False)
        self.g_dst = cbaa.new_cube(cfg, self.dev, init=False) if both_sides else None
        self.staging = torch.empty(staging_bytes, dtype=torch.uint8, device=self.dev)
        self.alloc = StagingAllocator(staging_bytes)
        # scratch for the largest batch the staging can hold, any split over streams
        worst = self._worst_scratch(staging_bytes // 8)
        self.compute = [torch.cuda.Stream(device=self.dev) for _ in range(2)]
        self.scratch = [cbaa.scratch_tensor(worst, self.dev) for _ in range(2)]
        self.copy = torch.cuda.Stream(device=self.dev)
        self.capacity = capacity
        self.rs = [cbaa.scratch_tensor(cbaa.cbaa_restore_scratch_bytes(cfg, capacity), self.dev)
                   for _ in range(2)]
        self.outs = [torch.empty(capacity * cbaa.HOST_BYTES, dtype=torch.uint8, device=self.dev)
                     for _ in range(2)]
        self.stats = [cbaa.stats_tensor(self.dev) for _ in range(2)]
        self.waiting = collections.deque()      # arrived, not admitted
        self.copying = []                       # admitted, copy in flight
        self.inflight = []                      # (event, chunks, stream index)
        self.done = []
        self.next_compute = 0
        self.batches = 0
        self.packets = 0
        self.submitted = 0

    def _worst_scratch(self, max_pairs: int) -> int:
        """Scratch for any batch the staging budget can hold: the library's own
        size query on the splits with the most chunks (and the one-stream case)."""
        import ctypes as C
        k = self.max_batch
        dummy = torch.empty((1, 2), dtype=torch.int32, device=self.dev)
        a, b = self.cubes[0]
        splits = [[max_pairs]]
        per = 65537   # one pair over a chunk: two chunks per stream
        if per * (k - 1) < max_pairs:
            splits.append([per] * (k - 1) + [max_pairs - per * (k - 1)])
        splits.append([max(1, max_pairs // k)] * k)
        best = 0
        for sizes in splits:
            table = cbaa._stream_table(self.cfg, [(dummy, a, b, cbaa.SIDE_SRC)] * len(sizes))
            for i, n in enumerate(sizes):
                table[i].n_pairs = n
            need = cbaa.lib().cbaa_update_batch_scratch_bytes(
                C.byref(cbaa._cfg(self.cfg)), table, len(sizes),
                C.byref(cbaa._tuning(self.tuning)) if self.tuning else None)
            best = max(best, int(need))
        return best

    # ---- request side ------------------------------------------------------
    def submit(self, router: int, host_pairs: torch.Tensor, t_arrival: Optional[float] = None) -> int:
        """Queues a chunk of (source, destination) pairs held in pinned host
        memory (int32 [n, 2] storage of the uint32 addresses) for router."""
        cid = self.submitted
        self.submitted += 1
        self.waiting.append(Chunk(cid, router, host_pairs, t_arrival or time.perf_counter()))
        return cid

    # ---- scheduling ----------------------------------------------------------
    def _admit(self) -> None:
        while self.waiting:
            c = self.waiting[0]
            nbytes = int(c.host.shape[0]) * 8
            if nbytes > self.alloc.size:
                raise ValueError("chunk larger than the staging budget")
            off = self.alloc.alloc(nbytes)
            if off is None:
                return
            self.waiting.popleft()
            c.off, c.nbytes = off, nbytes
            dst = self.staging[off:off + nbytes].view(torch.int32).view(-1, 2)
            with torch.cuda.stream(self.copy):
                dst.copy_(c.host, non_blocking=True)
                c.copied = torch.cuda.Event()
                c.copied.record(self.copy)
            self.copying.append(c)

    def _launch(self) -> None:
        ready = [c for c in self.copying if c.copied.query()]
        if not ready:
            return
        ready = ready[: self.max_batch]
        for c in ready:
            self.copying.remove(c)
        i = self.next_compute
        self.next_compute ^= 1
        st = self.compute[i]
        table = []
        for c in ready:
            st.wait_event(c.copied)
            pairs = self.staging[c.off:c.off + c.nbytes].view(torch.int32).view(-1, 2)
            a, b = self.cubes[c.router]
            table.append((pairs, a, b, cbaa.SIDE_SRC))
        # each compute stream owns a scratch; work on one stream runs in order
        cbaa.cbaa_update_batch(self.cfg, table, self.scratch[i], self.tuning, st)
        ev = torch.cuda.Event()
        ev.record(st)
        self.inflight.append((ev, ready, i))
        self.batches += 1

    def _retire(self, block: bool = False) -> None:
        keep = []
        for ev, chunks, i in self.inflight:
            if block:
                ev.synchronize()
            if ev.query():
                now = time.perf_counter()
                for c in chunks:
                    c.t_done = now
                    self.alloc.release(c.off, c.nbytes)
                    self.packets += int(c.host.shape[0])
                    self.done.append(c)
            else:
                keep.append((ev, chunks, i))
        self.inflight = keep

    def poll(self) -> None:
        self._retire()
        self._admit()
        self._launch()

    def drain(self) -> None:
        while self.waiting or self.copying or self.inflight:
            self.poll()
            if self.inflight and not self.copying and not self.waiting:
                self._retire(block=True)

    # ---- window end (global server) ----------------------------------------------
    def end_window(self, reset: bool = True) -> dict:
        """Drains, OR-merges the routers' cubes, restores the global cubes and
        (unless reset is False) zeroes the routers' cubes. Returns host lists
        and timings."""
        self.drain()
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        s = torch.cuda.current_stream(self.dev)
        cubes = [self.g_src] + ([self.g_dst] if self.both else [])
        for i, g in enumerate(cubes):   # per side: OR-merge and restore in one call
            cbaa.cbaa_merge_restore(self.cfg, g, [c[i] for c in self.cubes], self.theta,
                                    cbaa.THR_THM2, self.rs[i], self.outs[i], self.capacity,
                                    self.stats[i], s)
        for a, b in self.cubes if reset else []:
            cbaa.cbaa_cube_init(self.cfg, a, s)
            if b is not None:
                cbaa.cbaa_cube_init(self.cfg, b, s)
        torch.cuda.synchronize(self.dev)
        t1 = time.perf_counter()
        lists = []
        for i in range(len(cubes)):
            n = int(self.stats[i][0])
            if n > self.capacity:
                raise RuntimeError(f"restore capacity {self.capacity} below {n}")
            lists.append(cbaa.host_list(self.outs[i], n))
        return {"hosts": lists, "restore_ms": (t1 - t0) * 1e3}

    def latencies_ms(self) -> np.ndarray:
        return np.array([(c.t_done - c.t_arrival) * 1e3 for c in self.done])


def poisson_schedule(n_routers: int, window_s: float, chunk_lo: int, chunk_hi: int,
                     rate_per_router: float, seed: int):
    """Arrival times (seconds into the window), routers and chunk sizes:
    Poisson arrivals per router, log-uniform chunk sizes."""
    rng = np.random.default_rng(seed)
    events = []
    for r in range(n_routers):
        t = rng.exponential(1.0 / rate_per_router)
        while t < window_s:
            size = int(np.exp(rng.uniform(np.log(chunk_lo), np.log(chunk_hi))))
            events.append((t, r, size))
            t += rng.exponential(1.0 / rate_per_router)
    events.sort()
    return events


def run_window(server: Server, events, chunks_host, time_scale: float) -> dict:
    """Replays one window: event i (at simulated time t_i) is released at
    wall time t_i * time_scale after the start; the loop keeps admitting,
    launching and retiring until every chunk is in the cubes, then ends the
    window."""
    t0 = time.perf_counter()
    i = 0
    n = len(events)
    server.done.clear()
    while i < n or server.waiting or server.copying or server.inflight:
        now = time.perf_counter() - t0
        while i < n and events[i][0] * time_scale <= now:
            t_rel = t0 + events[i][0] * time_scale
            server.submit(events[i][1], chunks_host[i], t_rel)
            i += 1
        server.poll()
    t_last = time.perf_counter()
    res = server.end_window()
    lat = server.latencies_ms()
    pk = sum(int(c.host.shape[0]) for c in server.done)
    res.update({"chunks": len(server.done), "packets": pk, "wall_s": t_last - t0,
                "gpkt_s": pk / max(t_last - t0, 1e-9) / 1e9,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else 0.0,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else 0.0,
                "staging_peak_bytes": server.alloc.peak, "batches": server.batches})
    return res
