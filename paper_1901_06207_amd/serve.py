"""Serving loop for edge-router packet streams (continuous batching).

The global server of the paper's distributed model (Sec. 2, Sec. 3.3) keeps
the local cubes of the edge routers that are sending in HBM and serves their
packet chunks as they arrive:

* Admission by memory, twice. A chunk is admitted when a staging region of
  its size is free in a fixed device budget; its router's cubes must be
  resident, inside a second budget for cubes. A router that is not resident
  gets cubes when the cube budget has room; otherwise the least recently used
  resident router with no work in flight is retired: its cubes are OR-merged
  into the window's global cubes (Sec. 3.3: the merge is a bitwise OR, so
  merging a router early, or twice, changes nothing) and freed. A chunk whose
  router cannot be made resident yet waits.
* Continuous batching. An admitted chunk's copy to the device runs on a copy
  stream; every chunk whose copy has finished joins the next batched update
  (``cbaa_update_batch``) on one of two compute streams, so copies, updates
  and new arrivals overlap on the device.
* Window end. The global cubes, holding the retired routers, and the resident
  routers' cubes are OR-merged and restored in one call per side; the
  resident cubes start the next window empty.

Latencies: a chunk's update latency runs from its arrival to the completion of
the batch that took it; its result latency from its arrival to the moment the
restored lists of its window are on the host.

All arithmetic is in libcbaa's kernels; this module schedules, allocates
staging and cube memory, and records times.
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
    t_result: float = 0.0


class Server:
    def __init__(self, cfg, n_routers: int, both_sides: bool = True,
                 staging_bytes: int = 512 << 20, cube_budget_bytes: Optional[int] = None,
                 max_batch: int = cbaa.MAX_BATCH, capacity: int = 1 << 14,
                 theta: float = 1024.0, tuning=None, device="cuda"):
        self.cfg = cfg
        self.dev = torch.device(device)
        self.nr = n_routers
        self.both = both_sides
        self.theta = theta
        self.max_batch = max_batch
        self.tuning = tuning
        self.per_router = cbaa.cbaa_cube_bytes(cfg) * (2 if both_sides else 1)
        # by default every router fits: the budget only bites when it is given
        self.cube_budget = (cube_budget_bytes if cube_budget_bytes is not None
                            else n_routers * self.per_router)
        if self.cube_budget < self.per_router:
            raise ValueError("the cube budget holds no router's cubes")
        self.cubes = {}                          # resident router -> (src cube, dst cube or None)
        self.cube_used = 0
        self.cube_peak = 0
        self.inflight_of = collections.Counter()  # router -> chunks admitted, not yet updated
        self.last_use = {}                       # router -> admission tick (LRU)
        self.tick = 0
        self.retirements = 0
        self.retired_this_window = False
        self.graveyard = []                      # (event, tensors) freed once the event completes
        self.g_src = cbaa.new_cube(cfg, self.dev)
        self.g_dst = cbaa.new_cube(cfg, self.dev) if both_sides else None
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
        self.last_event = {}                    # router -> event of its last batch
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
        a = cbaa.new_cube(self.cfg, self.dev, init=False)
        b = cbaa.new_cube(self.cfg, self.dev, init=False) if self.both else None
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
        del a, b
        return best

    # ---- request side ------------------------------------------------------
    def submit(self, router: int, host_pairs: torch.Tensor, t_arrival: Optional[float] = None) -> int:
        """Queues a chunk of (source, destination) pairs held in pinned host
        memory (int32 [n, 2] storage of the uint32 addresses) for router."""
        if not 0 <= router < self.nr:
            raise ValueError(f"router {router} outside [0, {self.nr})")
        cid = self.submitted
        self.submitted += 1
        self.waiting.append(Chunk(cid, router, host_pairs, t_arrival or time.perf_counter()))
        return cid

    # ---- cube residency ------------------------------------------------------
    def _bury(self, stream, tensors) -> None:
        ev = torch.cuda.Event()
        ev.record(stream)
        self.graveyard.append((ev, tensors))

    def _reap(self, block: bool = False) -> None:
        keep = []
        for ev, tensors in self.graveyard:
            if block:
                ev.synchronize()
            if ev.query():
                self.cube_used -= self.per_router
            else:
                keep.append((ev, tensors))
        self.graveyard = keep

    def _retire(self, r: int) -> None:
        """OR-merges router r's cubes into the global cubes and frees them."""
        a, b = self.cubes.pop(r)
        st = self.compute[0]
        ev = self.last_event.pop(r, None)
        if ev is not None:
            st.wait_event(ev)
        # merges run on one stream, so they are ordered among themselves; only
        # the window end reads the global cubes, after a full synchronisation
        cbaa.cbaa_merge_or(self.cfg, self.g_src, [self.g_src, a], st)
        if b is not None:
            cbaa.cbaa_merge_or(self.cfg, self.g_dst, [self.g_dst, b], st)
        self._bury(st, (a, b))
        self.retirements += 1
        self.retired_this_window = True

    def _make_resident(self, r: int) -> bool:
        if r in self.cubes:
            return True
        self._reap()
        while self.cube_used + self.per_router > self.cube_budget:
            idle = [x for x in self.cubes if self.inflight_of[x] == 0]
            if not idle:
                if self.graveyard:          # cubes being freed: wait for them
                    self._reap(block=True)
                    continue
                return False
            self._retire(min(idle, key=lambda x: self.last_use.get(x, -1)))
            self._reap()
            if self.cube_used + self.per_router > self.cube_budget and self.graveyard:
                self._reap(block=True)
        st = self.compute[self.next_compute]
        a = cbaa.new_cube(self.cfg, self.dev, stream=st)
        b = cbaa.new_cube(self.cfg, self.dev, stream=st) if self.both else None
        self.compute[self.next_compute ^ 1].wait_stream(st)
        self.cubes[r] = (a, b)
        self.cube_used += self.per_router
        self.cube_peak = max(self.cube_peak, self.cube_used)
        return True

    # ---- scheduling ----------------------------------------------------------
    def _admit(self) -> None:
        while self.waiting:
            c = self.waiting[0]
            nbytes = int(c.host.shape[0]) * 8
            if nbytes > self.alloc.size:
                raise ValueError("chunk larger than the staging budget")
            if not self._make_resident(c.router):
                return
            off = self.alloc.alloc(nbytes)
            if off is None:
                return
            self.waiting.popleft()
            c.off, c.nbytes = off, nbytes
            self.tick += 1
            self.last_use[c.router] = self.tick
            self.inflight_of[c.router] += 1
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
        for c in ready:
            self.last_event[c.router] = ev
        self.inflight.append((ev, ready, i))
        self.batches += 1

    def _complete(self, block: bool = False) -> None:
        keep = []
        for ev, chunks, i in self.inflight:
            if block:
                ev.synchronize()
            if ev.query():
                now = time.perf_counter()
                for c in chunks:
                    c.t_done = now
                    self.alloc.release(c.off, c.nbytes)
                    self.inflight_of[c.router] -= 1
                    self.packets += int(c.host.shape[0])
                    self.done.append(c)
            else:
                keep.append((ev, chunks, i))
        self.inflight = keep

    def poll(self) -> None:
        self._complete()
        self._reap()
        self._admit()
        self._launch()

    def drain(self) -> None:
        while self.waiting or self.copying or self.inflight:
            self.poll()
            if self.inflight and not self.copying:
                self._complete(block=True)

    # ---- window end (global server) ----------------------------------------------
    def end_window(self, reset: bool = True) -> dict:
        """Drains, OR-merges the retired routers (held in the global cubes) and
        the resident routers' cubes, restores both sides and (unless reset is
        False) starts the next window from empty cubes. Returns host lists and
        timings; every chunk of the window gets its result time."""
        self.drain()
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        s = torch.cuda.current_stream(self.dev)
        glob = [self.g_src] + ([self.g_dst] if self.both else [])
        routers = sorted(self.cubes)
        for i, g in enumerate(glob):   # per side: OR-merge and restore in one call
            srcs = ([g] if self.retired_this_window else []) + [self.cubes[r][i] for r in routers]
            if not srcs:
                srcs = [g]
            cbaa.cbaa_merge_restore(self.cfg, g, srcs, self.theta, cbaa.THR_THM2, self.rs[i],
                                    self.outs[i], self.capacity, self.stats[i], s)
        if reset:
            for r in routers:
                for c in self.cubes[r]:
                    if c is not None:
                        cbaa.cbaa_cube_init(self.cfg, c, s)
            for g in glob:
                cbaa.cbaa_cube_init(self.cfg, g, s)
            self.retired_this_window = False
        torch.cuda.synchronize(self.dev)
        lists = []
        for i in range(len(glob)):
            n = int(self.stats[i][0])
            if n > self.capacity:
                raise RuntimeError(f"restore capacity {self.capacity} below {n}")
            lists.append(cbaa.host_list(self.outs[i], n))
        t1 = time.perf_counter()
        for c in self.done:
            if not c.t_result:
                c.t_result = t1
        self._reap(block=True)
        return {"hosts": lists, "restore_ms": (t1 - t0) * 1e3}

    def latencies_ms(self) -> np.ndarray:
        """Update latency of every finished chunk: arrival to its batch done."""
        return np.array([(c.t_done - c.t_arrival) * 1e3 for c in self.done])

    def result_latencies_ms(self) -> np.ndarray:
        """Result latency: arrival to its window's restored lists on the host."""
        return np.array([(c.t_result - c.t_arrival) * 1e3 for c in self.done if c.t_result])


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
    rlat = server.result_latencies_ms()
    pk = sum(int(c.host.shape[0]) for c in server.done)
    res.update({"chunks": len(server.done), "packets": pk, "wall_s": t_last - t0,
                "gpkt_s": pk / max(t_last - t0, 1e-9) / 1e9,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else 0.0,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else 0.0,
                "result_p50_ms": float(np.percentile(rlat, 50)) if rlat.size else 0.0,
                "result_p99_ms": float(np.percentile(rlat, 99)) if rlat.size else 0.0,
                "staging_peak_bytes": server.alloc.peak, "batches": server.batches,
                "cube_peak_bytes": server.cube_peak, "retirements": server.retirements})
    return res
