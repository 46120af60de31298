"""Seeded synthetic packet windows for CBAA tests and benchmarks.

This module only produces inputs: (source, destination) IPv4 pairs and the
construction-time truth about them. It holds none of the detector's arithmetic
(no mangling, no hashing, no cube), so both the HIP path and the CPU oracle can
consume its output without sharing any of the method.

Recipe (stands in for the paper's backbone-trace windows of Sec. 5.1, which
are not available):

* Host addresses and peer addresses come from one seeded 32-bit bijection
  ``B``: host k is ``B(k)`` and flow j's peer is ``B(2^31 + j)``. The two
  ranges are disjoint, so hosts and peers never collide and every flow's peer
  is distinct; a host's planted or assigned peer count is its exact
  cardinality by construction.
* Background sources: ``n_sources`` hosts with a Zipf rank-size law,
  ``d_k = 1 + floor(A * k**-s)`` for ranks k = 1..S, ``A`` found by bisection so
  that the degrees spend the background flow budget; the remainder goes to
  rank 1. Ranks are assigned to hosts by a seeded permutation. Background
  hosts are sources (host = src).
* Planted super hosts: ``n_planted`` hosts with log-uniform peer counts in
  ``[planted_lo, planted_hi]``; the first ``round(n_planted * (1 -
  fan_in_frac))`` are fan-out (host = src), the rest fan-in (host = dst).
* Duplicates: ``round(dup_frac * N)`` extra packets copy uniformly chosen
  flows, so the window holds exactly N packets.
* The packet order is a seeded random permutation.

All randomness comes from numpy's counter-based Philox generator.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["Trace", "make_window", "window_small", "window_core_edge", "split_routers",
           "bijection32", "construction_truth"]

_U32 = np.uint64(0xFFFFFFFF)


def _odd_from(rng: np.random.Generator) -> np.uint64:
    return np.uint64(int(rng.integers(0, 1 << 31)) * 2 + 1)


def bijection32(x: np.ndarray, key: tuple[int, int, int]) -> np.ndarray:
    """A keyed bijection on 32-bit integers (add, xorshift, odd multiply)."""
    add, m1, m2 = (np.uint64(k) for k in key)
    v = (x.astype(np.uint64) + add) & _U32
    v ^= v >> np.uint64(16)
    v = (v * m1) & _U32
    v ^= v >> np.uint64(15)
    v = (v * m2) & _U32
    v ^= v >> np.uint64(16)
    return v.astype(np.uint32)


@dataclasses.dataclass
class Trace:
    """One window of packets plus what the generator knows about it."""

    pairs: np.ndarray            # uint32 [N, 2]: (source, destination)
    seed: int
    params: dict
    planted_ips: np.ndarray      # uint32 [P]
    planted_deg: np.ndarray      # int64 [P]: exact distinct peers
    planted_side: np.ndarray     # int8 [P]: 0 = fan-out (host is source), 1 = fan-in
    bg_ips: np.ndarray           # uint32 [S]
    bg_deg: np.ndarray           # int64 [S]
    key: tuple = (0, 1, 1)       # the bijection's key

    @property
    def n(self) -> int:
        return int(self.pairs.shape[0])


def _zipf_degrees(n_sources: int, budget: int, s: float) -> np.ndarray:
    """Rank-size Zipf degrees d_k = 1 + floor(A k^-s) summing to ``budget``."""
    if n_sources == 0:
        return np.zeros(0, dtype=np.int64)
    if budget < n_sources:
        raise ValueError("background flow budget smaller than the number of sources")
    k = np.arange(1, n_sources + 1, dtype=np.float64)
    w = k ** (-s)

    def total(a: float) -> int:
        return int(n_sources + np.floor(a * w).sum())

    lo, hi = 0.0, float(budget)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) <= budget:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-9 * max(1.0, hi):
            break
    d = 1 + np.floor(lo * w).astype(np.int64)
    d[0] += budget - int(d.sum())
    return d


def make_window(n_packets: int, n_sources: int, n_planted: int, planted_lo: int, planted_hi: int,
                dup_frac: float = 0.0, zipf_s: float = 1.1, fan_in_frac: float = 0.0,
                seed: int = 1) -> Trace:
    rng = np.random.Generator(np.random.Philox(seed))
    key = (int(rng.integers(0, 1 << 32)), int(_odd_from(rng)), int(_odd_from(rng)))

    n_dup = int(round(dup_frac * n_packets))
    n_flows = n_packets - n_dup

    # planted degrees, log-uniform
    if n_planted:
        u = rng.random(n_planted)
        pdeg = np.floor(np.exp(math.log(planted_lo) + u * (math.log(planted_hi) - math.log(planted_lo))))
        pdeg = np.clip(pdeg.astype(np.int64), planted_lo, planted_hi)
    else:
        pdeg = np.zeros(0, dtype=np.int64)
    n_fan_in = int(round(n_planted * fan_in_frac))
    pside = np.zeros(n_planted, dtype=np.int8)
    if n_fan_in:
        pside[n_planted - n_fan_in:] = 1
    bg_budget = n_flows - int(pdeg.sum())
    if bg_budget < n_sources:
        raise ValueError("planted hosts do not fit the packet budget")

    bdeg_ranked = _zipf_degrees(n_sources, bg_budget, zipf_s)
    perm = rng.permutation(n_sources)
    bdeg = np.empty_like(bdeg_ranked)
    bdeg[perm] = bdeg_ranked

    host_idx = np.arange(n_sources + n_planted, dtype=np.uint64)
    host_ips = bijection32(host_idx, key)
    bg_ips = host_ips[:n_sources]
    pl_ips = host_ips[n_sources:]

    deg = np.concatenate([bdeg, pdeg])
    flow_host = np.repeat(host_ips, deg)
    flow_peer = bijection32(np.uint64(1 << 31) + np.arange(n_flows, dtype=np.uint64), key)
    fan_in_flow = np.repeat(np.concatenate([np.zeros(n_sources, np.int8), pside]), deg).astype(bool)
    src = np.where(fan_in_flow, flow_peer, flow_host)
    dst = np.where(fan_in_flow, flow_host, flow_peer)
    del flow_host, flow_peer, fan_in_flow

    flows = np.empty((n_flows, 2), dtype=np.uint32)
    flows[:, 0] = src
    flows[:, 1] = dst
    del src, dst
    if n_dup:
        dup = flows[rng.integers(0, n_flows, n_dup)]
        flows = np.concatenate([flows, dup])
        del dup
    order = rng.permutation(n_packets)
    pairs = flows[order]
    del flows, order

    params = dict(n_packets=n_packets, n_sources=n_sources, n_planted=n_planted,
                  planted_lo=planted_lo, planted_hi=planted_hi, dup_frac=dup_frac,
                  zipf_s=zipf_s, fan_in_frac=fan_in_frac)
    return Trace(pairs=np.ascontiguousarray(pairs), seed=seed, params=params,
                 planted_ips=pl_ips, planted_deg=pdeg, planted_side=pside,
                 bg_ips=bg_ips, bg_deg=bdeg, key=key)


def construction_truth(t: Trace, side: int) -> tuple[np.ndarray, np.ndarray]:
    """Every host of one side with its exact number of distinct peers, as the
    generator built it (side 0: hosts are sources, 1: destinations).

    Sources: background hosts, fan-out planted hosts, and the peers of fan-in
    planted hosts (one peer each). Destinations: fan-in planted hosts and the
    peers of every other flow (one peer each)."""
    n_bg = t.bg_ips.size
    deg = np.concatenate([t.bg_deg, t.planted_deg])
    fan_in = np.concatenate([np.zeros(n_bg, bool), t.planted_side.astype(bool)])

    def peers_of(mask):
        # flow k belongs to the host whose [start, end) range holds it; the
        # flows of the selected hosts, in host order
        idx = np.nonzero(np.repeat(mask, deg))[0].astype(np.uint64)
        return bijection32(np.uint64(1 << 31) + idx, t.key)

    if side == 0:
        out_pl = t.planted_side == 0
        peers = peers_of(fan_in)
        hosts = np.concatenate([t.bg_ips, t.planted_ips[out_pl], peers])
        counts = np.concatenate([t.bg_deg, t.planted_deg[out_pl], np.ones(peers.size, np.int64)])
    else:
        in_pl = t.planted_side == 1
        peers = peers_of(~fan_in)
        hosts = np.concatenate([t.planted_ips[in_pl], peers])
        counts = np.concatenate([t.planted_deg[in_pl], np.ones(peers.size, np.int64)])
    return hosts.astype(np.uint32), counts


def window_small(seed: int = 1) -> Trace:
    """One window of 1,000,000 packets: 100k Zipf(1.1) sources, 20 planted
    fan-out hosts of 2k-20k peers, no duplicates."""
    return make_window(1_000_000, 100_000, 20, 2_000, 20_000, dup_frac=0.0, zipf_s=1.1,
                       fan_in_frac=0.0, seed=seed)


def window_core_edge(seed: int = 11, scale: float = 1.0) -> Trace:
    """Core-edge window: 64 x 2^20 packets, 8M Zipf(1.1) sources, 1000 planted
    hosts of 1k-200k peers (half fan-out, half fan-in), 10% duplicates.

    ``scale`` < 1 shrinks packets, sources and planted hosts together (the
    planted range's top shrinks with it, never below 4k) for quicker cases of
    the same shape."""
    n_packets = int(round((64 << 20) * scale))
    n_sources = max(1, int(round(8_000_000 * scale)))
    n_planted = max(2, int(round(1000 * scale)))
    hi = 200_000 if scale >= 1.0 else max(4_000, int(200_000 * math.sqrt(scale)))
    return make_window(n_packets, n_sources, n_planted, 1_000, hi, dup_frac=0.10, zipf_s=1.1,
                       fan_in_frac=0.5, seed=seed)


def split_routers(pairs: np.ndarray, k: int, seed: int = 0) -> list[np.ndarray]:
    """Assigns every packet of a window to one of k edge routers at random."""
    rng = np.random.Generator(np.random.Philox(seed + 7919))
    who = rng.integers(0, k, pairs.shape[0])
    return [np.ascontiguousarray(pairs[who == i]) for i in range(k)]
