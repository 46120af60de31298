"""Serving loop: continuous batching with admission by memory. Every router's
cube and the restored lists are identical whether its chunks run alone or in
the mix with other routers' chunks (bit-exact: the cube is a set union); with
a cube budget smaller than the routers, routers are retired into the global
cubes and re-admitted and the lists still equal the oracle's; neither budget is
ever exceeded, and latencies are recorded."""

import numpy as np
import pytest

import oracle as O
import tracegen
from conftest import default_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06207_amd import cbaa
    cbaa.lib()
    return cbaa


def _chunks(n_routers, per_router, lo, hi, seed):
    import torch
    rng = np.random.default_rng(seed)
    chunks = []
    for r in range(n_routers):
        t = tracegen.make_window(int(hi * per_router * 0.6), 20_000, 3, 2_000, 8_000,
                                 dup_frac=0.1, fan_in_frac=0.5, seed=seed * 100 + r)
        pos = 0
        while pos < t.n:
            size = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
            q = t.pairs[pos:pos + size]
            pos += size
            h = torch.from_numpy(np.ascontiguousarray(q).view(np.int32)).pin_memory()
            chunks.append((r, q, h))
    order = rng.permutation(len(chunks))
    return [chunks[i] for i in order]


def test_results_same_alone_and_in_mix(cb):
    import torch
    from paper_1901_06207_amd import serve
    p = default_params()
    chunks = _chunks(4, 6, 20_000, 300_000, seed=5)
    srv = serve.Server(p, 4, both_sides=True, staging_bytes=16 << 20, theta=1024.0)
    for r, _, h in chunks:
        srv.submit(r, h)
    res = srv.end_window(reset=False)
    assert srv.batches >= 2 and srv.alloc.used == 0
    # alone: each router's chunks one by one into fresh cubes, then merge/restore
    alone = []
    for r in range(4):
        a, b = cb.new_cube(p), cb.new_cube(p)
        for rr, q, _ in chunks:
            if rr == r:
                cb.cbaa_update2(p, a, b, cb.pairs_to_device(q))
        torch.cuda.synchronize()
        assert np.array_equal(cb.cube_to_numpy(a), cb.cube_to_numpy(srv.cubes[r][0])), r
        assert np.array_equal(cb.cube_to_numpy(b), cb.cube_to_numpy(srv.cubes[r][1])), r
        alone.append((a, b))
    gs, gd = cb.new_cube(p, init=False), cb.new_cube(p, init=False)
    cb.cbaa_merge_or(p, gs, [x[0] for x in alone])
    cb.cbaa_merge_or(p, gd, [x[1] for x in alone])
    hs, _ = cb.restore(p, gs, 1024.0)
    hd, _ = cb.restore(p, gd, 1024.0)
    assert np.array_equal(res["hosts"][0], hs)
    assert np.array_equal(res["hosts"][1], hd)
    # and the oracle agrees on the merged traffic
    allq = np.concatenate([q for _, q, _ in chunks])
    oh, _ = O.restore(p, O.cube_of(p, allq, 0), 1024.0)
    assert np.array_equal(hs["ip"], oh["ip"]) and hs.size > 0


def test_admission_by_memory_and_latency(cb):
    from paper_1901_06207_amd import serve
    p = default_params()
    budget = 6 << 20
    chunks = _chunks(3, 8, 64_000, 700_000, seed=9)
    events = [(0.0005 * i, r, len(q)) for i, (r, q, _) in enumerate(chunks)]
    srv = serve.Server(p, 3, both_sides=False, staging_bytes=budget)
    res = serve.run_window(srv, events, [h for _, _, h in chunks], time_scale=1.0)
    assert res["chunks"] == len(chunks)
    assert res["packets"] == sum(len(q) for _, q, _ in chunks)
    assert 0 < srv.alloc.peak <= budget
    assert res["p99_ms"] >= res["p50_ms"] > 0
    # next window starts from emptied cubes that carry a valid header
    for a, _ in srv.cubes.values():
        assert int(a[cb.HEADER_WORDS:].abs().sum()) == 0
        assert cb.cbaa_cube_check(p, a) == 0


def test_cube_budget_retires_routers_and_keeps_results(cb):
    """Six routers, cubes for two: routers are retired (OR-merged into the
    global cubes, freed) and re-admitted when they send again; two windows in a
    row give the oracle's lists of each window's traffic."""
    from paper_1901_06207_amd import serve
    p = default_params()
    per = 2 * cb.cbaa_cube_bytes(p)
    srv = serve.Server(p, 6, both_sides=True, staging_bytes=8 << 20, cube_budget_bytes=2 * per)
    for w in range(2):
        print(f"[case] serving window {w} with a two-router cube budget", flush=True)
        chunks = _chunks(6, 4, 20_000, 200_000, seed=41 + w)
        events = [(0.0002 * i, r, len(q)) for i, (r, q, _) in enumerate(chunks)]
        before = srv.retirements
        res = serve.run_window(srv, events, [h for _, _, h in chunks], time_scale=1.0)
        assert res["chunks"] == len(chunks)
        assert srv.retirements > before
        assert 0 < res["cube_peak_bytes"] <= 2 * per
        assert res["result_p99_ms"] >= res["result_p50_ms"] >= res["p50_ms"] > 0
        allq = np.concatenate([q for _, q, _ in chunks])
        for side in (0, 1):
            want, _ = O.restore(p, O.cube_of(p, allq, side), 1024.0)
            got = res["hosts"][side]
            assert np.array_equal(got["ip"], want["ip"]), (w, side)
            assert np.array_equal(got["zeros"], want["zeros"])
            assert got.size > 0
