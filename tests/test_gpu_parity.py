"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: cube bytes, per-column zeros, array fills, restored IP / Z / sketch /
flag lists bit-exact; estimates within |d| <= 1e-9 * max(1, est) (device
log vs libm log, everything else is exact integer or the same IEEE double
operations in the same order)."""

import numpy as np
import pytest

import oracle as O
import tracegen
from conftest import TINY_CONFIGS, default_params, tiny_trace

pytestmark = pytest.mark.gpu

EST_RTOL = 1e-9


@pytest.fixture(scope="module")
def cb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06207_amd import cbaa
    cbaa.lib()
    return cbaa


def _say(*a):
    print("[case]", *a, flush=True)


def _update_scratch(cb, p, n, n_cubes, path, small=False):
    """Scratch for the partitioned path (None selects direct atomics)."""
    if path == "direct":
        return None
    need = cb.cbaa_update_scratch_bytes(p, n, n_cubes)
    if need == 0:          # configuration outside the partitioned path's limits
        return None
    if small:              # force several passes over the batch
        need = max(need // 3, 1)
        need = max(need, cb.cbaa_update_scratch_bytes(p, 65536, n_cubes))
    return cb.scratch_tensor(need)


def _gpu_cube(cb, p, pairs, side, path="direct", small=False):
    cube = cb.new_cube(p)
    scratch = _update_scratch(cb, p, len(pairs), 1, path, small)
    cb.cbaa_update(p, cube, cb.pairs_to_device(pairs), side, scratch)
    return cube


PATHS = ["direct", "partitioned"]


def _assert_hosts_equal(got, want):
    assert got.size == want.size, (got.size, want.size)
    for f in ("ip", "zeros", "cs", "flags"):
        assert np.array_equal(got[f], want[f]), f
    tol = EST_RTOL * np.maximum(1.0, np.abs(want["est"]))
    assert np.all(np.abs(got["est"] - want["est"]) <= tol)


# ---------------------------------------------------------------- update

@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("name", sorted(TINY_CONFIGS))
@pytest.mark.parametrize("side", [0, 1])
def test_update_tiny_configs_bitexact(cb, name, side, path):
    p = TINY_CONFIGS[name]
    t = tiny_trace(100 + side, n_hosts=3000, n_planted=30, fan_in=0.3)
    _say(name, side, path, t.n)
    got = cb.cube_to_numpy(_gpu_cube(cb, p, t.pairs, side, path))
    assert np.array_equal(got, O.cube_of(p, t.pairs, side))


@pytest.mark.parametrize("path", PATHS)
def test_update_small_window_bitexact(cb, small_window, path):
    p = default_params()
    _say("small window", path, small_window.n)
    got = cb.cube_to_numpy(_gpu_cube(cb, p, small_window.pairs, 0, path))
    assert np.array_equal(got, O.cube_of(p, small_window.pairs, 0))


@pytest.mark.parametrize("path,small", [("direct", False), ("partitioned", False),
                                        ("partitioned", True)])
def test_update2_both_sides_bitexact(cb, path, small):
    import torch
    p = default_params()
    t = tracegen.window_core_edge(12, scale=1 / 16)
    _say("update2", path, small, t.n)
    a, b = cb.new_cube(p), cb.new_cube(p)
    scratch = _update_scratch(cb, p, t.n, 2, path, small)
    cb.cbaa_update2(p, a, b, cb.pairs_to_device(t.pairs), scratch)
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(a), O.cube_of(p, t.pairs, 0))
    assert np.array_equal(cb.cube_to_numpy(b), O.cube_of(p, t.pairs, 1))


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 65535, 65536, 65537, 1000003])
def test_update_ragged_sizes(cb, n, path):
    p = default_params()
    rng = np.random.default_rng(n)
    pairs = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    _say("ragged", path, n)
    got = cb.cube_to_numpy(_gpu_cube(cb, p, pairs, 0, path))
    assert np.array_equal(got, O.cube_of(p, pairs, 0))


@pytest.mark.parametrize("path", PATHS)
def test_update_skewed_single_host_and_repeats(cb, path):
    p = default_params()
    rng = np.random.default_rng(5)
    n = 2_000_000
    one_host = np.stack([np.full(n, 0x0A0B0C0D, np.uint32),
                         rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)], axis=1)
    same_pair = np.tile(np.array([[1, 2]], np.uint32), (n, 1))
    for pairs in (one_host, same_pair):
        _say("skew", path)
        got = cb.cube_to_numpy(_gpu_cube(cb, p, pairs, 0, path))
        assert np.array_equal(got, O.cube_of(p, pairs, 0))


def test_update_partitioned_onto_nonempty_cube(cb):
    """The partitioned path ORs into what the cube already holds."""
    import torch
    p = default_params()
    t = tracegen.window_core_edge(15, scale=1 / 64)
    half = t.n // 2
    cube = _gpu_cube(cb, p, t.pairs[:half], 1, "direct")
    scratch = _update_scratch(cb, p, t.n - half, 1, "partitioned")
    cb.cbaa_update(p, cube, cb.pairs_to_device(t.pairs[half:]), 1, scratch)
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(cube), O.cube_of(p, t.pairs, 1))


def test_update_scratch_too_small_rejected(cb):
    p = default_params()
    tiny = cb.scratch_tensor(1024)
    cube = cb.new_cube(p)
    with pytest.raises(cb.CbaaError) as ei:
        cb.cbaa_update(p, cube, cb.pairs_to_device(np.ones((10, 2), np.uint32)), 0, tiny)
    assert ei.value.code == cb.CBAA_ESCRATCH


def test_update_concurrent_streams_and_batches(cb):
    """The same cube updated from several streams in random-size batches is
    the cube of the whole window."""
    import torch
    p = default_params()
    t = tracegen.window_core_edge(13, scale=1 / 32)
    rng = np.random.default_rng(6)
    cuts = np.sort(rng.choice(np.arange(1, t.n), 9, replace=False))
    parts = np.split(t.pairs, cuts)
    cube = cb.new_cube(p)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    dev = [cb.pairs_to_device(q) for q in parts]
    torch.cuda.synchronize()
    scratch = [_update_scratch(cb, p, max(len(q) for q in parts), 1, "partitioned")
               for _ in range(3)]
    for i, q in enumerate(dev):
        # alternate the two update paths on three streams
        cb.cbaa_update(p, cube, q, 0, scratch[i % 3] if i % 2 else None, stream=streams[i % 3])
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(cube), O.cube_of(p, t.pairs, 0))


# ---------------------------------------------------------------- merge

def test_merge_or_router_split(cb):
    import torch
    p = default_params()
    t = tracegen.window_core_edge(14, scale=1 / 64)
    parts = tracegen.split_routers(t.pairs, 11, seed=3)
    cubes = [_gpu_cube(cb, p, q, 0) for q in parts]
    whole = O.cube_of(p, t.pairs, 0)
    dst = cb.new_cube(p, init=False)
    cb.cbaa_merge_or(p, dst, cubes)          # 11 sources: two launches
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(dst), whole)
    cb.cbaa_merge_or(p, cubes[5], cubes[:7])  # destination aliases a source
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(cubes[5]),
                          O.cube_of(p, np.concatenate(parts[:7]), 0))


# ---------------------------------------------------------------- column statistics

@pytest.mark.parametrize("name", ["default_g64", "hetero_r5", "g128_r3"])
def test_column_zeros_and_fills(cb, name):
    import torch
    p = TINY_CONFIGS[name]
    t = tiny_trace(7, n_hosts=5000, n_planted=40)
    cube = _gpu_cube(cb, p, t.pairs, 0)
    S = 1 << p["r"]
    A = p["n_ra"] + p["n_va"]
    W = sum(1 << p["cbn"][a] for a in range(A))
    zeros = torch.empty(S * W, dtype=torch.int16, device="cuda")
    ones = torch.empty(S * A, dtype=torch.int32, device="cuda")
    cb.cbaa_column_zeros(p, cube, zeros, ones)
    torch.cuda.synchronize()
    wz, wo = O.column_zeros(p, O.cube_of(p, t.pairs, 0))
    assert np.array_equal(zeros.cpu().numpy().view(np.uint16), wz)
    assert np.array_equal(ones.cpu().numpy().view(np.uint32), wo)


# ---------------------------------------------------------------- restore

@pytest.mark.parametrize("name", sorted(TINY_CONFIGS))
@pytest.mark.parametrize("rule", [0, 1])
def test_restore_tiny_configs(cb, name, rule):
    p = TINY_CONFIGS[name]
    theta = 16.0 if p["log2_g"] == 6 else 32.0
    t = tiny_trace(200 + rule, n_hosts=3000, n_planted=30, fan_in=0.3)
    cube_np = O.cube_of(p, t.pairs, 0)
    _say("restore", name, rule)
    cube = _gpu_cube(cb, p, t.pairs, 0)
    got, st = cb.restore(p, cube, theta, rule)
    want, wst = O.restore(p, cube_np, theta, rule)
    assert st["hot_columns"] == wst["hot_columns"]
    assert st["tuples_checked"] <= wst["cp_valid"]
    _assert_hosts_equal(got, want)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_restore_small_window(cb, seed):
    p = default_params()
    t = tracegen.window_small(seed)
    cube = _gpu_cube(cb, p, t.pairs, 0)
    got, st = cb.restore(p, cube, 1024.0)
    want, wst = O.restore(p, O.cube_of(p, t.pairs, 0), 1024.0)
    _say("small window restore", seed, got.size, st)
    assert got.size > 50
    _assert_hosts_equal(got, want)


def test_restore_capacity_overflow_and_empty(cb):
    import torch
    p = default_params()
    t = tracegen.window_small(4)
    cube = _gpu_cube(cb, p, t.pairs, 0)
    scratch = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, 8))
    out = torch.empty(8 * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    cb.cbaa_restore(p, cube, 1024.0, 0, scratch, out, 8, st)
    torch.cuda.synchronize()
    assert int(st[0]) > 8
    cut = cb.host_list(out, 8)
    full, _ = cb.restore(p, cube, 1024.0, capacity=8)   # grows and retries
    assert full.size == int(st[0])
    # a cut output: 8 distinct hosts of the full list, in ascending IP order
    assert np.all(np.diff(cut["ip"].astype(np.int64)) > 0)
    rows = {int(h["ip"]): h for h in full}
    for h in cut:
        ref = rows[int(h["ip"])]
        assert (h["zeros"], h["cs"], h["flags"]) == (ref["zeros"], ref["cs"], ref["flags"])
    empty, est = cb.restore(p, cb.new_cube(p), 1024.0)
    assert empty.size == 0 and est["hot_columns"] == 0
    # capacity 0: counts only
    scratch0 = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, 0))
    cb.cbaa_restore(p, cube, 1024.0, 0, scratch0, None, 0, st)
    torch.cuda.synchronize()
    assert int(st[0]) == full.size


def test_restore_saturated_host(cb):
    import torch
    p = TINY_CONFIGS["ra4_va2"]
    host = 0xC0A80001
    pairs = np.stack([np.full(20000, host, np.uint32),
                      np.arange(20000, dtype=np.uint32) * np.uint32(2654435761)], axis=1)
    cube = _gpu_cube(cb, p, pairs, 0)
    got, _ = cb.restore(p, cube, 16.0)
    want, _ = O.restore(p, O.cube_of(p, pairs, 0), 16.0)
    _assert_hosts_equal(got, want)
    assert host in got["ip"].tolist()
    assert got["flags"][got["ip"] == host][0] == cb.FLAG_SATURATED


def _cube_from_numpy(cb, p, cube_np):
    """A device cube with a valid header of p holding the oracle's bits."""
    return cb.cube_from_bits(p, cube_np)


def _set_columns(p, cube_np, cs, a, cols):
    """All g bits of the listed columns of array a in sketch cs."""
    g = 1 << p["log2_g"]
    R = g // 64
    ncol = [1 << c for c in p["cbn"][: p["n_ra"] + p["n_va"]]]
    W = sum(ncol)
    aoff = int(sum(ncol[:a]))
    for rb in range(R):
        cube_np[(cs * R + rb) * W + aoff + np.asarray(cols)] = np.uint64(0xFFFFFFFFFFFFFFFF)


def test_restore_long_hot_list_on_the_trace_cube(cb):
    """A window cube whose RA 0 in sketch 3 has 1500 saturated columns: that
    hot list no longer fits the per-list gather buffer, so the join reads the
    cube directly; the result is the oracle's."""
    p = default_params()
    t = tracegen.window_small(2)
    cube_np = O.cube_of(p, t.pairs, 0).copy()
    _set_columns(p, cube_np, 3, 0, np.arange(1000, 2500))
    _say("long hot list")
    got, st = cb.restore(p, _cube_from_numpy(cb, p, cube_np), 1024.0)
    want, wst = O.restore(p, cube_np, 1024.0)
    assert st["hot_columns"] == wst["hot_columns"] and wst["hot_columns"] > 1500
    _assert_hosts_equal(got, want)


def test_restore_tens_of_thousands_of_hosts(cb):
    """Sketch 0 with RA 0, RA 1 and the VA fully set and one RA 2 column set:
    every LP with that RA 2 column restores (2^(28-12) = 65536 hosts, all
    saturated), which takes the long-list join and the large-list sort."""
    p = default_params()
    g = 1 << p["log2_g"]
    words = (1 << p["r"]) * (g // 64) * sum(1 << c for c in p["cbn"][:4])
    cube_np = np.zeros(words, np.uint64)
    _set_columns(p, cube_np, 0, 0, np.arange(4096))
    _set_columns(p, cube_np, 0, 1, np.arange(4096))
    _set_columns(p, cube_np, 0, 2, [1234])
    _set_columns(p, cube_np, 0, 3, np.arange(4096))
    _say("65536 hosts")
    got, st = cb.restore(p, _cube_from_numpy(cb, p, cube_np), 1024.0)
    want, _ = O.restore(p, cube_np, 1024.0)
    assert want.size == 65536
    _assert_hosts_equal(got, want)
    assert np.all(np.diff(got["ip"].astype(np.int64)) > 0)


@pytest.mark.parametrize("k,alias", [(1, False), (2, False), (3, True), (16, False), (17, True)])
def test_merge_restore_equals_merge_then_restore(cb, k, alias):
    """The fused window end (OR-merge counted in one pass, then the restore)
    gives the cube and the host list of cbaa_merge_or followed by
    cbaa_restore, for k routers (k > 16 takes the merge-first path), with the
    destination one of the sources or not; and the oracle's hosts."""
    import torch
    p = default_params()
    t = tracegen.window_small(7)
    parts = tracegen.split_routers(t.pairs, k, seed=7)
    srcs = [_gpu_cube(cb, p, q, 0) for q in parts]
    dst = srcs[0] if alias else cb.new_cube(p, init=False)
    want_cube = O.cube_of(p, t.pairs, 0)
    cap = 4096
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    _say("merge restore", k, alias)
    cb.cbaa_merge_restore(p, dst, srcs, 1024.0, cb.THR_THM2, rs, out, cap, st)
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(dst), want_cube)
    got = cb.host_list(out, int(st[0]))
    want, _ = O.restore(p, want_cube, 1024.0)
    _assert_hosts_equal(got, want)
    # the same window through the two separate calls
    g2 = cb.new_cube(p, init=False)
    cb.cbaa_merge_or(p, g2, [s_ for s_ in srcs if s_ is not dst] + ([dst] if alias else []))
    got2, _ = cb.restore(p, g2, 1024.0)
    _assert_hosts_equal(got2, got)


def _merge_restore(cb, p, dst, srcs, cap=4096):
    import torch
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    cb.cbaa_merge_restore(p, dst, srcs, 1024.0, cb.THR_THM2, rs, out, cap, st)
    torch.cuda.synchronize()
    return cb.host_list(out, int(st[0])), st.cpu().numpy().copy()


@pytest.mark.parametrize("k", [1, 2, 5, 16])
def test_merge_restore_without_destination(cb, k):
    """With no destination the merged cube is not stored and the restore reads
    every column it needs as the OR of the router cubes: the host list and the
    restore counters are those of the stored case, and the oracle's hosts."""
    p = default_params()
    t = tracegen.window_small(8)
    parts = tracegen.split_routers(t.pairs, k, seed=8)
    srcs = [_gpu_cube(cb, p, q, 0) for q in parts]
    _say("merge restore, no destination", k)
    got, st = _merge_restore(cb, p, None, srcs)
    ref, st_ref = _merge_restore(cb, p, cb.new_cube(p, init=False), srcs)
    assert np.array_equal(st, st_ref)
    _assert_hosts_equal(got, ref)
    want, _ = O.restore(p, O.cube_of(p, t.pairs, 0), 1024.0)
    _assert_hosts_equal(got, want)


def test_merge_restore_without_destination_long_hot_list(cb):
    """The long-hot-list cube (a list too long for the gather buffer, so the
    join reads cube columns directly) split over three router cubes: with no
    destination those direct reads OR the three sources."""
    p = default_params()
    t = tracegen.window_small(2)
    cube_np = O.cube_of(p, t.pairs, 0).copy()
    _set_columns(p, cube_np, 3, 0, np.arange(1000, 2500))
    rng = np.random.default_rng(3)
    who = rng.integers(0, 3, cube_np.size)   # every word of the cube goes to one router
    srcs = [_cube_from_numpy(cb, p, np.where(who == i, cube_np, np.uint64(0))) for i in range(3)]
    _say("merge restore, no destination, long hot list")
    got, st = _merge_restore(cb, p, None, srcs)
    want, wst = O.restore(p, cube_np, 1024.0)
    assert st[1] == wst["hot_columns"] and wst["hot_columns"] > 1500
    _assert_hosts_equal(got, want)


def test_merge_restore_without_destination_needs_at_most_16_sources(cb):
    p = default_params()
    srcs = [cb.new_cube(p) for _ in range(17)]
    import torch
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, 16))
    out = torch.empty(16 * 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="16 source cubes"):
        cb.cbaa_merge_restore(p, None, srcs, 1024.0, cb.THR_THM2, rs, out, 16, cb.stats_tensor())


# ---------------------------------------------------------------- estimate

def test_estimate_matches_oracle(cb):
    p = default_params()
    t = tracegen.window_small(5)
    cube = _gpu_cube(cb, p, t.pairs, 0)
    rng = np.random.default_rng(2)
    hosts = np.concatenate([t.planted_ips, t.bg_ips[:5000],
                            rng.integers(0, 1 << 32, 1000, dtype=np.uint64).astype(np.uint32)])
    est, zeros, layers = cb.estimate(p, cube, hosts, layers=True)
    cube_np = O.cube_of(p, t.pairs, 0)
    west, wz, _ = O.estimate(p, cube_np, hosts)
    assert np.array_equal(zeros, wz)
    assert np.all(np.abs(est - west) <= EST_RTOL * np.maximum(1.0, west))
    assert np.array_equal(layers, O.host_layer_zeros(p, cube_np, hosts))


# ---------------------------------------------------------------- full core-edge window

@pytest.fixture(scope="module")
def core_edge():
    return tracegen.window_core_edge(11)


@pytest.fixture(scope="module")
def core_edge_cubes(core_edge):
    """The oracle's source- and destination-keyed cubes of the window."""
    return [O.cube_of(default_params(), core_edge.pairs, side) for side in (0, 1)]


def test_full_core_edge_window(cb, core_edge, core_edge_cubes):
    """The 64Mi-packet window through cbaa_update2 and cbaa_restore: both
    cubes bit-exact and both restored lists equal to the oracle's."""
    import torch
    p = default_params()
    t = core_edge
    _say("core-edge full", t.n)
    a, b = cb.new_cube(p), cb.new_cube(p)
    scratch = _update_scratch(cb, p, t.n, 2, "partitioned")
    cb.cbaa_update2(p, a, b, cb.pairs_to_device(t.pairs), scratch)
    torch.cuda.synchronize()
    for side, cube in ((0, a), (1, b)):
        want_cube = core_edge_cubes[side]
        assert np.array_equal(cb.cube_to_numpy(cube), want_cube)
        got, st = cb.restore(p, cube, 1024.0)
        want, _ = O.restore(p, want_cube, 1024.0)
        _say("core-edge restore side", side, got.size, st)
        _assert_hosts_equal(got, want)


def test_benchmark_step_on_core_edge_window(cb, core_edge, core_edge_cubes):
    """The benchmark's timed step at full size, call for call: the window
    split over two edge routers (seed 11), one cbaa_update_batch of both
    routers' streams flagged fresh into cubes holding stale bits, then per side
    cbaa_merge_restore with no destination (the merged cube not stored). The
    router cubes OR to the oracle's cube of the window, and the restored lists
    are the oracle's under both threshold rules."""
    import torch
    p = default_params()
    t = core_edge
    parts = tracegen.split_routers(t.pairs, 2, seed=11)
    local = []
    for _ in parts:
        a, b = cb.new_cube(p, init=False), cb.new_cube(p, init=False)
        a.fill_(-1)
        b.fill_(-1)
        local.append((a, b))
    table = [(cb.pairs_to_device(q), a, b, cb.SIDE_SRC, cb.BATCH_FRESH)
             for q, (a, b) in zip(parts, local)]
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table))
    _say("benchmark step, update", [len(q) for q in parts])
    cb.cbaa_update_batch(p, table, scratch)
    torch.cuda.synchronize()
    cap = 1 << 14
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    for side in (0, 1):
        merged = cb.cube_to_numpy(local[0][side]) | cb.cube_to_numpy(local[1][side])
        assert np.array_equal(merged, core_edge_cubes[side]), side
        del merged
        for rule in (cb.THR_THM2, cb.THR_PAPER):
            _say("benchmark step, window end", side, rule)
            cb.cbaa_merge_restore(p, None, [x[side] for x in local], 1024.0, rule, rs, out, cap, st)
            s = cb.stats_dict(st)
            assert s["status"] == 0 and s["n_hosts"] <= cap
            got = cb.host_list(out, s["n_hosts"])
            want, wst = O.restore(p, core_edge_cubes[side], 1024.0, rule)
            _say("  hosts", got.size, "tuple space", s["tuple_space"], wst)
            assert s["tuple_space"] == wst["tuples"]
            _assert_hosts_equal(got, want)


# ---------------------------------------------------------------- g = 8192

@pytest.mark.parametrize("path", PATHS)
def test_g8192_update_restore_estimate(cb, path):
    """Columns of 8192 bits (128 row blocks; two 64-bit words per lane in the
    join and the estimate): cube, restored list and estimates against the
    oracle."""
    p = dict(default_params(), log2_g=13)
    t = tracegen.window_small(6)
    _say("g8192", path)
    cube = _gpu_cube(cb, p, t.pairs, 0, path)
    want_cube = O.cube_of(p, t.pairs, 0)
    assert np.array_equal(cb.cube_to_numpy(cube), want_cube)
    for rule in (cb.THR_THM2, cb.THR_PAPER):
        got, st = cb.restore(p, cube, 1024.0, rule)
        want, _ = O.restore(p, want_cube, 1024.0, rule)
        assert got.size > 10
        _assert_hosts_equal(got, want)
    hosts = np.concatenate([t.planted_ips, t.bg_ips[:3000]])
    est, zeros = cb.estimate(p, cube, hosts)
    west, wz, _ = O.estimate(p, want_cube, hosts)
    assert np.array_equal(zeros, wz)
    assert np.all(np.abs(est - west) <= EST_RTOL * np.maximum(1.0, west))


@pytest.mark.parametrize("k,stored", [(2, False), (3, True), (16, False), (17, True)])
def test_merge_scan_then_restore_scanned_equals_the_fused_call(cb, k, stored):
    """The window end in two calls (merge, column scan and hot lists; then
    the tuple check and ordering from the scratch) gives the fused call's
    cube, stats and host list, and the oracle's hosts."""
    import torch
    p = default_params()
    t = tracegen.window_small(9)
    parts = tracegen.split_routers(t.pairs, k, seed=9)
    srcs = [_gpu_cube(cb, p, q, 0) for q in parts]
    _say("merge scan + restore scanned", k, stored)
    ref, st_ref = _merge_restore(cb, p, cb.new_cube(p, init=False) if stored else None, srcs)
    cap = 4096
    dst = cb.new_cube(p, init=False) if stored else None
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()
    cb.cbaa_merge_scan(p, dst, srcs, 1024.0, cb.THR_THM2, rs, out, cap, st)
    cb.cbaa_restore_scanned(p, dst, srcs, 1024.0, cb.THR_THM2, rs, out, cap, st)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), st_ref)
    got = cb.host_list(out, int(st[0]))
    _assert_hosts_equal(got, ref)
    want_cube = O.cube_of(p, t.pairs, 0)
    if stored:
        assert np.array_equal(cb.cube_to_numpy(dst), want_cube)
    want, _ = O.restore(p, want_cube, 1024.0)
    _assert_hosts_equal(got, want)


def test_two_sides_with_the_second_scan_after_the_first(cb):
    """Both sides of a window on two streams, the second side's merge scan
    waiting on an event after the first side's hot lists, each side's tuple
    check after its own scan: both lists equal the fused calls' and the
    oracle's."""
    import torch
    p = default_params()
    t = tracegen.window_small(10)
    parts = tracegen.split_routers(t.pairs, 2, seed=10)
    local = [(_gpu_cube(cb, p, q, 0), _gpu_cube(cb, p, q, 1)) for q in parts]
    cap = 4096
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rs = [cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap)) for _ in range(2)]
    outs = [torch.empty(cap * 16, dtype=torch.uint8, device="cuda") for _ in range(2)]
    sts = [cb.stats_tensor() for _ in range(2)]
    _say("two sides, ordered scans")
    fork = torch.cuda.Event()
    fork.record(torch.cuda.current_stream())
    for s_ in streams:
        s_.wait_event(fork)
    args = [(p, None, [x[i] for x in local], 1024.0, cb.THR_THM2, rs[i], outs[i], cap, sts[i],
             streams[i]) for i in range(2)]
    cb.cbaa_merge_scan(*args[0])
    scanned = torch.cuda.Event()
    scanned.record(streams[0])
    streams[1].wait_event(scanned)
    cb.cbaa_merge_scan(*args[1])
    cb.cbaa_restore_scanned(*args[0])
    cb.cbaa_restore_scanned(*args[1])
    torch.cuda.synchronize()
    for side in range(2):
        got = cb.host_list(outs[side], int(sts[side][0]))
        ref, st_ref = _merge_restore(cb, p, None, [x[side] for x in local])
        assert np.array_equal(sts[side].cpu().numpy(), st_ref)
        _assert_hosts_equal(got, ref)
        want, _ = O.restore(p, O.cube_of(p, t.pairs, side), 1024.0)
        _assert_hosts_equal(got, want)
