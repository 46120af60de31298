"""Batched update of several edge routers' streams through one sequence of
launches, its tile/partition shapes, HIP-graph capture and replay, and the
autotuner -- all against the CPU oracle (bit-exact cubes)."""

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


def _streams(seed, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for i, n in enumerate(sizes):
        if n < 50_000:
            out.append(rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32))
            continue
        t = tracegen.make_window(n, max(1, n // 8), 2, 300, 3000, dup_frac=0.1,
                                 fan_in_frac=0.5, seed=int(rng.integers(1, 1 << 30)))
        out.append(t.pairs)
    return out


@pytest.mark.parametrize("two", [False, True])
def test_batch_uneven_streams_bitexact(cb, two):
    import torch
    p = default_params()
    sizes = [70_000, 0, 1, 300_000, 4_099, 1_200_000, 65_536]
    parts = _streams(3 + two, sizes)
    cubes = []
    table = []
    for i, q in enumerate(parts):
        a = cb.new_cube(p)
        b = cb.new_cube(p) if two else None
        cubes.append((a, b))
        table.append((cb.pairs_to_device(q) if len(q) else torch.zeros((0, 2), dtype=torch.int32,
                                                                        device="cuda"),
                      a, b, i % 2))
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table))
    cb.cbaa_update_batch(p, table, scratch)
    torch.cuda.synchronize()
    for i, (q, (a, b)) in enumerate(zip(parts, cubes)):
        side = 0 if two else i % 2
        assert np.array_equal(cb.cube_to_numpy(a), O.cube_of(p, q, side)), i
        if two:
            assert np.array_equal(cb.cube_to_numpy(b), O.cube_of(p, q, 1)), i


@pytest.mark.parametrize("tuning", [dict(chunk_pairs=16384), dict(chunk_pairs=131072, seg_records=8192),
                                    dict(apply_blocks=37), dict(chunk_pairs=1024, seg_records=1024,
                                                                apply_blocks=2048),
                                    dict(chunk_pairs=32768, seg_records=262144, apply_blocks=768)])
def test_batch_tunings_and_shared_cube(cb, tuning):
    """Every tile/partition shape gives the same cube; two streams that share
    a cube give the cube of their union."""
    import torch
    p = default_params()
    parts = _streams(9, [500_000, 123_457, 800_000])
    shared = cb.new_cube(p)
    own = cb.new_cube(p)
    table = [(cb.pairs_to_device(parts[0]), shared, None, 0),
             (cb.pairs_to_device(parts[1]), own, None, 1),
             (cb.pairs_to_device(parts[2]), shared, None, 0)]
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table, tuning))
    cb.cbaa_update_batch(p, table, scratch, tuning)
    torch.cuda.synchronize()
    assert np.array_equal(cb.cube_to_numpy(shared),
                          O.cube_of(p, np.concatenate([parts[0], parts[2]]), 0))
    assert np.array_equal(cb.cube_to_numpy(own), O.cube_of(p, parts[1], 1))


def _skewed(seed, n):
    """n pairs from distinct sources to one destination: in the source-keyed
    cube every record lands in the row block of that destination's bit, so a
    few bins hold n / 2^r records each (several apply items per bin)."""
    rng = np.random.default_rng(seed)
    src = rng.choice(1 << 32, n, replace=False).astype(np.uint32)
    return np.stack([src, np.full(n, 0x0A000001, np.uint32)], axis=1)


@pytest.mark.parametrize("two", [False, True])
@pytest.mark.parametrize("tuning", [None, dict(chunk_pairs=4096, seg_records=2048)])
def test_fresh_streams_overwrite_their_cubes(cb, two, tuning):
    """Streams flagged fresh start from empty cubes whatever the cubes held
    (all-ones here): stale bits vanish, an empty stream leaves an empty cube,
    bins split over several apply items are cleared before they are OR-ed,
    and a stream without the flag in the same batch still ORs into its cube."""
    import torch
    p = default_params()
    parts = _streams(31 + two, [70_000, 0, 300_000, 4_099]) + [_skewed(5, 120_000)]
    table, cubes, fresh = [], [], []
    for i, q in enumerate(parts):
        a = cb.new_cube(p, init=False)
        b = cb.new_cube(p, init=False) if two else None
        is_fresh = i != 3                      # stream 3 keeps the OR semantics
        for c in (a, b):
            if c is None:
                continue
            if is_fresh:
                c.fill_(-1)                    # stale content to be overwritten
            else:
                cb.cbaa_cube_init(p, c)
        cubes.append((a, b))
        fresh.append(is_fresh)
        dq = cb.pairs_to_device(q) if len(q) else torch.zeros((0, 2), dtype=torch.int32, device="cuda")
        table.append((dq, a, b, 0, cb.BATCH_FRESH if is_fresh else 0))
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table, tuning))
    cb.cbaa_update_batch(p, table, scratch, tuning)
    torch.cuda.synchronize()
    for i, (q, (a, b)) in enumerate(zip(parts, cubes)):
        assert np.array_equal(cb.cube_to_numpy(a), O.cube_of(p, q, 0)), (i, fresh[i])
        if two:
            assert np.array_equal(cb.cube_to_numpy(b), O.cube_of(p, q, 1)), (i, fresh[i])


def test_fresh_batch_without_pairs_empties_cubes(cb):
    import torch
    p = default_params()
    a = cb.new_cube(p, init=False)
    a.fill_(-1)
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    table = [(empty, a, None, 0, cb.BATCH_FRESH)]
    cb.cbaa_update_batch(p, table, cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table)))
    torch.cuda.synchronize()
    assert not cb.cube_to_numpy(a).any()


def test_batch_rejects_bad_tables(cb):
    import torch
    p = default_params()
    a, b, c = cb.new_cube(p), cb.new_cube(p), cb.new_cube(p)
    pr = cb.pairs_to_device(np.ones((10, 2), np.uint32))
    scratch = cb.scratch_tensor(1 << 20)
    with pytest.raises(cb.CbaaError):          # mixed one- and two-cube streams
        cb.cbaa_update_batch(p, [(pr, a, b, 0), (pr, a, None, 0)], scratch)
    with pytest.raises(cb.CbaaError):          # too many streams
        cb.cbaa_update_batch(p, [(pr, a, None, 0)] * 33, scratch)
    with pytest.raises(cb.CbaaError):          # scratch too small
        cb.cbaa_update_batch(p, [(pr, a, None, 0)], cb.scratch_tensor(256))
    with pytest.raises(cb.CbaaError):          # tuning out of range
        cb.cbaa_update_batch(p, [(pr, a, None, 0)], scratch, dict(chunk_pairs=1000))
    with pytest.raises(cb.CbaaError):          # a fresh stream's cube named twice
        cb.cbaa_update_batch(p, [(pr, a, None, 0, cb.BATCH_FRESH), (pr, a, None, 1)], scratch)
    with pytest.raises(cb.CbaaError):          # ... also as another stream's second cube
        cb.cbaa_update_batch(p, [(pr, a, b, 0, cb.BATCH_FRESH), (pr, b, c, 0)], scratch)
    with pytest.raises(cb.CbaaError):          # unknown flag bits
        cb.cbaa_update_batch(p, [(pr, a, None, 0, 2)], scratch)
    torch.cuda.synchronize()


@pytest.mark.parametrize("fresh", [False, True])
def test_graph_capture_replays_batch_merge_restore(cb, fresh):
    """The per-window sequence -- zero the routers' cubes (or flag them fresh),
    batched update, OR-merge into the global cube, restore -- captured once in
    a HIP graph and replayed; every replay equals the eager run and the
    oracle."""
    import torch
    p = default_params()
    parts = _streams(17, [400_000, 900_000, 50_000, 250_000])
    cubes = [cb.new_cube(p) for _ in parts]
    glob = cb.new_cube(p, init=False)
    d_parts = [cb.pairs_to_device(q) for q in parts]
    table = [(q, c, None, 0, cb.BATCH_FRESH if fresh else 0) for q, c in zip(d_parts, cubes)]
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table))
    cap = 4096
    rs = cb.scratch_tensor(cb.cbaa_restore_scratch_bytes(p, cap))
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    st = cb.stats_tensor()

    def window():
        if not fresh:
            for c in cubes:
                cb.cbaa_cube_init(p, c)
        cb.cbaa_update_batch(p, table, scratch)
        cb.cbaa_merge_or(p, glob, cubes)
        cb.cbaa_restore(p, glob, 64.0, cb.THR_THM2, rs, out, cap, st)

    window()
    torch.cuda.synchronize()
    want_cube = cb.cube_to_numpy(glob).copy()
    n = int(st[0])
    want_hosts = cb.host_list(out, n)
    oracle_cube = O.cube_of(p, np.concatenate(parts), 0)
    assert np.array_equal(want_cube, oracle_cube)
    oh, _ = O.restore(p, oracle_cube, 64.0)
    assert np.array_equal(want_hosts["ip"], oh["ip"]) and n > 0

    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        window()
    torch.cuda.synchronize()
    for rep in range(3):
        glob.fill_(-1)           # eager work between replays
        for c in cubes:          # stale router cubes: replays must not depend on them
            c.fill_(-1)
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cb.cube_to_numpy(glob), want_cube), rep
        assert int(st[0]) == n
        assert np.array_equal(cb.host_list(out, n), want_hosts), rep


def test_autotuner_picks_a_valid_shape(cb):
    import torch
    from paper_1901_06207_amd import autotune
    p = default_params()
    parts = _streams(23, [2_000_000, 300_000])
    cubes = [cb.new_cube(p) for _ in parts]
    table = [(cb.pairs_to_device(q), c, None, 0) for q, c in zip(parts, cubes)]
    res = autotune.tune_update(p, table, repeats=2)
    assert res["best"] in [c["tuning"] for c in res["candidates"]]
    assert all(c["ms"] > 0 for c in res["candidates"])
    for c in cubes:
        cb.cbaa_cube_init(p, c)
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table, res["best"]))
    cb.cbaa_update_batch(p, table, scratch, res["best"])
    torch.cuda.synchronize()
    for q, c in zip(parts, cubes):
        assert np.array_equal(cb.cube_to_numpy(c), O.cube_of(p, q, 0))


def test_batch_of_32_streams_with_a_64mi_stream(cb):
    """CBAA_MAX_BATCH streams in one call: uneven sizes from empty to a full
    64Mi-packet core-edge window, both cubes per stream, fresh streams that own
    their cubes next to OR-ing streams that share two cube pairs holding earlier
    bits. Every cube equals the oracle's (fresh: the stream's own pairs; shared:
    the earlier bits OR-ed with every stream's pairs)."""
    import torch
    p = default_params()
    assert cb.MAX_BATCH == 32
    rng = np.random.default_rng(32)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(2_000), np.log(1_500_000), 31))]
    sizes[3], sizes[17] = 0, 1
    print("[case] batch of 32 streams, one of 64Mi packets", flush=True)
    parts = _streams(32, sizes)
    big = tracegen.window_core_edge(14).pairs          # 64 x 2^20 packets
    parts.insert(9, big)
    fresh_idx = [0, 9, 20, 31]                          # own their cubes, start empty
    shared = [(cb.new_cube(p), cb.new_cube(p)) for _ in range(2)]
    # earlier bits in the shared cubes
    prior = _streams(99, [200_000, 150_000])
    for (a, b), q in zip(shared, prior):
        cb.cbaa_update2(p, a, b, cb.pairs_to_device(q))
    own = {}
    table = []
    for i, q in enumerate(parts):
        d = cb.pairs_to_device(q) if len(q) else torch.zeros((0, 2), dtype=torch.int32,
                                                             device="cuda")
        if i in fresh_idx:
            a, b = cb.new_cube(p, init=False), cb.new_cube(p, init=False)
            a.fill_(-1)                                  # stale content the call must overwrite
            b.fill_(-1)
            own[i] = (a, b)
            table.append((d, a, b, cb.SIDE_SRC, cb.BATCH_FRESH))
        else:
            a, b = shared[i % 2]
            table.append((d, a, b, cb.SIDE_SRC, 0))
    assert len(table) == 32
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table))
    cb.cbaa_update_batch(p, table, scratch)
    torch.cuda.synchronize()
    del scratch, table
    for i in fresh_idx:
        a, b = own[i]
        for side, cube in ((0, a), (1, b)):
            want = O.new_cube(p)
            O.update_omp(p, want, parts[i], side)
            assert np.array_equal(cb.cube_to_numpy(cube), want), (i, side)
        assert cb.cbaa_cube_check(p, a) == cb.CBAA_OK
    for j, (a, b) in enumerate(shared):
        for side, cube in ((0, a), (1, b)):
            want = O.new_cube(p)
            O.update_omp(p, want, prior[j], side)
            for i, q in enumerate(parts):
                if i not in fresh_idx and i % 2 == j:
                    O.update_omp(p, want, q, side)
            assert np.array_equal(cb.cube_to_numpy(cube), want), (j, side)


@pytest.mark.parametrize("dims", [dict(r=5, cl_bs=[5, 14, 23]), dict(log2_g=13),
                                  dict(r=5, cl_bs=[5, 14, 23], log2_g=13)])
def test_batch_with_up_to_4096_bins_per_cube(cb, dims):
    """Cubes of 2048 and 4096 bins per cube (32 sketches, 8192-bit columns,
    both) take the partitioned path's second shape (14 pairs per thread
    beside larger LDS counters): both cubes of uneven streams, fresh and
    OR-ing, bit-exact against the oracle."""
    import torch
    p = dict(default_params(), **dims)
    assert cb.cbaa_update_scratch_bytes(p, 1 << 20, 2) > 0      # partitioned, not direct
    print("[case] batch with", dims, flush=True)
    parts = _streams(77, [400_000, 0, 1_300_000, 70_001])
    table, cubes = [], []
    for i, q in enumerate(parts):
        a, b = cb.new_cube(p), cb.new_cube(p)
        if i == 3:   # an OR-ing stream onto cubes holding earlier bits
            cb.cbaa_update2(p, a, b, cb.pairs_to_device(parts[0]))
        cubes.append((a, b))
        d = cb.pairs_to_device(q) if len(q) else torch.zeros((0, 2), dtype=torch.int32, device="cuda")
        table.append((d, a, b, cb.SIDE_SRC, 0 if i == 3 else cb.BATCH_FRESH))
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table))
    cb.cbaa_update_batch(p, table, scratch)
    torch.cuda.synchronize()
    for i, (q, (a, b)) in enumerate(zip(parts, cubes)):
        src = np.concatenate([parts[0], q]) if i == 3 else q
        assert np.array_equal(cb.cube_to_numpy(a), O.cube_of(p, src, 0)), i
        assert np.array_equal(cb.cube_to_numpy(b), O.cube_of(p, src, 1)), i


def _skewed_stream(seed):
    """Three histogram chunks of 65536 pairs: random pairs, then one host
    with 65536 distinct destinations, then one destination with 65536
    distinct sources. Only the first chunk is sampled, where every bin (one
    row block of one sketch) gets about 64 records; the two hosts' sketches
    get about 1024 records in each of their 64 row blocks' bins, several
    times the room the sample gives them."""
    rng = np.random.default_rng(seed)
    n = 65536
    rand = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    peers = rng.choice(1 << 32, 2 * n, replace=False).astype(np.uint32)
    out = np.column_stack([np.full(n, 0x0A000001, np.uint32), peers[:n]])
    inn = np.column_stack([peers[n:], np.full(n, 0xC0A80101, np.uint32)])
    return np.concatenate([rand, out, inn])


@pytest.mark.parametrize("two", [False, True])
def test_bins_the_sample_underestimates_overflow_exactly(cb, two):
    """Records beyond a bin's sampled room take the overflow list and are
    OR-ed in after the apply: fresh and OR-ing streams, one and two cubes,
    bit-exact against the oracle."""
    import torch
    p = default_params()
    tuning = dict(chunk_pairs=65536)
    print("[case] overflow two=%s" % two, flush=True)
    parts = [_skewed_stream(5), _skewed_stream(6), _skewed_stream(7)]
    earlier = _streams(8, [200_000])[0]
    table, cubes = [], []
    for i, q in enumerate(parts):
        a = cb.new_cube(p)
        b = cb.new_cube(p) if two else None
        if i == 2:   # OR onto cubes holding earlier bits
            if two:
                cb.cbaa_update2(p, a, b, cb.pairs_to_device(earlier))
            else:
                cb.cbaa_update(p, a, cb.pairs_to_device(earlier), cb.SIDE_DST)
        cubes.append((a, b))
        side = cb.SIDE_SRC if two or i == 0 else cb.SIDE_DST
        table.append((cb.pairs_to_device(q), a, b, side, 0 if i == 2 else cb.BATCH_FRESH))
    scratch = cb.scratch_tensor(cb.cbaa_update_batch_scratch_bytes(p, table, tuning))
    cb.cbaa_update_batch(p, table, scratch, tuning)
    torch.cuda.synchronize()
    for i, (q, (a, b)) in enumerate(zip(parts, cubes)):
        src = np.concatenate([earlier, q]) if i == 2 else q
        side = 0 if two or i == 0 else 1
        assert np.array_equal(cb.cube_to_numpy(a), O.cube_of(p, src, side)), i
        if two:
            assert np.array_equal(cb.cube_to_numpy(b), O.cube_of(p, src, 1)), i
