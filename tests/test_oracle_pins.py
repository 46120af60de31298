"""Pins of the CPU oracle to things other than itself: the paper's printed
dimensions, closed forms, invariants the method guarantees, textbook linear
counting, brute force over the whole IPv4 space, and exact counting by nested
loops. No GPU needed."""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
import tracegen
from conftest import GOLDEN, TINY_CONFIGS, default_params, tiny_params, tiny_trace


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- dimensions

def test_cube_is_128MB_at_paper_dimensions():
    g = _golden("paper_dims.json")
    p = default_params()
    assert (p["r"], p["n_ra"], p["n_va"], p["log2_g"]) == (g["r"], g["n_ra"], g["n_va"], g["log2_g"])
    assert p["cbn"] == g["cbn"]
    assert O.cube_words(p) * 8 == g["cube_bytes"]


def test_ep_cp_lengths_default_offsets():
    # Sec. 3.3: EPs are pairwise disjoint and cover LP; CP(i) = cbn(i) - |EP(i)|.
    p = default_params()
    ep, cp = O.ep_cp(p)
    assert sum(ep) == 32 - p["r"]
    assert ep == [10, 9, 9] and cp == [2, 3, 3]
    p2 = dict(p, cl_bs=[4, 12, 20])
    assert O.ep_cp(p2) == ([8, 8, 12], [4, 4, 0])


def test_invalid_configs_rejected():
    p = default_params()
    assert not O.config_ok(dict(p, cl_bs=[4, 20, 23]))     # |EP(0)|=16 > cbn: LP bits lost
    assert not O.config_ok(dict(p, cl_bs=[3, 14, 23]))     # start bit inside RP
    assert not O.config_ok(dict(p, cl_bs=[14, 4, 23]))     # not increasing
    assert not O.config_ok(dict(p, n_ra=1))


# ---------------------------------------------------------------- thresholds

def test_threshold_closed_form_no_sharing():
    """eps = 0 reduces both rules to floor(g e^{-theta/g}) (golden values)."""
    gold = _golden("threshold_eps0.json")
    for case in gold["cases"]:
        p = default_params()
        p["log2_g"] = case["log2_g"]
        S = 1 << p["r"]
        ones = np.zeros(S * 4, np.uint32)
        for rule in (O.THR_THM2, O.THR_PAPER):
            eps, zmax = O.thresholds(p, ones, case["theta"], rule)
            assert np.all(eps == 0.0)
            assert np.all(zmax == case["zmax"]), (case, rule)


def _cube_with_union_zeros(p, host, z_target, other_fill_bits=0, seed=0):
    """A cube where `host`'s union column has exactly z_target zeros: set the
    same g - z_target bits in each of its columns; optionally sprinkle other
    bits into columns that are not the host's."""
    rng = np.random.default_rng(seed)
    cube = O.new_cube(p)
    cs, cols = O.host_columns(p, host)
    g = 1 << p["log2_g"]
    R = g // 64
    A = p["n_ra"] + p["n_va"]
    cnt = [1 << p["cbn"][a] for a in range(A)]
    W = sum(cnt)
    aoff = np.cumsum([0] + cnt[:-1])
    bits = rng.choice(g, g - z_target, replace=False)
    for a in range(A):
        for b in bits:
            cube[(cs * R + b // 64) * W + aoff[a] + cols[a]] |= np.uint64(1) << np.uint64(b % 64)
    return cube, cs


def test_threshold_is_the_estimate_crossing_theta():
    """Thm. 2: est >= theta  <=>  Z <= Zmax. Checked through the estimator on
    union columns with Z = Zmax and Z = Zmax + 1 (reading THM2)."""
    p = default_params()
    theta = 1024.0
    host = 0x0A000001
    for z in (3189, 3190):
        cube, cs = _cube_with_union_zeros(p, host, z)
        _, ones = O.column_zeros(p, cube)
        eps, zmax = O.thresholds(p, ones, theta, O.THR_THM2)
        est, zz, _ = O.estimate(p, cube, np.array([host], np.uint32))
        assert zz[0] == z
        assert (est[0] >= theta) == (z <= zmax[cs])


def test_eps_is_product_of_fills_thm1():
    """Thm. 1 via simulation: the fraction of one bits in the union column of
    addresses that never occur equals eps, the product of the array fills."""
    p = dict(default_params(), r=1, cbn=[11, 10, 10, 10], cl_bs=[1, 12, 22])
    assert O.config_ok(p)
    t = tracegen.make_window(6_000_000, 3_000_000, 0, 1, 2, seed=3)
    cube = O.cube_of(p, t.pairs, O.SIDE_SRC)
    _, ones = O.column_zeros(p, cube)
    eps, _ = O.thresholds(p, ones, 1024.0)
    rng = np.random.default_rng(9)
    probe = rng.integers(0, 1 << 32, 6000, dtype=np.uint64).astype(np.uint32)
    probe = probe[~np.isin(probe, t.pairs[:, 0])]
    _, zeros, _ = O.estimate(p, cube, probe)
    g = 1 << p["log2_g"]
    cs = np.array([O.host_columns(p, int(h))[0] for h in probe[:64]])
    frac_one = 1.0 - zeros.astype(np.float64) / g
    # both sketches have near-equal fill; compare the mean with the mean eps
    assert 0.003 < eps.mean() < 0.2
    sigma = math.sqrt(eps.mean() * (1 - eps.mean()) / (g * probe.size))
    # neighbouring bits of one column are not independent draws; allow 6 sigma
    assert abs(frac_one.mean() - eps.mean()) < 6 * sigma + 0.02 * eps.mean(), (frac_one.mean(), eps)
    assert cs.size > 0


# ---------------------------------------------------------------- hashing / bijections

@pytest.mark.slow
def test_mangle_is_a_bijection_exhaustive():
    """Sec. 3.1: mangling is undone by its inverse for all 2^32 addresses."""
    p = default_params()
    assert O.check_mangle_bijection(p) == 0
    assert O.check_mangle_bijection(dict(p, seed_mangle=0xDEADBEEF)) == 0


def test_mangle_fixed_points_of_definition():
    # fmix32(0) = 0, so M(seed) = 0; the inverse maps 0 back to the seed.
    p = default_params()
    assert O.mangle(p, p["seed_mangle"]) == 0
    assert O.unmangle(p, 0) == p["seed_mangle"]


def test_hash_ranges_and_uniformity():
    p = default_params()
    g = 1 << p["log2_g"]
    xs = np.arange(200_000, dtype=np.uint32) * np.uint32(2654435761)
    bv = np.array([O.hash_bv(p, int(x)) for x in xs[:40000]])
    assert bv.min() >= 0 and bv.max() < g
    hist = np.bincount(bv >> 6, minlength=64)
    exp = bv.size / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 130  # 63 dof, p ~ 1e-6
    va = np.array([O.hash_va(p, 0, int(x) & ((1 << 28) - 1)) for x in xs[:40000]])
    assert va.max() < (1 << p["cbn"][3])


@pytest.mark.parametrize("name", ["default", "nowrap", "ra4", "ra2_r6"])
def test_lp_roundtrip_exhaustive(name):
    """Sec. 3.3: the EPs of a host's RA columns concatenate back to its LP,
    and its column tuple passes every CP check, for every LP."""
    p = {"default": default_params(),
         "nowrap": dict(default_params(), cl_bs=[4, 12, 20]),
         "ra4": TINY_CONFIGS["ra4_va2"],
         "ra2_r6": TINY_CONFIGS["ra2_va0"]}[name]
    assert O.check_lp_roundtrip(p) == 0


def test_cp_check_iff_tuple_is_some_hosts_columns():
    """A tuple passes Alg. 3's CP checks iff it equals the RA columns of the
    LP it reassembles to."""
    rng = np.random.default_rng(4)
    for p in (default_params(), dict(default_params(), cl_bs=[4, 12, 20]), TINY_CONFIGS["ra4_va2"]):
        n = p["n_ra"]
        L = 32 - p["r"]
        offs = [b - p["r"] for b in p["cl_bs"]]
        n_valid = 0
        for _ in range(3000):
            t = [int(rng.integers(0, 1 << p["cbn"][i])) for i in range(n)]
            if rng.random() < 0.3:  # force plausible tuples: columns of a random LP
                lp = int(rng.integers(0, 1 << L))
                t = [((lp >> o) | (lp << (L - o))) & ((1 << L) - 1) & ((1 << p["cbn"][i]) - 1)
                     if o else lp & ((1 << p["cbn"][i]) - 1) for i, o in enumerate(offs)]
            lp = O.tuple_check(p, t)
            # recompute the tuple's LP' from EPs and its columns independently
            ep, _ = O.ep_cp(p)
            lp2 = 0
            for i in range(n):
                e = t[i] & ((1 << ep[i]) - 1)
                o = offs[i]
                lp2 |= ((e << o) | (e >> (L - o))) & ((1 << L) - 1) if o else e
            cols = [(((lp2 >> o) | (lp2 << (L - o))) if o else lp2) & ((1 << p["cbn"][i]) - 1)
                    for i, o in enumerate(offs)]
            if lp is None:
                assert cols != t
            else:
                n_valid += 1
                assert lp == lp2 and cols == t
        assert n_valid > 500


# ---------------------------------------------------------------- cube contents

def _brute_cube(p, pairs, side):
    """Cube from the set of distinct (host, peer) pairs, one bit at a time,
    addressed by the documented layout."""
    g = 1 << p["log2_g"]
    R = g // 64
    A = p["n_ra"] + p["n_va"]
    cnt = [1 << p["cbn"][a] for a in range(A)]
    W = sum(cnt)
    aoff = np.cumsum([0] + cnt[:-1])
    cube = O.new_cube(p)
    seen = set()
    for s, d in pairs.tolist():
        host, peer = (s, d) if side == O.SIDE_SRC else (d, s)
        if (host, peer) in seen:
            continue
        seen.add((host, peer))
        cs, cols = O.host_columns(p, host)
        b = O.hash_bv(p, peer)
        for a in range(A):
            cube[(cs * R + b // 64) * W + aoff[a] + cols[a]] |= np.uint64(1) << np.uint64(b % 64)
    return cube


@pytest.mark.parametrize("side", [0, 1])
def test_update_equals_set_of_distinct_pairs(side):
    p = TINY_CONFIGS["hetero_r5"]
    t = tiny_trace(11, n_hosts=400, n_planted=5, fan_in=0.4)
    assert np.array_equal(O.cube_of(p, t.pairs, side), _brute_cube(p, t.pairs, side))


def test_update_invariant_to_order_and_duplicates():
    p = default_params()
    t = tiny_trace(12, n_hosts=2000, n_planted=10, lo=500, hi=3000)
    base = O.cube_of(p, t.pairs, O.SIDE_SRC)
    rng = np.random.default_rng(1)
    shuffled = t.pairs[rng.permutation(t.n)]
    dup = np.concatenate([t.pairs, t.pairs[rng.integers(0, t.n, t.n // 2)]])
    assert np.array_equal(base, O.cube_of(p, shuffled, O.SIDE_SRC))
    assert np.array_equal(base, O.cube_of(p, dup, O.SIDE_SRC))


def test_or_merge_of_router_cubes_is_cube_of_union():
    """Sec. 3.3: the global server ORs the routers' cubes; the result is the
    cube of all traffic, whatever the split, order or repetition."""
    p = default_params()
    t = tiny_trace(13, n_hosts=3000, n_planted=10, lo=500, hi=3000)
    whole = O.cube_of(p, t.pairs, O.SIDE_SRC)
    parts = tracegen.split_routers(t.pairs, 4, seed=2)
    cubes = [O.cube_of(p, q, O.SIDE_SRC) for q in parts]
    assert np.array_equal(O.merge_or(p, cubes), whole)
    assert np.array_equal(O.merge_or(p, cubes[::-1] + [cubes[0]]), whole)   # order, idempotence
    lost = O.merge_or(p, cubes[1:])      # a router that never reports
    assert np.array_equal(lost, O.cube_of(p, np.concatenate(parts[1:]), O.SIDE_SRC))


# ---------------------------------------------------------------- estimator statistics

@pytest.mark.parametrize("n", [64, 1024, 4096, 20000])
def test_linear_counting_expectation_lone_hosts(n):
    """Eq. 1 (linear counting): a host alone in its columns with n distinct
    peers leaves E[Z] = g (1 - 1/g)^n zeros; Var from the occupancy law."""
    p = default_params()
    g = 1 << p["log2_g"]
    T = 60 if n <= 4096 else 30
    hosts = tracegen.bijection32(np.arange(T, dtype=np.uint64), (17, 2654435761, 40503))
    peers = tracegen.bijection32(np.arange(T * n, dtype=np.uint64) + np.uint64(1 << 31),
                                 (5, 2246822519, 3266489917))
    pairs = np.stack([np.repeat(hosts, n), peers], axis=1).astype(np.uint32)
    cube = O.cube_of(p, pairs, O.SIDE_SRC)
    est, zeros, _ = O.estimate(p, cube, hosts)
    q = 1.0 - 1.0 / g
    ez = g * q ** n
    var = g * (g - 1) * (1 - 2.0 / g) ** n + ez - ez * ez
    se = math.sqrt(var / T)
    assert abs(zeros.mean() - ez) < 5 * se + 1.0, (zeros.mean(), ez, se)
    # the estimate is close to n while far from saturation
    assert abs(np.median(est) - n) < 0.08 * n + 4


def test_thm2_correction_reduces_bias_under_sharing():
    """Thm. 2: under heavy bit sharing the eps-corrected estimate is closer to
    the truth than plain linear counting on the union column."""
    p = dict(default_params(), r=1, cbn=[11, 10, 10, 10], cl_bs=[1, 12, 22])
    g = 1 << p["log2_g"]
    bg = tracegen.make_window(6_000_000, 3_000_000, 0, 1, 2, seed=21)
    n = 3000
    T = 40
    hosts = tracegen.bijection32(np.arange(T, dtype=np.uint64) + np.uint64(7 << 20),
                                 (99, 2654435761, 40503))
    peers = tracegen.bijection32(np.arange(T * n, dtype=np.uint64) + np.uint64(3 << 30),
                                 (1, 2246822519, 3266489917))
    tgt = np.stack([np.repeat(hosts, n), peers], axis=1).astype(np.uint32)
    cube = O.cube_of(p, np.concatenate([bg.pairs, tgt]), O.SIDE_SRC)
    est, zeros, _ = O.estimate(p, cube, hosts)
    plain = -g * np.log(np.maximum(zeros, 1) / g)
    _, ones = O.column_zeros(p, cube)
    eps, _ = O.thresholds(p, ones, 1024.0)
    assert eps.min() > 3e-3          # sharing is material
    bias_thm2 = abs(est.mean() - n)
    bias_plain = abs(plain.mean() - n)
    assert bias_thm2 < bias_plain
    assert bias_thm2 < 0.05 * n


# ---------------------------------------------------------------- row fills

def _layout(p):
    g = 1 << p["log2_g"]
    A = p["n_ra"] + p["n_va"]
    ncol = [1 << p["cbn"][a] for a in range(A)]
    return g, A, ncol, sum(ncol), [int(sum(ncol[:a])) for a in range(A)]


def test_row_ones_by_unpacking_every_bit():
    """Per-row counts against unpacking the whole cube bit by bit with numpy,
    addressed by the layout formula (g = 64 and g = 128 configurations)."""
    for name in ("default_g64", "g128_r3", "ra4_va2"):
        p = TINY_CONFIGS[name]
        g, A, ncol, W, aoff = _layout(p)
        S, R = 1 << p["r"], g // 64
        cube = O.cube_of(p, tiny_trace(9).pairs, O.SIDE_SRC)
        bits = np.unpackbits(cube.view(np.uint8), bitorder="little").reshape(S, R, W, 64)
        want = np.zeros((S, A, g), np.int64)
        for a in range(A):
            per = bits[:, :, aoff[a]:aoff[a] + ncol[a], :].sum(axis=2)   # [S, R, 64]
            want[:, a, :] = per.reshape(S, g)
        assert np.array_equal(O.row_ones(p, cube), want), name


def test_row_ones_sum_to_the_array_fills():
    """Summed over rows, the per-row counts are each array's one bits as the
    column scan counts them."""
    p = default_params()
    cube = O.cube_of(p, tracegen.window_small(3).pairs, O.SIDE_SRC)
    _, ones = O.column_zeros(p, cube)
    assert np.array_equal(O.row_ones(p, cube).sum(axis=2).ravel(), ones.astype(np.int64))


def test_row_shared_equals_g_eps_when_rows_fill_evenly():
    """Every column of array a holds k_a rows in a cyclic pattern, so each row
    is set in the same number of columns: the row-aware mass is g * eps of
    Thm. 1 (product of fills), up to rounding."""
    p = default_params()
    g, A, ncol, W, aoff = _layout(p)
    S, R = 1 << p["r"], g // 64
    cube = np.zeros(S * R * W, np.uint64)
    ks = [4, 16, 2, 8]
    for a, k in enumerate(ks):
        for col in range(ncol[a]):
            for j in range(k):
                b = (col * k + j) % g
                cube[(0 * R + b // 64) * W + aoff[a] + col] |= np.uint64(1 << (b % 64))
    rows = O.row_ones(p, cube)
    assert np.all(rows[0] == rows[0][:, :1])          # even rows
    shared = O.row_shared(p, rows)
    _, ones = O.column_zeros(p, cube)
    eps, _ = O.thresholds(p, ones, 1024.0)
    assert shared[0] == pytest.approx(g * eps[0], rel=1e-12)
    assert shared[0] == pytest.approx(g * np.prod([k / g for k in ks]), rel=1e-12)
    assert np.all(shared[1:] == 0.0)


def test_row_shared_counts_a_full_row_once():
    """A row set in every column of every array of a sketch adds exactly 1."""
    p = default_params()
    g, A, ncol, W, aoff = _layout(p)
    S, R = 1 << p["r"], g // 64
    cube = np.zeros(S * R * W, np.uint64)
    b0 = 777
    cube[(2 * R + b0 // 64) * W: (2 * R + b0 // 64 + 1) * W] = np.uint64(1 << (b0 % 64))
    shared = O.row_shared(p, O.row_ones(p, cube))
    assert shared[2] == 1.0 and shared.sum() == 1.0


def test_row_aware_count_removes_fan_in_row_pollution():
    """Ten destinations with 150k distinct sources each set their row bit in
    most source-keyed columns. Lone hosts with 5 peers then read as ~5 + the
    polluted rows under Thm. 2; the row-aware denominator g - sum_b q_b brings
    the estimate back to ~5."""
    p = default_params()
    g = 1 << p["log2_g"]
    rng = np.random.default_rng(4)
    srcs = rng.choice(1 << 32, 1_500_000, replace=False).astype(np.uint32)
    dsts = rng.integers(0, 1 << 32, 10, dtype=np.uint64).astype(np.uint32)
    fan_in = np.stack([srcs, np.repeat(dsts, 150_000)], axis=1)
    T, n = 200, 5
    hosts = tracegen.bijection32(np.arange(T, dtype=np.uint64) + np.uint64(5 << 24),
                                 (3, 2654435761, 40503))
    peers = tracegen.bijection32(np.arange(T * n, dtype=np.uint64) + np.uint64(1 << 30),
                                 (7, 2246822519, 3266489917))
    lone = np.stack([np.repeat(hosts, n), peers], axis=1).astype(np.uint32)
    cube = O.cube_of(p, np.concatenate([fan_in, lone]), O.SIDE_SRC)
    est, zeros, _ = O.estimate(p, cube, hosts)
    shared = O.row_shared(p, O.row_ones(p, cube))
    cs = np.array([O.host_columns(p, int(h))[0] for h in hosts])
    row_est = -g * np.log(np.maximum(zeros, 1) / (g - shared[cs]))
    assert shared.min() > 5.0                       # polluted rows are material
    assert np.median(est) > n + 4.0                 # Thm. 2 overcounts them
    assert abs(np.median(row_est) - n) < 1.0        # the row-aware count does not
    assert abs(np.mean(row_est) - n) < 1.0


# ---------------------------------------------------------------- restore

@pytest.mark.slow
@pytest.mark.parametrize("name,rule", [("default_g64", O.THR_THM2), ("nowrap_g64", O.THR_PAPER),
                                       ("ra4_va2", O.THR_THM2), ("ra2_va0", O.THR_THM2)])
def test_restore_equals_bruteforce_over_all_ipv4(name, rule):
    """Algs. 2 + 3 return exactly the IPs whose union column passes the
    threshold, found by testing all 2^32 addresses."""
    p = TINY_CONFIGS[name]
    theta = 16.0 if p["log2_g"] == 6 else 32.0
    t = tiny_trace(31 + len(name), n_hosts=3000, n_planted=30, fan_in=0.3)
    cube = O.cube_of(p, t.pairs, O.SIDE_SRC)
    got, st = O.restore(p, cube, theta, rule)
    want = O.restore_bruteforce(p, cube, theta, rule)
    assert st["cp_valid"] >= st["accepted"] == got.size
    assert got.size > 10
    assert np.array_equal(got, want)


def test_restore_output_sorted_unique_and_sound(small_window):
    p = default_params()
    cube = O.cube_of(p, small_window.pairs, O.SIDE_SRC)
    hosts, st = O.restore(p, cube, 1024.0)
    assert np.all(np.diff(hosts["ip"].astype(np.int64)) > 0)
    _, ones = O.column_zeros(p, cube)
    _, zmax = O.thresholds(p, ones, 1024.0)
    est, zeros, _ = O.estimate(p, cube, hosts["ip"])
    assert np.array_equal(zeros, hosts["zeros"])
    assert np.all(hosts["zeros"] <= zmax[hosts["cs"]])
    assert np.allclose(est, hosts["est"], rtol=0, atol=0)
    # every planted host (2k-20k peers, far above theta) is restored
    assert np.all(np.isin(small_window.planted_ips, hosts["ip"]))


def test_restore_empty_and_saturated():
    """An empty cube has no hot column; a host whose every column is full has
    Z = 0, is restored with the SATURATED flag and a finite estimate."""
    p = TINY_CONFIGS["ra4_va2"]
    hosts, st = O.restore(p, O.new_cube(p), 16.0)
    assert hosts.size == 0 and st["hot_columns"] == 0
    cube, cs = _cube_with_union_zeros(p, 0xC0A80001, 0)
    got, st = O.restore(p, cube, 16.0)
    assert got["ip"].tolist() == [0xC0A80001]
    assert got["flags"][0] == O.FLAG_SATURATED and got["zeros"][0] == 0
    assert np.isfinite(got["est"][0]) and got["est"][0] > 16.0


# ---------------------------------------------------------------- exact counts, rates

def test_exact_counts_vs_nested_loops():
    t = tiny_trace(41, n_hosts=300, n_planted=4, fan_in=0.5)
    for side in (0, 1):
        hosts, counts = O.exact_counts(t.pairs, side)
        ref = {}
        for s, d in t.pairs.tolist():
            h, q = (s, d) if side == 0 else (d, s)
            lst = ref.setdefault(h, [])
            if q not in lst:          # the list method of Sec. 3.1
                lst.append(q)
        assert hosts.tolist() == sorted(ref)
        assert counts.tolist() == [len(ref[h]) for h in sorted(ref)]


def test_generator_truth_matches_exact_counts():
    t = tracegen.window_core_edge(3, scale=1 / 256)
    hs, cs = O.exact_counts(t.pairs, 0)
    hd, cd = O.exact_counts(t.pairs, 1)
    src = dict(zip(hs.tolist(), cs.tolist()))
    dst = dict(zip(hd.tolist(), cd.tolist()))
    for ip, d, side in zip(t.planted_ips.tolist(), t.planted_deg.tolist(), t.planted_side.tolist()):
        assert (src if side == 0 else dst)[ip] == d
    for ip, d in zip(t.bg_ips.tolist(), t.bg_deg.tolist()):
        assert src[ip] == d


def test_construction_truth_is_exact():
    t = tracegen.window_core_edge(5, scale=1 / 512)
    for side in (0, 1):
        h, c = tracegen.construction_truth(t, side)
        order = np.argsort(h)
        hs, cs = O.exact_counts(t.pairs, side)
        assert np.array_equal(h[order], hs)
        assert np.array_equal(c[order], cs)


def test_detection_rates_definitions():
    """Sec. 5.2: FNR = |H minus detected| / |H|, FPR = |detected with fewer than
    theta peers| / |H| (both over |H|), FTR = FNR + FPR."""
    hosts = np.array([1, 2, 3, 4, 5], np.uint32)
    counts = np.array([10, 20, 30, 5, 1], np.uint32)
    r = O.detection_rates(np.array([2, 3, 4, 9], np.uint32), hosts, counts, 10)
    assert r["n_true"] == 3
    assert r["fnr"] == pytest.approx(1 / 3)     # host 1 missed
    assert r["fpr"] == pytest.approx(2 / 3)     # hosts 4 and 9 below theta
    assert r["ftr"] == pytest.approx(1.0)


# ---------------------------------------------------------------- thresholds at eps > 0

def test_threshold_closed_form_with_sharing():
    """Both rules at eps > 0 against values worked by hand (golden file):
    array fills are powers of two, so eps is exact and each floor is far from
    an integer boundary."""
    gold = _golden("threshold_eps_pos.json")
    for case in gold["cases"]:
        p = dict(default_params(), log2_g=case["log2_g"])
        g, A = 1 << p["log2_g"], p["n_ra"] + p["n_va"]
        S = 1 << p["r"]
        ones = np.array([[num * (1 << p["cbn"][a]) * g // den for a, (num, den)
                          in enumerate(case["fills"])]] * S, np.uint32).ravel()
        assert ones.size == S * A
        for rule, key in ((O.THR_THM2, "thm2"), (O.THR_PAPER, "paper")):
            eps, zmax = O.thresholds(p, ones, case["theta"], rule)
            assert np.all(eps == case["eps"]), (case, rule)
            assert np.all(zmax == case[key]), (case, rule, zmax[0])
        assert case["thm2"] == math.floor(case["thm2_real"])
        assert case["paper"] == math.floor(case["paper_real"])


def _filled_cube(p, fills, seed):
    """A cube whose array a has each bit set with probability fills[a]
    (a power of two: the AND of k random words has density 2^-k)."""
    rng = np.random.default_rng(seed)
    g, A, ncol, W, aoff = _layout(p)
    S, R = 1 << p["r"], g // 64
    cube = np.zeros((S, R, W), np.uint64)
    for a, f in enumerate(fills):
        k = int(round(-math.log2(f)))
        w = np.full((S, R, ncol[a]), np.uint64(0xFFFFFFFFFFFFFFFF))
        for _ in range(k):
            w &= rng.integers(0, 1 << 64, (S, R, ncol[a]), dtype=np.uint64)
        cube[:, :, aoff[a]:aoff[a] + ncol[a]] = w
    return cube.ravel()


def _set_host_union(p, cube, host, rows):
    """Overwrite every column of `host` with exactly the bits in `rows`, so
    its union column (Def. 2) is that set."""
    g, A, ncol, W, aoff = _layout(p)
    R = g // 64
    cs, cols = O.host_columns(p, host)
    words = np.zeros(R, np.uint64)
    for b in rows:
        words[b // 64] |= np.uint64(1) << np.uint64(b % 64)
    for a in range(A):
        for rb in range(R):
            cube[(cs * R + rb) * W + aoff[a] + cols[a]] = words[rb]
    return cs


SHARED_CFG = dict(default_params(), cbn=[10, 10, 10, 10], cl_bs=[4, 14, 24])


@pytest.mark.parametrize("fills", [(0.5, 0.5, 0.25, 0.25), (0.5, 0.5, 0.5, 0.5)])
def test_thm2_threshold_is_estimate_crossing_with_sharing(fills):
    """Thm. 2 at material sharing (eps = 1/64 and 1/16): for union columns
    with every zero count around the threshold, the Thm. 2 estimate reaches
    theta exactly when Z <= Zmax of rule THM2."""
    p = SHARED_CFG
    assert O.config_ok(p)
    g = 1 << p["log2_g"]
    theta = 1024.0
    cube = _filled_cube(p, fills, seed=5)
    host = 0x0A0B0C0D
    rng = np.random.default_rng(6)
    seen = set()
    zmax0 = int(math.floor((g - g * np.prod(fills)) * math.exp(-theta / g)))
    for z in range(zmax0 - 4, zmax0 + 5):
        rows = rng.choice(g, g - z, replace=False)
        cs = _set_host_union(p, cube, host, rows)
        _, ones = O.column_zeros(p, cube)
        eps, zmax = O.thresholds(p, ones, theta, O.THR_THM2)
        assert eps[cs] > 0.5 * np.prod(fills)
        est, zz, _ = O.estimate(p, cube, np.array([host], np.uint32))
        assert zz[0] == z
        assert (est[0] >= theta) == (z <= zmax[cs]), (z, zmax[cs], est[0])
        seen.add(bool(z <= zmax[cs]))
    assert seen == {True, False}


@pytest.mark.parametrize("fills", [(0.5, 0.5, 0.25, 0.25), (0.5, 0.5, 0.5, 0.5)])
def test_paper_threshold_is_crossing_of_its_correction(fills):
    """The printed threshold of Sec. 3.3, Z <= g(1+eps)e^{-theta/g} - g eps,
    says the same as -g ln((Z + g eps) / (g + g eps)) >= theta. Zmax of rule
    PAPER must sit exactly where that log form crosses theta."""
    p = SHARED_CFG
    g = 1 << p["log2_g"]
    cube = _filled_cube(p, fills, seed=7)
    _, ones = O.column_zeros(p, cube)
    for theta in (256.0, 1024.0, 2048.0):
        eps, zmax = O.thresholds(p, ones, theta, O.THR_PAPER)
        for cs in range(1 << p["r"]):
            e, zm = float(eps[cs]), int(zmax[cs])

            def corrected(z):
                return -g * math.log((z + g * e) / (g + g * e))

            assert e > 0.5 * np.prod(fills)
            assert corrected(zm) >= theta > corrected(zm + 1), (cs, theta, zm)


# ---------------------------------------------------------------- column statistics

@pytest.mark.parametrize("name", ["default_g64", "g128_r3", "ra4_va2", "hetero_r5"])
def test_column_zeros_by_unpacking_every_bit(name):
    """Per-column zero counts and per-array one counts (Alg. 2's inputs)
    against numpy unpacking every bit of the cube by the layout formula."""
    p = TINY_CONFIGS[name]
    g, A, ncol, W, aoff = _layout(p)
    S, R = 1 << p["r"], g // 64
    cube = O.cube_of(p, tiny_trace(17).pairs, O.SIDE_SRC)
    bits = np.unpackbits(cube.view(np.uint8), bitorder="little").reshape(S, R, W, 64)
    col_ones = bits.sum(axis=(1, 3))                      # [S, W]
    zeros, ones = O.column_zeros(p, cube)
    assert np.array_equal(zeros.reshape(S, W), g - col_ones)
    want_ones = np.stack([col_ones[:, aoff[a]:aoff[a] + ncol[a]].sum(axis=1) for a in range(A)], 1)
    assert np.array_equal(ones.reshape(S, A), want_ones)
    assert col_ones.max() > 0 and (g - col_ones).min() < g


def test_openmp_timing_legs_equal_the_plain_oracle():
    """The benchmark's multi-core CPU leg computes what the plain oracle does:
    the atomic-OR update gives the same cube bytes, the bucketed sort-unique
    the same (host, count) list, on a window with duplicates and both sides."""
    import tracegen
    p = default_params()
    t = tracegen.make_window(400_000, 40_000, 12, 1_000, 8_000, dup_frac=0.1, fan_in_frac=0.5,
                             seed=31)
    for side in (O.SIDE_SRC, O.SIDE_DST):
        want = O.cube_of(p, t.pairs, side)
        got = O.new_cube(p)
        O.update_omp(p, got, t.pairs, side)
        assert np.array_equal(got, want)
        h0, c0 = O.exact_counts(t.pairs, side)
        h1, c1 = O.exact_counts_omp(t.pairs, side)
        assert np.array_equal(h0, h1) and np.array_equal(c0, c1)
    # hosts that share a top byte, and a run of one host's repeated pairs
    pairs = np.array([[0x01000005, 9], [0x01000005, 9], [0x01000004, 9], [0x01FFFFFF, 1],
                      [0x01000004, 8], [0xFF000000, 2]], dtype=np.uint32)
    h, c = O.exact_counts_omp(pairs, O.SIDE_SRC)
    assert h.tolist() == [0x01000004, 0x01000005, 0x01FFFFFF, 0xFF000000]
    assert c.tolist() == [2, 1, 1, 1]
    assert O.omp_threads() >= 1
