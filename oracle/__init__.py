"""CBAA oracle: ctypes wrapper over the plain C reference (cbaa_oracle.c).

TEST INFRASTRUCTURE ONLY: tests/, the smoke entry and the benchmark's CPU
baseline leg may import this package; the product path never does. It shares
no code with the HIP library.

Every function takes a plain dict of configuration parameters with the keys
``r, n_ra, n_va, log2_g, cbn, cl_bs, seed_mangle, seed_bv, seed_va``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbaa_oracle.c")
_LIB = os.path.join(_HERE, "libcbaa_oracle.so")

SIDE_SRC, SIDE_DST = 0, 1
THR_THM2, THR_PAPER = 0, 1
FLAG_SATURATED = 1


def build() -> str:
    """Compiles the oracle with gcc (fp contraction off so no FMA reorders roundings)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
           "-Wall", "-Wextra", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class RefConfig(C.Structure):
    _fields_ = [("r", C.c_uint32), ("n_ra", C.c_uint32), ("n_va", C.c_uint32),
                ("log2_g", C.c_uint32), ("cbn", C.c_uint32 * 6), ("cl_bs", C.c_uint32 * 4),
                ("seed_mangle", C.c_uint32), ("seed_bv", C.c_uint32), ("seed_va", C.c_uint32 * 2)]


class RefHost(C.Structure):
    _fields_ = [("ip", C.c_uint32), ("zeros", C.c_uint16), ("cs", C.c_uint8),
                ("flags", C.c_uint8), ("est", C.c_double)]


class RefStats(C.Structure):
    _fields_ = [("hot_columns", C.c_uint64), ("tuples", C.c_uint64), ("cp_valid", C.c_uint64),
                ("accepted", C.c_uint64)]


HOST_DTYPE = np.dtype([("ip", "<u4"), ("zeros", "<u2"), ("cs", "u1"), ("flags", "u1"),
                       ("est", "<f8")])

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    P = C.POINTER
    cfgp = P(RefConfig)
    u64p, u32p, u16p, u8p, f64p, i32p = (C.c_void_p,) * 6
    sig = {
        "ref_config_check": (C.c_int, [cfgp]),
        "ref_cube_words": (C.c_uint64, [cfgp]),
        "ref_mangle": (C.c_uint32, [cfgp, C.c_uint32]),
        "ref_unmangle": (C.c_uint32, [cfgp, C.c_uint32]),
        "ref_hash_bv": (C.c_uint32, [cfgp, C.c_uint32]),
        "ref_hash_va": (C.c_uint32, [cfgp, C.c_uint32, C.c_uint32]),
        "ref_host_columns": (None, [cfgp, C.c_uint32, u32p, u32p]),
        "ref_update": (None, [cfgp, u64p, u32p, C.c_uint64, C.c_int]),
        "ref_merge_or": (None, [cfgp, u64p, C.c_void_p, C.c_int]),
        "ref_column_zeros": (None, [cfgp, u64p, u16p, u32p]),
        "ref_thresholds": (None, [cfgp, u32p, C.c_double, C.c_int, f64p, i32p]),
        "ref_restore": (C.c_int, [cfgp, u64p, C.c_double, C.c_int, C.c_void_p, C.c_uint64,
                                  P(C.c_uint64), P(RefStats)]),
        "ref_restore_bruteforce": (C.c_int, [cfgp, u64p, C.c_double, C.c_int, C.c_void_p,
                                             C.c_uint64, P(C.c_uint64)]),
        "ref_estimate": (None, [cfgp, u64p, u32p, C.c_uint64, f64p, u16p, u8p]),
        "ref_host_layer_zeros": (None, [cfgp, u64p, u32p, C.c_uint64, u16p]),
        "ref_exact_counts": (C.c_uint64, [u32p, C.c_uint64, C.c_int, u32p, u32p]),
        "ref_exact_counts_omp": (C.c_uint64, [u32p, C.c_uint64, C.c_int, u32p, u32p]),
        "ref_update_omp": (None, [cfgp, u64p, u32p, C.c_uint64, C.c_int]),
        "ref_omp_threads": (C.c_int, []),
        "ref_row_ones": (None, [cfgp, u64p, u32p]),
        "ref_row_shared": (None, [cfgp, u32p, f64p]),
        "ref_check_mangle_bijection": (C.c_uint64, [cfgp]),
        "ref_check_lp_roundtrip": (C.c_uint64, [cfgp]),
        "ref_tuple_check": (C.c_int, [cfgp, u32p, P(C.c_uint32)]),
        "ref_ep_cp": (None, [cfgp, u32p, i32p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_params() -> dict:
    """The paper's evaluated dimensions (Sec. 5.3: r=4, |RA|=3, |VA|=1,
    g=c=2^12) with RA start bits (4, 14, 23) and fixed seeds."""
    return dict(r=4, n_ra=3, n_va=1, log2_g=12, cbn=[12, 12, 12, 12], cl_bs=[4, 14, 23],
                seed_mangle=0x243F6A88, seed_bv=0x85A308D3, seed_va=[0x13198A2E, 0x03707344])


def _cfg(p: dict) -> RefConfig:
    c = RefConfig()
    c.r, c.n_ra, c.n_va, c.log2_g = p["r"], p["n_ra"], p["n_va"], p["log2_g"]
    for i, v in enumerate(p["cbn"]):
        c.cbn[i] = v
    for i, v in enumerate(p["cl_bs"]):
        c.cl_bs[i] = v
    c.seed_mangle, c.seed_bv = p["seed_mangle"], p["seed_bv"]
    for i, v in enumerate(p["seed_va"]):
        c.seed_va[i] = v
    if _load().ref_config_check(C.byref(c)) != 0:
        raise ValueError(f"oracle rejects configuration {p}")
    return c


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def config_ok(p: dict) -> bool:
    try:
        _cfg(p)
        return True
    except ValueError:
        return False


def cube_words(p: dict) -> int:
    return int(_load().ref_cube_words(C.byref(_cfg(p))))


def new_cube(p: dict) -> np.ndarray:
    return np.zeros(cube_words(p), dtype=np.uint64)


def mangle(p: dict, ip: int) -> int:
    return int(_load().ref_mangle(C.byref(_cfg(p)), ip))


def unmangle(p: dict, m: int) -> int:
    return int(_load().ref_unmangle(C.byref(_cfg(p)), m))


def hash_bv(p: dict, oip: int) -> int:
    return int(_load().ref_hash_bv(C.byref(_cfg(p)), oip))


def hash_va(p: dict, j: int, lp: int) -> int:
    return int(_load().ref_hash_va(C.byref(_cfg(p)), j, lp))


def host_columns(p: dict, iip: int) -> tuple[int, list[int]]:
    cs = np.zeros(1, np.uint32)
    cols = np.zeros(6, np.uint32)
    _load().ref_host_columns(C.byref(_cfg(p)), iip, _ptr(cs), _ptr(cols))
    return int(cs[0]), [int(x) for x in cols[: p["n_ra"] + p["n_va"]]]


def update(p: dict, cube: np.ndarray, pairs: np.ndarray, side: int) -> None:
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32)
    assert cube.dtype == np.uint64 and cube.size == cube_words(p)
    _load().ref_update(C.byref(_cfg(p)), _ptr(cube), _ptr(pairs), pairs.shape[0], side)


def cube_of(p: dict, pairs: np.ndarray, side: int) -> np.ndarray:
    cube = new_cube(p)
    update(p, cube, pairs, side)
    return cube


def update_omp(p: dict, cube: np.ndarray, pairs: np.ndarray, side: int) -> None:
    """update() split over all host cores with atomic ORs (a timing leg)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32)
    assert cube.dtype == np.uint64 and cube.size == cube_words(p)
    _load().ref_update_omp(C.byref(_cfg(p)), _ptr(cube), _ptr(pairs), pairs.shape[0], side)


def omp_threads() -> int:
    return int(_load().ref_omp_threads())


def merge_or(p: dict, cubes: list[np.ndarray]) -> np.ndarray:
    dst = new_cube(p)
    arr = (C.c_void_p * len(cubes))(*[_ptr(c) for c in cubes])
    _load().ref_merge_or(C.byref(_cfg(p)), _ptr(dst), arr, len(cubes))
    return dst


def column_zeros(p: dict, cube: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    S = 1 << p["r"]
    A = p["n_ra"] + p["n_va"]
    W = sum(1 << p["cbn"][a] for a in range(A))
    zeros = np.zeros(S * W, np.uint16)
    ones = np.zeros(S * A, np.uint32)
    _load().ref_column_zeros(C.byref(_cfg(p)), _ptr(cube), _ptr(zeros), _ptr(ones))
    return zeros, ones


def row_ones(p: dict, cube: np.ndarray) -> np.ndarray:
    """uint32 [2^r, |RA|+|VA|, g]: columns of each array with each bit set."""
    S, A, g = 1 << p["r"], p["n_ra"] + p["n_va"], 1 << p["log2_g"]
    out = np.zeros(S * A * g, np.uint32)
    _load().ref_row_ones(C.byref(_cfg(p)), _ptr(cube), _ptr(out))
    return out.reshape(S, A, g)


def row_shared(p: dict, rows: np.ndarray) -> np.ndarray:
    """fp64 [2^r]: sum over rows of the product over arrays of row fill."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.zeros(1 << p["r"], np.float64)
    _load().ref_row_shared(C.byref(_cfg(p)), _ptr(rows), _ptr(out))
    return out


def thresholds(p: dict, ones: np.ndarray, theta: float, rule: int = THR_THM2):
    S = 1 << p["r"]
    ones = np.ascontiguousarray(ones, dtype=np.uint32)
    eps = np.zeros(S, np.float64)
    zmax = np.zeros(S, np.int32)
    _load().ref_thresholds(C.byref(_cfg(p)), _ptr(ones), float(theta), rule, _ptr(eps), _ptr(zmax))
    return eps, zmax


def restore(p: dict, cube: np.ndarray, theta: float, rule: int = THR_THM2, cap: int = 1 << 20):
    """Literal Alg. 2 + Alg. 3; returns (hosts sorted by ip, stats dict)."""
    out = np.zeros(cap, HOST_DTYPE)
    n = C.c_uint64(0)
    st = RefStats()
    rc = _load().ref_restore(C.byref(_cfg(p)), _ptr(cube), float(theta), rule, _ptr(out), cap,
                             C.byref(n), C.byref(st))
    if rc != 0:
        raise OverflowError(f"{n.value} hosts exceed capacity {cap}")
    stats = dict(hot_columns=st.hot_columns, tuples=st.tuples, cp_valid=st.cp_valid,
                 accepted=st.accepted)
    return out[: n.value].copy(), stats


def restore_bruteforce(p: dict, cube: np.ndarray, theta: float, rule: int = THR_THM2,
                       cap: int = 1 << 20) -> np.ndarray:
    """Every IP of the 2^32 space whose union column passes the threshold."""
    out = np.zeros(cap, HOST_DTYPE)
    n = C.c_uint64(0)
    rc = _load().ref_restore_bruteforce(C.byref(_cfg(p)), _ptr(cube), float(theta), rule,
                                        _ptr(out), cap, C.byref(n))
    if rc != 0:
        raise OverflowError(f"{n.value} hosts exceed capacity {cap}")
    return out[: n.value].copy()


def estimate(p: dict, cube: np.ndarray, hosts: np.ndarray):
    hosts = np.ascontiguousarray(hosts, dtype=np.uint32)
    n = hosts.size
    est = np.zeros(n, np.float64)
    zeros = np.zeros(n, np.uint16)
    flags = np.zeros(n, np.uint8)
    _load().ref_estimate(C.byref(_cfg(p)), _ptr(cube), _ptr(hosts), n, _ptr(est), _ptr(zeros),
                         _ptr(flags))
    return est, zeros, flags


def host_layer_zeros(p: dict, cube: np.ndarray, hosts: np.ndarray) -> np.ndarray:
    hosts = np.ascontiguousarray(hosts, dtype=np.uint32)
    A = p["n_ra"] + p["n_va"]
    out = np.zeros((hosts.size, A), np.uint16)
    _load().ref_host_layer_zeros(C.byref(_cfg(p)), _ptr(cube), _ptr(hosts), hosts.size, _ptr(out))
    return out


def exact_counts(pairs: np.ndarray, side: int) -> tuple[np.ndarray, np.ndarray]:
    """Exact |OP(h)| for every host (sort-unique); hosts ascending."""
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32)
    n = pairs.shape[0]
    hosts = np.zeros(max(n, 1), np.uint32)
    counts = np.zeros(max(n, 1), np.uint32)
    nh = _load().ref_exact_counts(_ptr(pairs), n, side, _ptr(hosts), _ptr(counts))
    return hosts[:nh].copy(), counts[:nh].copy()


def exact_counts_omp(pairs: np.ndarray, side: int) -> tuple[np.ndarray, np.ndarray]:
    """exact_counts() over all host cores (bucketed by the host's top byte)."""
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32)
    n = pairs.shape[0]
    hosts = np.zeros(max(n, 1), np.uint32)
    counts = np.zeros(max(n, 1), np.uint32)
    nh = _load().ref_exact_counts_omp(_ptr(pairs), n, side, _ptr(hosts), _ptr(counts))
    return hosts[:nh].copy(), counts[:nh].copy()


def check_mangle_bijection(p: dict) -> int:
    return int(_load().ref_check_mangle_bijection(C.byref(_cfg(p))))


def check_lp_roundtrip(p: dict) -> int:
    return int(_load().ref_check_lp_roundtrip(C.byref(_cfg(p))))


def tuple_check(p: dict, t: list[int]):
    arr = np.zeros(4, np.uint32)
    arr[: len(t)] = t
    lp = C.c_uint32(0)
    ok = _load().ref_tuple_check(C.byref(_cfg(p)), _ptr(arr), C.byref(lp))
    return (int(lp.value) if ok else None)


def ep_cp(p: dict) -> tuple[list[int], list[int]]:
    ep = np.zeros(4, np.uint32)
    cp = np.zeros(4, np.int32)
    _load().ref_ep_cp(C.byref(_cfg(p)), _ptr(ep), _ptr(cp))
    n = p["n_ra"]
    return [int(x) for x in ep[:n]], [int(x) for x in cp[:n]]


def detection_rates(detected: np.ndarray, hosts: np.ndarray, counts: np.ndarray,
                    theta: float) -> dict:
    """FNR and FPR of Sec. 5.2 (both over |H|), FTR = FPR + FNR, plus the
    conventional precision and recall. A detected host with fewer than theta
    peers (or never seen) is a false positive."""
    truth = dict(zip(hosts.tolist(), counts.tolist()))
    H = {h for h, c in truth.items() if c >= theta}
    D = set(int(x) for x in detected)
    fn = H - D
    fp = {h for h in D if truth.get(h, 0) < theta}
    nH = max(len(H), 1)
    return dict(n_true=len(H), n_detected=len(D), fnr=len(fn) / nH, fpr=len(fp) / nH,
                ftr=(len(fn) + len(fp)) / nH,
                precision=(len(D) - len(fp)) / max(len(D), 1), recall=(len(H) - len(fn)) / nH)
