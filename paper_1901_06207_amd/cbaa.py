"""Python binding of libcbaa (ctypes). Argument marshalling only: every step of
the detector runs in the library's HIP kernels; PyTorch provides device
memory and streams.

The functions named ``cbaa_*`` mirror the C ABI of ``include/cbaa.h`` one to
one (tensors in place of device pointers, ``stream=None`` meaning torch's
current stream). A few conveniences (``new_cube``, ``restore``, ``estimate``)
allocate buffers with torch and call those.

Loading fails loudly when the built library is missing: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbaa.so")

CBAA_OK, CBAA_EINVAL, CBAA_ECONFIG, CBAA_ESCRATCH, CBAA_EHIP = 0, -1, -2, -3, -4
SIDE_SRC, SIDE_DST = 0, 1
THR_THM2, THR_PAPER = 0, 1
FLAG_SATURATED = 1
STATUS_CONFIG, STATUS_BUDGET = 1, 2
MAX_RA, MAX_VA = 4, 2
HEADER_BYTES = 256
HEADER_WORDS = HEADER_BYTES // 8
CUBE_MAGIC = 0x4542554341414243
CUBE_VALID, CUBE_MIXED = 0, 1
DEFAULT_MAX_CHECKS = 1 << 28
STATS_FIELDS = ("n_hosts", "hot_columns", "partial_checked", "tuples_checked", "tuple_space",
                "status")


class CbaaError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class cbaa_config(C.Structure):
    _fields_ = [("r", C.c_uint32), ("n_ra", C.c_uint32), ("n_va", C.c_uint32),
                ("log2_g", C.c_uint32), ("cbn", C.c_uint32 * 6), ("cl_bs", C.c_uint32 * 4),
                ("seed_mangle", C.c_uint32), ("seed_bv", C.c_uint32),
                ("seed_va", C.c_uint32 * 2)]


class cbaa_restore_stats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in STATS_FIELDS]


STATS_BYTES = C.sizeof(cbaa_restore_stats)


class cbaa_stream_batch(C.Structure):
    _fields_ = [("d_pairs", C.c_void_p), ("n_pairs", C.c_uint64), ("d_cube", C.c_void_p),
                ("d_cube_dst", C.c_void_p), ("side", C.c_int), ("flags", C.c_int)]


class cbaa_tuning(C.Structure):
    _fields_ = [("chunk_pairs", C.c_uint32), ("seg_records", C.c_uint32),
                ("apply_blocks", C.c_uint32), ("reserved", C.c_uint32)]


NOALLOC_SCRATCH_BYTES = 64 << 20
MAX_BATCH = 32

HOST_DTYPE = np.dtype([("ip", "<u4"), ("zeros", "<u2"), ("cs", "u1"), ("flags", "u1"),
                       ("est", "<f8")])
HOST_BYTES = 16


@dataclasses.dataclass(frozen=True)
class Config:
    """Detector configuration (fields of cbaa_config)."""

    r: int = 4
    n_ra: int = 3
    n_va: int = 1
    log2_g: int = 12
    cbn: tuple = (12, 12, 12, 12)
    cl_bs: tuple = (4, 14, 23)
    seed_mangle: int = 0x243F6A88
    seed_bv: int = 0x85A308D3
    seed_va: tuple = (0x13198A2E, 0x03707344)

    @classmethod
    def from_dict(cls, p: dict) -> "Config":
        return cls(r=p["r"], n_ra=p["n_ra"], n_va=p["n_va"], log2_g=p["log2_g"],
                   cbn=tuple(p["cbn"]), cl_bs=tuple(p["cl_bs"]), seed_mangle=p["seed_mangle"],
                   seed_bv=p["seed_bv"], seed_va=tuple(p["seed_va"]))

    def to_c(self) -> cbaa_config:
        c = cbaa_config()
        c.r, c.n_ra, c.n_va, c.log2_g = self.r, self.n_ra, self.n_va, self.log2_g
        for i, v in enumerate(self.cbn):
            c.cbn[i] = v
        for i, v in enumerate(self.cl_bs):
            c.cl_bs[i] = v
        c.seed_mangle, c.seed_bv = self.seed_mangle, self.seed_bv
        for i, v in enumerate(self.seed_va):
            c.seed_va[i] = v
        return c

    @property
    def n_arrays(self) -> int:
        return self.n_ra + self.n_va

    @property
    def g(self) -> int:
        return 1 << self.log2_g

    @property
    def n_sketches(self) -> int:
        return 1 << self.r

    @property
    def slab_words(self) -> int:
        return sum(1 << self.cbn[a] for a in range(self.n_arrays))


_lib = None


def lib():
    """The loaded libcbaa; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcbaa.so not built at {LIB_PATH}: run "
                          "python -m paper_1901_06207_amd.build_lib")
    L = C.CDLL(LIB_PATH)
    cfgp = C.POINTER(cbaa_config)
    vp, u64, i32, dbl = C.c_void_p, C.c_uint64, C.c_int, C.c_double
    sig = {
        "cbaa_abi_version": (C.c_uint32, []),
        "cbaa_config_default": (i32, [cfgp]),
        "cbaa_config_validate": (i32, [cfgp]),
        "cbaa_cube_bytes": (u64, [cfgp]),
        "cbaa_config_hash": (u64, [cfgp]),
        "cbaa_cube_check": (i32, [cfgp, vp, vp]),
        "cbaa_update_scratch_bytes": (u64, [cfgp, u64, i32]),
        "cbaa_restore_scratch_bytes": (u64, [cfgp, u64]),
        "cbaa_cube_init": (i32, [cfgp, vp, vp]),
        "cbaa_update": (i32, [cfgp, vp, vp, u64, i32, vp, u64, vp]),
        "cbaa_update2": (i32, [cfgp, vp, vp, vp, u64, vp, u64, vp]),
        "cbaa_merge_or": (i32, [cfgp, vp, C.POINTER(vp), i32, vp]),
        "cbaa_update_batch_scratch_bytes": (u64, [cfgp, C.POINTER(cbaa_stream_batch), i32,
                                                  C.POINTER(cbaa_tuning)]),
        "cbaa_update_batch": (i32, [cfgp, C.POINTER(cbaa_stream_batch), i32,
                                    C.POINTER(cbaa_tuning), vp, u64, vp]),
        "cbaa_column_zeros": (i32, [cfgp, vp, vp, vp, vp]),
        "cbaa_restore": (i32, [cfgp, vp, dbl, i32, u64, vp, u64, vp, u64, vp, vp]),
        "cbaa_estimate": (i32, [cfgp, vp, vp, u64, vp, vp, vp, vp, u64, vp]),
        "cbaa_merge_restore": (i32, [cfgp, vp, C.POINTER(vp), i32, dbl, i32, u64, vp, u64, vp, u64,
                                     vp, vp]),
        "cbaa_merge_scan": (i32, [cfgp, vp, C.POINTER(vp), i32, dbl, i32, u64, vp, u64, vp, u64,
                                  vp, vp]),
        "cbaa_restore_scanned": (i32, [cfgp, vp, C.POINTER(vp), i32, dbl, i32, u64, vp, u64, vp,
                                       u64, vp, vp]),
        "cbaa_merge_restore_noalloc": (i32, [cfgp, vp, C.POINTER(vp), i32, dbl, i32, u64, vp, u64,
                                             vp, vp]),
        "cbaa_mlp_param_count": (C.c_uint32, [C.c_uint32]),
        "cbaa_mlp_init": (i32, [C.c_uint32, C.c_uint32, i32, vp, vp, vp]),
        "cbaa_mlp_features": (i32, [cfgp, vp, vp, u64, C.c_uint32, vp, vp, u64, vp]),
        "cbaa_mlp_forward": (i32, [C.c_uint32, vp, vp, vp, u64, vp, vp]),
        "cbaa_mlp_loss_grad": (i32, [C.c_uint32, vp, vp, vp, vp, u64, vp, vp, vp]),
        "cbaa_mlp_adam": (i32, [C.c_uint32, vp, vp, vp, vp, vp, C.c_uint32, C.c_float,
                                C.c_float, C.c_float, C.c_float, vp]),
        "cbaa_probe_copy": (i32, [vp, vp, u64, C.c_uint32, C.c_uint32, vp]),
        "cbaa_probe_addresses": (i32, [vp, u64, C.c_uint32, C.c_uint32, vp]),
        "cbaa_probe_atomic_or": (i32, [vp, u64, vp, u64, vp]),
        "cbaa_strerror": (C.c_char_p, [i32]),
        "cbaa_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, where: str) -> None:
    if rc != CBAA_OK:
        L = lib()
        raise CbaaError(rc, where, f"{L.cbaa_strerror(rc).decode()}: {L.cbaa_last_error().decode()}")


def _cfg(cfg) -> cbaa_config:
    if isinstance(cfg, cbaa_config):
        return cfg
    if isinstance(cfg, dict):
        cfg = Config.from_dict(cfg)
    return cfg.to_c()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev_ptr(t: Optional[torch.Tensor], name: str, min_bytes: int = 0) -> Optional[int]:
    """Device address of a contiguous tensor holding at least min_bytes."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    nbytes = t.numel() * t.element_size()
    if nbytes < min_bytes:
        raise ValueError(f"{name} holds {nbytes} bytes, the call needs {min_bytes}")
    return t.data_ptr()


def _cube_ptr(cfg, t: Optional[torch.Tensor], name: str) -> Optional[int]:
    return _dev_ptr(t, name, cbaa_cube_bytes(cfg))


# ---- C ABI, one to one ------------------------------------------------------

def cbaa_abi_version() -> int:
    return int(lib().cbaa_abi_version())


def cbaa_config_default() -> Config:
    c = cbaa_config()
    _check(lib().cbaa_config_default(C.byref(c)), "cbaa_config_default")
    return Config(r=c.r, n_ra=c.n_ra, n_va=c.n_va, log2_g=c.log2_g, cbn=tuple(c.cbn)[:4],
                  cl_bs=tuple(c.cl_bs)[:3], seed_mangle=c.seed_mangle, seed_bv=c.seed_bv,
                  seed_va=tuple(c.seed_va))


def cbaa_config_validate(cfg) -> int:
    return int(lib().cbaa_config_validate(C.byref(_cfg(cfg))))


def cbaa_last_error() -> str:
    return lib().cbaa_last_error().decode()


def cbaa_cube_bytes(cfg) -> int:
    return int(lib().cbaa_cube_bytes(C.byref(_cfg(cfg))))


def cbaa_config_hash(cfg) -> int:
    return int(lib().cbaa_config_hash(C.byref(_cfg(cfg))))


def cbaa_cube_check(cfg, cube: torch.Tensor, stream=None) -> int:
    """CBAA_OK, or CBAA_ECONFIG when the cube lacks this configuration's valid
    header (returned, not raised; synchronises the stream)."""
    rc = int(lib().cbaa_cube_check(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"),
                                   _stream(stream)))
    if rc not in (CBAA_OK, CBAA_ECONFIG):
        _check(rc, "cbaa_cube_check")
    return rc


def cbaa_update_scratch_bytes(cfg, n_pairs: int, n_cubes: int) -> int:
    return int(lib().cbaa_update_scratch_bytes(C.byref(_cfg(cfg)), n_pairs, n_cubes))


def cbaa_restore_scratch_bytes(cfg, capacity: int) -> int:
    return int(lib().cbaa_restore_scratch_bytes(C.byref(_cfg(cfg)), capacity))


def cbaa_cube_init(cfg, cube: torch.Tensor, stream=None) -> None:
    _check(lib().cbaa_cube_init(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"), _stream(stream)),
           "cbaa_cube_init")


def _pairs_ptr(pairs: torch.Tensor) -> tuple[Optional[int], int]:
    if pairs.element_size() != 4 or pairs.dim() != 2 or pairs.shape[1] != 2:
        raise ValueError("pairs must be a [N, 2] tensor of 32-bit integers")
    n = int(pairs.shape[0])
    return (_dev_ptr(pairs, "pairs") if n else None), n


def cbaa_update(cfg, cube: torch.Tensor, pairs: torch.Tensor, side: int,
                scratch: Optional[torch.Tensor] = None, stream=None) -> None:
    p, n = _pairs_ptr(pairs)
    sb = scratch.numel() * scratch.element_size() if scratch is not None else 0
    _check(lib().cbaa_update(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"), p, n, side,
                             _dev_ptr(scratch, "scratch"), sb, _stream(stream)), "cbaa_update")


def cbaa_update2(cfg, cube_src: torch.Tensor, cube_dst: torch.Tensor, pairs: torch.Tensor,
                 scratch: Optional[torch.Tensor] = None, stream=None) -> None:
    p, n = _pairs_ptr(pairs)
    sb = scratch.numel() * scratch.element_size() if scratch is not None else 0
    _check(lib().cbaa_update2(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube_src, "cube_src"),
                              _cube_ptr(cfg, cube_dst, "cube_dst"), p, n, _dev_ptr(scratch, "scratch"),
                              sb, _stream(stream)), "cbaa_update2")


BATCH_FRESH = 1


def _stream_table(cfg, streams):
    """streams: sequence of (pairs, cube, cube_dst or None, side[, flags])."""
    arr = (cbaa_stream_batch * len(streams))()
    for i, entry in enumerate(streams):
        pairs, cube, cube_dst, side = entry[:4]
        arr[i].flags = entry[4] if len(entry) > 4 else 0
        p, n = _pairs_ptr(pairs)
        arr[i].d_pairs = p
        arr[i].n_pairs = n
        arr[i].d_cube = _cube_ptr(cfg, cube, "cube")
        arr[i].d_cube_dst = _cube_ptr(cfg, cube_dst, "cube_dst")
        arr[i].side = side
    return arr


def _tuning(t) -> Optional[cbaa_tuning]:
    if t is None:
        return None
    if isinstance(t, cbaa_tuning):
        return t
    return cbaa_tuning(int(t.get("chunk_pairs", 0)), int(t.get("seg_records", 0)),
                       int(t.get("apply_blocks", 0)), 0)


def cbaa_update_batch_scratch_bytes(cfg, streams, tuning=None) -> int:
    t = _tuning(tuning)
    return int(lib().cbaa_update_batch_scratch_bytes(C.byref(_cfg(cfg)), _stream_table(cfg, streams),
                                                     len(streams), C.byref(t) if t else None))


def cbaa_update_batch(cfg, streams, scratch: torch.Tensor, tuning=None, stream=None) -> None:
    t = _tuning(tuning)
    sb = scratch.numel() * scratch.element_size()
    _check(lib().cbaa_update_batch(C.byref(_cfg(cfg)), _stream_table(cfg, streams), len(streams),
                                   C.byref(t) if t else None, _dev_ptr(scratch, "scratch"), sb,
                                   _stream(stream)), "cbaa_update_batch")


def cbaa_merge_or(cfg, dst: torch.Tensor, srcs: Sequence[torch.Tensor], stream=None) -> None:
    if dst is None:
        raise ValueError("cbaa_merge_or needs a destination cube")
    arr = (C.c_void_p * len(srcs))(*[_cube_ptr(cfg, s, "src") for s in srcs])
    _check(lib().cbaa_merge_or(C.byref(_cfg(cfg)), _cube_ptr(cfg, dst, "dst"), arr, len(srcs),
                               _stream(stream)), "cbaa_merge_or")


def cbaa_column_zeros(cfg, cube: torch.Tensor, zeros: torch.Tensor, ones: torch.Tensor,
                      stream=None) -> None:
    c = Config.from_dict(cfg) if isinstance(cfg, dict) else cfg
    _check(lib().cbaa_column_zeros(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"),
                                   _dev_ptr(zeros, "zeros", 2 * c.n_sketches * c.slab_words),
                                   _dev_ptr(ones, "ones", 4 * c.n_sketches * c.n_arrays),
                                   _stream(stream)), "cbaa_column_zeros")


def cbaa_restore(cfg, cube: torch.Tensor, theta: float, rule: int, scratch: torch.Tensor,
                 out: Optional[torch.Tensor], capacity: int, stats: torch.Tensor,
                 stream=None, max_checks: int = 0) -> None:
    sb = scratch.numel() * scratch.element_size()
    _check(lib().cbaa_restore(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"), float(theta), rule,
                              max_checks, _dev_ptr(scratch, "scratch"), sb,
                              _dev_ptr(out, "out", capacity * HOST_BYTES) if capacity else None,
                              capacity, _dev_ptr(stats, "stats", STATS_BYTES), _stream(stream)),
           "cbaa_restore")


def cbaa_merge_restore(cfg, dst: Optional[torch.Tensor], srcs: Sequence[torch.Tensor],
                       theta: float, rule: int, scratch: torch.Tensor, out: Optional[torch.Tensor],
                       capacity: int, stats: torch.Tensor, stream=None,
                       max_checks: int = 0) -> None:
    """dst None: the merged cube is not stored (at most 16 sources)."""
    arr = (C.c_void_p * len(srcs))(*[_cube_ptr(cfg, x, "src") for x in srcs])
    sb = scratch.numel() * scratch.element_size()
    _check(lib().cbaa_merge_restore(C.byref(_cfg(cfg)),
                                    _cube_ptr(cfg, dst, "dst") if dst is not None else None,
                                    arr, len(srcs),
                                    float(theta), rule, max_checks, _dev_ptr(scratch, "scratch"),
                                    sb,
                                    _dev_ptr(out, "out", capacity * HOST_BYTES) if capacity
                                    else None, capacity,
                                    _dev_ptr(stats, "stats", STATS_BYTES), _stream(stream)),
           "cbaa_merge_restore")


def _merge_phase(name, cfg, dst, srcs, theta, rule, scratch, out, capacity, stats, stream,
                 max_checks):
    arr = (C.c_void_p * len(srcs))(*[_cube_ptr(cfg, x, "src") for x in srcs])
    sb = scratch.numel() * scratch.element_size()
    _check(getattr(lib(), name)(C.byref(_cfg(cfg)),
                                _cube_ptr(cfg, dst, "dst") if dst is not None else None,
                                arr, len(srcs), float(theta), rule, max_checks,
                                _dev_ptr(scratch, "scratch"), sb,
                                _dev_ptr(out, "out", capacity * HOST_BYTES) if capacity else None,
                                capacity, _dev_ptr(stats, "stats", STATS_BYTES), _stream(stream)),
           name)


def cbaa_merge_scan(cfg, dst: Optional[torch.Tensor], srcs: Sequence[torch.Tensor],
                    theta: float, rule: int, scratch: torch.Tensor, out: Optional[torch.Tensor],
                    capacity: int, stats: torch.Tensor, stream=None, max_checks: int = 0) -> None:
    """First half of cbaa_merge_restore (merge and column scan)."""
    _merge_phase("cbaa_merge_scan", cfg, dst, srcs, theta, rule, scratch, out, capacity, stats,
                 stream, max_checks)


def cbaa_restore_scanned(cfg, dst: Optional[torch.Tensor], srcs: Sequence[torch.Tensor],
                         theta: float, rule: int, scratch: torch.Tensor,
                         out: Optional[torch.Tensor], capacity: int, stats: torch.Tensor,
                         stream=None, max_checks: int = 0) -> None:
    """Second half of cbaa_merge_restore, with the same arguments as the first."""
    _merge_phase("cbaa_restore_scanned", cfg, dst, srcs, theta, rule, scratch, out, capacity,
                 stats, stream, max_checks)


def cbaa_merge_restore_noalloc(cfg, dst: Optional[torch.Tensor], srcs: Sequence[torch.Tensor],
                               theta: float, rule: int, out: Optional[torch.Tensor],
                               capacity: int, stats: torch.Tensor, stream=None,
                               max_checks: int = 0) -> None:
    """cbaa_merge_restore on the library's own per-device scratch array."""
    arr = (C.c_void_p * len(srcs))(*[_cube_ptr(cfg, x, "src") for x in srcs])
    _check(lib().cbaa_merge_restore_noalloc(
        C.byref(_cfg(cfg)), _cube_ptr(cfg, dst, "dst") if dst is not None else None, arr,
        len(srcs), float(theta), rule, max_checks,
        _dev_ptr(out, "out", capacity * HOST_BYTES) if capacity else None, capacity,
        _dev_ptr(stats, "stats", STATS_BYTES), _stream(stream)),
        "cbaa_merge_restore_noalloc")


def cbaa_estimate(cfg, cube: torch.Tensor, hosts: torch.Tensor, est: torch.Tensor,
                  zeros: torch.Tensor, layer_zeros: Optional[torch.Tensor],
                  scratch: torch.Tensor, stream=None) -> None:
    n = int(hosts.numel())
    sb = scratch.numel() * scratch.element_size()
    A = (Config.from_dict(cfg) if isinstance(cfg, dict) else cfg).n_arrays
    _check(lib().cbaa_estimate(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"),
                               _dev_ptr(hosts, "hosts", 4 * n) if n else None, n,
                               _dev_ptr(est, "est", 8 * n) if n else None,
                               _dev_ptr(zeros, "zeros", 2 * n) if n else None,
                               _dev_ptr(layer_zeros, "layer_zeros", 2 * n * A) if n else None,
                               _dev_ptr(scratch, "scratch"), sb, _stream(stream)),
           "cbaa_estimate")


# ---- measurement probes (include/cbaa_probe.h) ---------------------------------

PROBE_NONTEMPORAL = 1


def cbaa_probe_copy(dst: torch.Tensor, src: torch.Tensor, nbytes: int, blocks: int = 0,
                    flags: int = 0, stream=None) -> None:
    _check(lib().cbaa_probe_copy(_dev_ptr(dst, "dst", nbytes), _dev_ptr(src, "src", nbytes),
                                 nbytes, blocks, flags, _stream(stream)), "cbaa_probe_copy")


def cbaa_probe_addresses(addr: torch.Tensor, log2_words: int, seed: int, stream=None) -> None:
    n = int(addr.numel())
    _check(lib().cbaa_probe_addresses(_dev_ptr(addr, "addr", 4 * n), n, log2_words, seed,
                                      _stream(stream)), "cbaa_probe_addresses")


def cbaa_probe_atomic_or(buf: torch.Tensor, addr: torch.Tensor, stream=None) -> None:
    words = buf.numel() * buf.element_size() // 4
    n = int(addr.numel())
    _check(lib().cbaa_probe_atomic_or(_dev_ptr(buf, "buf", 4 * words), words,
                                      _dev_ptr(addr, "addr", 4 * n), n, _stream(stream)),
           "cbaa_probe_atomic_or")


# ---- learned estimator (include/cbaa_mlp.h) ------------------------------------

def cbaa_mlp_param_count(n_features: int) -> int:
    return int(lib().cbaa_mlp_param_count(n_features))


def cbaa_mlp_init(n_features: int, seed: int, master: torch.Tensor, wbf: torch.Tensor,
                  zero_output: bool = False, stream=None) -> None:
    _check(lib().cbaa_mlp_init(n_features, seed, int(zero_output), _dev_ptr(master, "master"),
                               _dev_ptr(wbf, "wbf"), _stream(stream)), "cbaa_mlp_init")


def cbaa_mlp_features(cfg, cube: torch.Tensor, hosts: torch.Tensor, n_features: int,
                      x: torch.Tensor, scratch: torch.Tensor, stream=None) -> None:
    n = int(hosts.numel())
    sb = scratch.numel() * scratch.element_size()
    _check(lib().cbaa_mlp_features(C.byref(_cfg(cfg)), _cube_ptr(cfg, cube, "cube"),
                                   _dev_ptr(hosts, "hosts", 4 * n) if n else None, n, n_features,
                                   _dev_ptr(x, "x", 4 * n * n_features) if n else None,
                                   _dev_ptr(scratch, "scratch"),
                                   sb, _stream(stream)), "cbaa_mlp_features")


def cbaa_mlp_forward(n_features: int, master: torch.Tensor, wbf: torch.Tensor, x: torch.Tensor,
                     y: torch.Tensor, stream=None) -> None:
    n = int(y.numel())
    _check(lib().cbaa_mlp_forward(n_features, _dev_ptr(master, "master"), _dev_ptr(wbf, "wbf"),
                                  _dev_ptr(x, "x") if n else None, n,
                                  _dev_ptr(y, "y") if n else None, _stream(stream)),
           "cbaa_mlp_forward")


def cbaa_mlp_loss_grad(n_features: int, master: torch.Tensor, wbf: torch.Tensor, x: torch.Tensor,
                       t: torch.Tensor, grad: torch.Tensor, loss: torch.Tensor,
                       stream=None) -> None:
    _check(lib().cbaa_mlp_loss_grad(n_features, _dev_ptr(master, "master"), _dev_ptr(wbf, "wbf"),
                                    _dev_ptr(x, "x"), _dev_ptr(t, "t"), int(t.numel()),
                                    _dev_ptr(grad, "grad"), _dev_ptr(loss, "loss"),
                                    _stream(stream)), "cbaa_mlp_loss_grad")


def cbaa_mlp_adam(n_features: int, master: torch.Tensor, wbf: torch.Tensor, grad: torch.Tensor,
                  m: torch.Tensor, v: torch.Tensor, step: int, lr: float, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(lib().cbaa_mlp_adam(n_features, _dev_ptr(master, "master"), _dev_ptr(wbf, "wbf"),
                               _dev_ptr(grad, "grad"), _dev_ptr(m, "m"), _dev_ptr(v, "v"), step,
                               lr, beta1, beta2, eps, _stream(stream)), "cbaa_mlp_adam")


# ---- conveniences (torch allocation around the calls above) -------------------

def new_cube(cfg, device="cuda", init: bool = True, stream=None) -> torch.Tensor:
    nbytes = cbaa_cube_bytes(cfg)
    if nbytes == 0:
        _check(CBAA_ECONFIG, "new_cube")
    cube = torch.empty(nbytes // 8, dtype=torch.int64, device=device)
    if init:
        cbaa_cube_init(cfg, cube, stream)
    return cube


def scratch_tensor(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def stats_tensor(device="cuda") -> torch.Tensor:
    return torch.zeros(len(STATS_FIELDS), dtype=torch.int64, device=device)


def stats_dict(st: torch.Tensor) -> dict:
    """A cbaa_restore_stats tensor (read back to the host) as a dict."""
    return dict(zip(STATS_FIELDS, (int(v) for v in st.cpu().tolist())))


def host_list(out: torch.Tensor, n: int) -> np.ndarray:
    raw = out[: n * HOST_BYTES].cpu().numpy()
    return raw.view(HOST_DTYPE).copy()


def restore(cfg, cube: torch.Tensor, theta: float, rule: int = THR_THM2, capacity: int = 1 << 16,
            stream=None, max_checks: int = 0) -> tuple[np.ndarray, dict]:
    """Restores the super hosts of `cube`; grows the output until it fits.
    Returns (structured array sorted by ip, stats dict)."""
    dev = cube.device
    while True:
        scratch = scratch_tensor(cbaa_restore_scratch_bytes(cfg, capacity), dev)
        out = torch.empty(max(capacity, 1) * HOST_BYTES, dtype=torch.uint8, device=dev)
        st = stats_tensor(dev)
        cbaa_restore(cfg, cube, theta, rule, scratch, out, capacity, st, stream,
                     max_checks=max_checks)
        torch.cuda.synchronize(dev)
        stats = stats_dict(st)
        n = stats["n_hosts"]
        if n <= capacity:
            return host_list(out, n), stats
        capacity = n


def estimate(cfg, cube: torch.Tensor, hosts: np.ndarray, layers: bool = False, stream=None):
    """Thm. 2 estimates for inner IPs: (est float64, zeros uint16[, layer zeros])."""
    dev = cube.device
    n = int(len(hosts))
    A = Config.from_dict(cfg).n_arrays if isinstance(cfg, dict) else cfg.n_arrays
    h = torch.from_numpy(np.ascontiguousarray(hosts, dtype=np.uint32).view(np.int32)).to(dev)
    est = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    zeros = torch.empty(max(n, 1), dtype=torch.int16, device=dev)
    lz = torch.empty(max(n, 1) * A, dtype=torch.int16, device=dev) if layers else None
    scratch = scratch_tensor(cbaa_restore_scratch_bytes(cfg, 0), dev)
    cbaa_estimate(cfg, cube, h, est, zeros, lz, scratch, stream)
    torch.cuda.synchronize(dev)
    res = (est[:n].cpu().numpy(), zeros[:n].cpu().numpy().view(np.uint16))
    if layers:
        res = res + (lz[: n * A].cpu().numpy().view(np.uint16).reshape(n, A),)
    return res


def pairs_to_device(pairs: np.ndarray, device="cuda") -> torch.Tensor:
    """uint32 [N, 2] host pairs -> int32 [N, 2] device tensor (same bits)."""
    a = np.ascontiguousarray(pairs, dtype=np.uint32).view(np.int32)
    return torch.from_numpy(a).to(device)


def cube_to_numpy(cube: torch.Tensor) -> np.ndarray:
    """The cube's bits (the words after its header) as uint64."""
    return cube.cpu().numpy().view(np.uint64)[HEADER_WORDS:]


def cube_header(cube: torch.Tensor) -> np.ndarray:
    """The cube's header: 32 uint64 words."""
    return cube[:HEADER_WORDS].cpu().numpy().view(np.uint64)


def cube_from_bits(cfg, bits: np.ndarray, device="cuda") -> torch.Tensor:
    """A device cube with a valid header of `cfg` holding the given bits."""
    cube = new_cube(cfg, device)
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    if b.size != cube.numel() - HEADER_WORDS:
        raise ValueError(f"{b.size} words of bits, the configuration's cube holds "
                         f"{cube.numel() - HEADER_WORDS}")
    cube[HEADER_WORDS:].copy_(torch.from_numpy(b.view(np.int64)))
    return cube
