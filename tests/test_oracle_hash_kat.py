"""Known-answer pins of the oracle's mixers against their published
definitions, from models written here that share nothing with the oracle:

* the mangling M(x) = fmix32(x ^ seed) (Sec. 3.1 asks for an invertible
  mangling): fmix32 is the finalizer of MurmurHash3_x86_32. A Python model
  of the whole hash is first checked against the hash's published test
  vectors (tests/golden/murmur3_x86_32.json); its finalizer then gives the
  expected mangling of random addresses.
* H_bv and H_j (Alg. 1, Sec. 3.2 "random hash functions") take the top bits
  of lowbias32(x ^ seed) from C. Wellons' hash-prospector. The same source
  publishes the exact inverse of lowbias32 with its own constants; applying
  that inverse to a chosen output y gives the input whose hash must start
  with y's top bits.
"""

import json
import os

import numpy as np

import oracle as O
from conftest import GOLDEN, default_params

M32 = 0xFFFFFFFF


def _rotl(x, r):
    return ((x << r) | (x >> (32 - r))) & M32


def _fmix32(h):
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & M32
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & M32
    h ^= h >> 16
    return h


def _murmur3_x86_32(data: bytes, seed: int) -> int:
    c1, c2 = 0xCC9E2D51, 0x1B873593
    h = seed
    nb = len(data) // 4
    for i in range(nb):
        k = int.from_bytes(data[4 * i:4 * i + 4], "little")
        k = _rotl((k * c1) & M32, 15)
        h ^= (k * c2) & M32
        h = (_rotl(h, 13) * 5 + 0xE6546B64) & M32
    tail = data[4 * nb:]
    if tail:
        k = int.from_bytes(tail, "little")
        k = _rotl((k * c1) & M32, 15)
        h ^= (k * c2) & M32
    h ^= len(data)
    return _fmix32(h)


def _lowbias32_inverse(x):
    # the inverse published next to lowbias32 (hash-prospector)
    x ^= x >> 16
    x = (x * 0x43021123) & M32
    x ^= (x >> 15) ^ (x >> 30)
    x = (x * 0x1D69E2A5) & M32
    x ^= x >> 16
    return x


def test_model_reproduces_published_murmur3_vectors():
    with open(os.path.join(GOLDEN, "murmur3_x86_32.json")) as f:
        vec = json.load(f)["vectors"]
    assert len(vec) >= 16
    for v in vec:
        assert _murmur3_x86_32(bytes.fromhex(v["hex"]), v["seed"]) == v["hash"], v


def test_mangle_is_fmix32_of_address_xor_seed():
    p = dict(default_params(), seed_mangle=0)
    # empty-input vectors: the whole hash is fmix32(seed)
    assert O.mangle(p, 1) == 0x514E28B7
    assert O.mangle(p, 0xFFFFFFFF) == 0x81F16F39
    rng = np.random.default_rng(7)
    xs = rng.integers(0, 1 << 32, 4000, dtype=np.uint64).tolist()
    q = default_params()
    for x in xs:
        assert O.mangle(p, x) == _fmix32(x)
        assert O.mangle(q, x) == _fmix32(x ^ q["seed_mangle"])
        assert O.unmangle(q, _fmix32(x ^ q["seed_mangle"])) == x


def test_bit_and_va_hashes_are_top_bits_of_lowbias32():
    """For outputs y chosen at random, the published inverse gives the input
    x with lowbias32(x) = y; the oracle's H_bv(x ^ seed_bv) must then be the
    top log2_g bits of y and H_j(x ^ seed_va[j]) the top cbn bits."""
    rng = np.random.default_rng(8)
    ys = rng.integers(0, 1 << 32, 4000, dtype=np.uint64).tolist()
    for log2_g in (6, 12, 15):
        p = dict(default_params(), log2_g=log2_g)
        for y in ys[:1500]:
            x = _lowbias32_inverse(y)
            assert O.hash_bv(p, x ^ p["seed_bv"]) == y >> (32 - log2_g)
    p = dict(default_params(), n_va=2, cbn=[12, 12, 12, 16, 9])
    for j, bits in ((0, 16), (1, 9)):
        for y in ys:
            lp = _lowbias32_inverse(y) ^ p["seed_va"][j]
            assert O.hash_va(p, j, lp) == y >> (32 - bits)
