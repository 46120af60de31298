import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU case (exhaustive or full-size)")


def default_params() -> dict:
    """Paper-default dimensions (Sec. 5.3) with the library's default offsets and seeds."""
    return dict(r=4, n_ra=3, n_va=1, log2_g=12, cbn=[12, 12, 12, 12], cl_bs=[4, 14, 23],
                seed_mangle=0x243F6A88, seed_bv=0x85A308D3, seed_va=[0x13198A2E, 0x03707344])


def tiny_params(**kw) -> dict:
    """g = 64 (one 64-bit word per column) variants for brute-force cases."""
    p = default_params()
    p["log2_g"] = 6
    p.update(kw)
    return p


# Small configurations exercising every structural option the library accepts.
TINY_CONFIGS = {
    "default_g64": tiny_params(),
    "nowrap_g64": tiny_params(cl_bs=[4, 12, 20], cbn=[12, 12, 12, 12]),
    "ra2_va0": tiny_params(r=6, n_ra=2, n_va=0, cbn=[14, 14, 0, 0], cl_bs=[6, 19]),
    "ra4_va2": tiny_params(n_ra=4, n_va=2, cbn=[8, 8, 8, 8, 10, 9], cl_bs=[4, 11, 18, 25]),
    "hetero_r5": tiny_params(r=5, n_ra=3, n_va=1, cbn=[11, 10, 10, 9], cl_bs=[5, 14, 23]),
    "g128_r3": tiny_params(r=3, log2_g=7, cbn=[11, 11, 11, 10], cl_bs=[3, 13, 22]),
}


def tiny_trace(seed: int, n_hosts: int = 3000, n_planted: int = 30, lo: int = 20, hi: int = 120,
               fan_in: float = 0.0):
    import tracegen
    n_bg = 3 * n_hosts
    rng = np.random.default_rng(seed)
    pdeg_mean = (hi - lo) / max(np.log(hi / lo), 1e-9)
    n_packets = int(n_bg + n_planted * pdeg_mean * 1.5) + 200
    return tracegen.make_window(n_packets, n_hosts, n_planted, lo, hi, dup_frac=0.05, zipf_s=1.1,
                                fan_in_frac=fan_in, seed=int(rng.integers(1, 1 << 30)))


@pytest.fixture(scope="session")
def small_window():
    import tracegen
    return tracegen.window_small(1)
