"""bench.py's command-line contract on the CPU: it runs on one GPU only and
says so for any other GPU count, before touching a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    assert "--workload" in r.stdout and "batched" in r.stdout


def test_detection_accuracy_matches_the_oracle_rates():
    """The benchmark's scoring of a restored list (Sec. 5.2) agrees with the
    oracle's definition of the rates on a window with misses, false hits and
    an address that never appears as a host."""
    import numpy as np

    import bench
    import oracle as O
    import tracegen
    t = tracegen.make_window(200_000, 20_000, 10, 600, 3_000, dup_frac=0.05, seed=4)
    hosts, counts = O.exact_counts(t.pairs, 0)
    theta = 1024
    rng = np.random.default_rng(2)
    big = hosts[counts >= theta]
    small = hosts[(counts < theta) & (counts > 100)]
    detected = np.concatenate([big[: max(1, big.size - 3)], small[:4],
                               np.array([0xDEADBEEF], np.uint32)])
    rng.shuffle(detected)
    est = np.full(detected.size, 1500.0)
    got = bench.detection_accuracy(detected, est, hosts, counts, theta)
    want = O.detection_rates(detected, hosts, counts, theta)
    for k in ("n_true", "fnr", "fpr", "ftr", "precision", "recall"):
        assert got[k] == want[k], k
    assert got["fnr"] > 0 and got["fpr"] > 0
    # the estimate's error is taken over the true super hosts restored
    c = dict(zip(hosts.tolist(), counts.tolist()))
    rel = [abs(1500.0 - c[h]) / c[h] for h in detected.tolist() if c.get(h, 0) >= theta]
    assert abs(got["est_rel_err_mean"] - float(np.mean(rel))) < 1e-12
