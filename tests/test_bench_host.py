"""CPU: the benchmark's host logic. It refuses more than one GPU, its distribution-free
interval for the median is the binomial one, its comparison with the oracle's stored
caps catches a single changed word, and the HBM traffic it reports for the dominant
kernels comes from counter runs taken on the kernel sources in the tree."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n", [6, 10, 20, 51])
def test_median_interval_is_the_binomial_order_statistic_interval(n):
    x = np.random.default_rng(n).permutation(np.arange(n, dtype=np.float64))  # order statistic k is k - 1
    lo, hi = bench.median_ci95(x)
    # the interval [x_(j), x_(n+1-j)] with j the largest index for which P(B < j) <= 2.5 %,
    # B ~ binomial(n, 1/2): counted here from the definition
    p_below = lambda j: sum(math.comb(n, i) for i in range(j)) / 2 ** n  # P(B <= j - 1)
    j = max(k for k in range(1, n // 2 + 1) if p_below(k) <= 0.025)
    assert (lo, hi) == (float(j - 1), float(n - j))
    assert p_below(j) <= 0.025 < p_below(j + 1)
    assert lo <= np.median(x) <= hi


def test_median_interval_needs_six_samples():
    assert bench.median_ci95([1.0, 2.0, 3.0, 4.0, 5.0]) is None


def _stored_caps(name):
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        return [np.array([[int(w, 16) for w in row] for row in e["cap"]], dtype=np.uint64)
                for e in json.load(f)["entries"]]


def test_golden_check_matches_stored_caps_and_catches_one_changed_word():
    caps = _stored_caps("caps_135x2p20.json")
    assert bench.golden_check("commit-135x2^20", caps)["bit_exact"] is True
    bad = [c.copy() for c in caps]
    bad[0][3, 2] ^= np.uint64(1)
    r = bench.golden_check("commit-135x2^20", bad)
    assert r["bit_exact"] is False and r["matched"] == 0
    batch = _stored_caps("caps_batch64.json")
    assert bench.golden_check("commit-batch-64", batch)["matched"] == 64
    assert bench.golden_check("commit-batch-64", batch[:-1])["matched"] == 0  # count mismatch
    assert bench.golden_check("open-8192", caps)["golden"] is None


@pytest.mark.parametrize("workload", ["commit-135x2^20", "commit-80x2^18"])
def test_recorded_traffic_belongs_to_the_current_kernel_sources(workload):
    """profiles/traffic.json holds the calibrated FETCH_SIZE + WRITE_SIZE of the leaf
    kernel and the LDE passes, each with a digest of the sources it was measured on; a
    kernel changed since then must be profiled again (the benchmark reports null)."""
    leaf = bench._traffic_record("k_leaf_hash_mf", workload)
    assert leaf is not None, "k_leaf_hash_mf changed since its counters were taken"
    assert bench.measured_lde_traffic(workload) is not None, "an LDE pass changed since its counters were taken"
    alg = {"commit-135x2^20": (135 << 23) * 8 + (1 << 23) * 32, "commit-80x2^18": (80 << 21) * 8 + (1 << 21) * 32}
    assert 0.99 < leaf["hbm_bytes_per_dispatch"] / alg[workload] < 1.05
