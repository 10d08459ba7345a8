"""The seeded workload inputs are what the frozen tables say they are."""
import json
import os

import numpy as np

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_batch_instances_match_frozen_table():
    n, d, s = workloads.batch_instances()
    ref = json.load(open(os.path.join(GOLDEN, "batch_instances_4096.json")))
    assert n.tolist() == ref["n"] and d.tolist() == ref["d"] and s.tolist() == ref["seed"]


def test_batch_instances_distribution():
    n, d, s = workloads.batch_instances()
    assert n.dtype == np.uint64 and d.dtype == np.uint32 and s.dtype == np.uint64
    assert n.min() >= 1000 and n.max() <= 10**7 and d.min() >= 1 and d.max() <= 32
    assert s.tolist() == list(range(4096))
    # log-uniform n: mean (10^7 - 10^3) / (4 ln 10) = 1.086e6; uniform d: mean 16.5
    assert abs(n.mean() / 1.0856e6 - 1) < 0.15 and abs(d.mean() - 16.5) < 0.6
    logn = np.log10(n.astype(np.float64))
    assert abs(np.mean(logn) - 5.0) < 0.05
