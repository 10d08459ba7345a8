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


def test_served_trace_shape():
    t = workloads.served_trace()
    n, d, kind = t["n"], t["d"], t["kind"]
    assert len(n) == 4000 and np.all(np.diff(t["arrival_s"]) > 0)
    rate = len(n) / t["arrival_s"][-1]
    assert 1800 < rate < 2200  # Poisson arrivals at 2000/s
    big = (n == (1 << 27)) & (d == 16)
    assert 0.01 < big.mean() < 0.03
    assert set(np.unique(d).tolist()) <= {2, 4, 8, 16, 32, 64}
    assert n.min() >= 10**4 and n[~big].max() <= 10**8
    assert 0.45 < kind.mean() < 0.55
    assert np.all(t["first_k"][kind == 1] == np.minimum(n[kind == 1], 100000))
    assert np.all(t["first_k"][kind == 0] == 0)
    assert t["seed"].tolist() == list(range(4000))
    # offered load: mean edges per request x rate, about 5e11 edges/s
    offered = float((n.astype(np.float64) * d).mean()) * rate
    assert 3e11 < offered < 8e11


def test_seed_graph_is_seeded_and_in_range():
    a = workloads.seed_graph(100, 1000)
    b = workloads.seed_graph(100, 1000)
    assert a.dtype == np.uint32 and a.size == 2000
    assert np.array_equal(a, b)
    assert a.max() < 100 and len(np.unique(a)) == 100
    assert not np.array_equal(a, workloads.seed_graph(100, 1000, seed=1))
