"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

Nothing here computes any part of the generator: this module only draws
the parameters of workloads (instance tables, request traces) from numpy's
PCG64 stream.  Both the CPU oracle and the GPU path read their instances
from these functions, so they always see the same inputs.
"""
from __future__ import annotations

import numpy as np

BATCH_SEED = 0x5EED


def batch_instances(count: int = 4096, seed: int = BATCH_SEED):
    """The batched workload: `count` independent plain BA graphs.

    n is log-uniform on [10^3, 10^7] (rounded, clamped), d uniform on 1..32,
    and the hash seed of instance j is j.  Mean n = (10^7 - 10^3) / (4 ln 10)
    = 1.086e6 and mean d = 16.5, so the expected total is 7.3e10 edges
    (587 GB of uint32 pairs), more than one GPU's HBM: it runs in rounds.
    Returns (n uint64[count], d uint32[count], seed uint64[count]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(count)
    n = np.clip(np.rint(10.0 ** (3.0 + 4.0 * u)), 1e3, 1e7).astype(np.uint64)
    d = (1 + rng.integers(0, 32, size=count)).astype(np.uint32)
    s = np.arange(count, dtype=np.uint64)
    return n, d, s


SERVED_SEED = 0x5E4FED


def served_trace(count: int = 4000, rate: float = 2000.0, seed: int = SERVED_SEED, n_lo: float = 1e4,
                 n_hi: float = 1e8, big_frac: float = 0.02):
    """The served workload: `count` requests with Poisson arrivals at `rate`
    per second.  A fraction big_frac asks for the n=2^27, d=16 graph; the
    rest have n log-uniform on [n_lo, n_hi] and d uniform on {2,4,...,64}.
    Half the requests want the whole edge list, half the streamed degrees
    of the first min(10^5, n) nodes.  The hash seed of request j is j.
    Returns a dict of numpy arrays: arrival_s, n, d, seed, kind (0 edges,
    1 degrees), first_k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=count))
    u = rng.random(count)
    n = np.clip(np.rint(10.0 ** (np.log10(n_lo) + (np.log10(n_hi) - np.log10(n_lo)) * u)), n_lo, n_hi)
    n = n.astype(np.uint64)
    d = (2 ** rng.integers(1, 7, size=count)).astype(np.uint32)
    big = rng.random(count) < big_frac
    n[big] = 1 << 27
    d[big] = 16
    kind = (rng.random(count) < 0.5).astype(np.uint32)
    first_k = np.where(kind == 1, np.minimum(n, 100000), 0).astype(np.uint64)
    return {"arrival_s": arrival, "n": n, "d": d, "seed": np.arange(count, dtype=np.uint64), "kind": kind,
            "first_k": first_k}


SEED_GRAPH_SEED = 0x5EED6

def seed_graph(n0: int = 100, m0: int = 1000, seed: int = SEED_GRAPH_SEED):
    """The seed graph of the generalized-model workload: m0 edges between
    nodes 0..n0-1, both endpoints uniform (a random multigraph, loops
    allowed), as the 2*m0 node IDs of positions 0..2*m0-1 (uint32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n0, size=2 * m0).astype(np.uint32)
