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
