"""The threaded oracle helper used by the full-size GPU parity tests gives
exactly the sequential oracle's results (ragged piece boundaries, a range
that does not start at 0, positions beyond 2^32)."""
import numpy as np

import oracle
from tests import oracle_par


def test_threaded_edges_equal_one_sequential_call():
    for d, seed, b, c in [(7, 5, 12345, 5_000_003), (64, 42, (1 << 31) + 11, 4_194_305)]:
        ref, _ = oracle.edges_range(d, seed, b, c)
        assert np.array_equal(oracle_par.edges_u32(d, seed, b, c), ref.astype(np.uint32))


def test_threaded_stream_equals_one_sequential_call():
    for d, seed, b, c, k in [(64, 42, 3, 10_000_001, 100000), (16, 7, (1 << 33) + 5, 3_000_017, 700)]:
        deg, cs = oracle_par.stream(d, seed, b, c, k)
        rdeg, rcs, _ = oracle.stream(d, seed, b, c, k)
        assert np.array_equal(deg, rdeg) and cs == rcs
