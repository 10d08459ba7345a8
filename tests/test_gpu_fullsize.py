"""GPU parity at the full sizes of the two workloads, in the launch
configuration bench.py times.

* Stored graph n=2^26, d=16, seed=7 (2^30 edges): every edge and every degree
  against the sequential Batagelj-Brandes oracle (about 30 s of CPU), bit-exact.
* Streamed degrees n=2^30, d=64, seed=42 (2^36 edges, 64-bit positions): (a)
  the degrees of the first 10^5 nodes and the checksum over all 2^36 edges
  against the oracle's per-edge recomputation over the same edges, run on
  every granted host core in disjoint ranges (about a minute), bit-exact;
  (b) invariance under splitting the edges into shuffled ranges; (c) the
  mean-field degree law E[deg v] ~ d*sqrt(n/v) and deg >= d.
* The same streaming workload at the reduced n=2^24 (2^30 edges), whole.
"""
import random
import sys

import numpy as np
import pytest

import oracle
from tests import oracle_par

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1602_07106_amd as ba  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ba.lib()
    yield
    torch.cuda.synchronize()


def test_headline_graph_every_edge_and_degree():
    n, d, seed = 1 << 26, 16, 7
    m = n * d
    _say("stored graph, full size", n, d, seed)
    out = torch.empty((m, 2), dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = ba.workspace(n, d, m)
    ba.generate(n, d, seed, degrees=True, out=out, deg_out=deg, ws=ws)  # the call bench.py times
    plain = torch.empty_like(out)
    ba.generate(n, d, seed, out=plain)  # the chain kernel without the target list
    torch.cuda.synchronize()
    assert torch.equal(out, plain)
    del plain, ws
    _say("oracle: sequential Batagelj-Brandes over 2^30 edges")
    E, calls = oracle.bb_generate(n, d, seed)
    assert calls == m  # BB draws one position per edge
    flat = out.view(-1)
    step = 1 << 27
    for s in range(0, 2 * m, step):
        got = flat[s:s + step].cpu().numpy().view(np.uint32)
        if not np.array_equal(got, E[s:s + step]):
            j = int(np.flatnonzero(got != E[s:s + step])[0])
            pytest.fail("edge array differs first at position %d" % (s + j))
    ref = oracle.count_degrees(E, n)
    del E
    got = deg.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref.astype(np.uint32))
    assert int(got.astype(np.uint64).sum()) == 2 * m


def test_streaming_workload_full_size():
    n, d, seed, k = 1 << 30, 64, 42, 100000
    m = n * d
    _say("streamed degrees, full size", n, d, seed, k)
    deg, cs = ba.degrees(n, d, seed, k)
    full = deg.cpu().numpy().view(np.uint64).copy()

    # (b) the same edges in shuffled ranges of ragged sizes
    cuts = sorted(random.Random(11).sample(range(1, m), 6))
    bounds = list(zip([0] + cuts, cuts + [m]))
    random.Random(12).shuffle(bounds)
    acc = torch.zeros(k, dtype=torch.int64, device="cuda")
    acc_cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    for b, e in bounds:
        ba.degrees_range(n, d, seed, b, e - b, k, acc, acc_cs)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy().view(np.uint64), full)
    assert int(acc_cs.item()) & ((1 << 64) - 1) == cs

    # (a) every edge: the oracle's stream over all 2^36 edges, on all granted host cores
    _say("oracle stream over all", m, "edges on", oracle_par.THREADS, "threads")
    rdeg, rcs = oracle_par.stream(d, seed, 0, m, k)
    assert np.array_equal(full, rdeg)
    assert cs == rcs

    # (c) properties at full size: every node has its d own edges, and the
    # mean-field BA law E[deg v] = d sqrt(n/v) holds on average over v
    assert (full >= d).all()
    v = np.arange(1000, k)
    ratio = full[1000:].astype(np.float64) / (d * np.sqrt(n / v))
    assert abs(ratio.mean() - 1.0) < 0.05


def test_streaming_workload_reduced_n_whole():
    # the streaming workload at n = 2^24 (same d and seed): 2^30 edges, all
    # compared, on the LDS tier the automatic choice takes (64K) and the other
    n, d, seed, k = 1 << 24, 64, 42, 100000
    m = n * d
    _say("streamed degrees, reduced n", n, d, seed, k)
    rdeg, rcs = oracle_par.stream(d, seed, 0, m, k)
    for tier in (ba.TIER_AUTO, ba.TIER_16K):
        deg, cs = ba.degrees(n, d, seed, k, tier=tier)
        torch.cuda.synchronize()
        assert np.array_equal(deg.cpu().numpy().view(np.uint64), rdeg), tier
        assert cs == rcs, tier
