"""Pins of the oracle's graph semantics against the paper and the mathematics.

* Brute force: for every choice function on tiny inputs, sequential
  Batagelj-Brandes (paper Section 2) equals the per-edge chain of figure
  generateEdge.  This is the exactness argument of the method, checked on all
  cases rather than assumed.
* Exact rationals: Batagelj-Brandes with uniform choices has the distribution
  of the preferential-attachment process of Section 1 (target chosen with
  probability proportional to its current degree).
* Cross-language: a literal big-integer Python transcription of generateEdge
  with the same hash equals the C oracle.
* Special cases, invariants (second endpoint <= first, degree sum 2m, degree
  >= d, prefix stability), the expected chain length of Section 2 (at most 2)
  and the power-law degree tail of the Barabasi-Albert model.
"""
import itertools
import math
import random
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1


# ---------------------------------------------------------------- brute force


def _chain(c, i, d):
    """generateEdge with an arbitrary choice function c (odd position -> 0..p-1)."""
    r = 2 * i + 1
    while True:
        r = c[r]
        if r % 2 == 0:
            return i // d, r // (2 * d)


@pytest.mark.parametrize("n,d", [(1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (1, 3), (2, 2), (3, 2), (2, 3), (1, 6)])
def test_bb_equals_chain_for_every_choice_function(n, d):
    m = n * d
    odd = list(range(1, 2 * m, 2))
    count = 0
    for choice in itertools.product(*[range(p) for p in odd]):
        c = dict(zip(odd, choice))
        x = [c[2 * i + 1] for i in range(m)]
        E = oracle.bb_with_choices(n, d, x)
        for i in range(m):
            assert (int(E[2 * i]), int(E[2 * i + 1])) == _chain(c, i, d)
        count += 1
    assert count == math.prod(odd)


@pytest.mark.parametrize("n,d", [(3, 2), (6, 1), (2, 3), (4, 1)])
def test_bb_distribution_is_preferential_attachment(n, d):
    m = n * d
    # Batagelj-Brandes: x_i uniform on 0..2i, all sequences equally likely.
    total = math.prod(2 * i + 1 for i in range(m))
    bb = Counter()
    for x in itertools.product(*[range(2 * i + 1) for i in range(m)]):
        E = oracle.bb_with_choices(n, d, list(x))
        bb[tuple(int(v) for v in E[1::2])] += 1
    bb = {k: Fraction(c, total) for k, c in bb.items()}
    # Preferential attachment: node t is chosen with probability deg(t)/(2i+1),
    # degrees counted over the 2i+1 endpoints placed so far (including the new
    # edge's own source, so self-loops are allowed).
    pa = {}
    for vs in itertools.product(*[range(i // d + 1) for i in range(m)]):
        deg = Counter()
        p = Fraction(1)
        for i, v in enumerate(vs):
            deg[i // d] += 1
            p *= Fraction(deg[v], 2 * i + 1)
            if p == 0:
                break
            deg[v] += 1
        if p:
            pa[vs] = p
    assert bb == pa
    assert sum(pa.values()) == 1


# ---------------------------------------------------------- cross-language


def _py_fmix64(z):
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def _py_generate_edge(i, d, seed):
    key = (seed * 0x9E3779B97F4A7C15) & M64
    r = 2 * i + 1
    while True:
        r = (_py_fmix64(r ^ key) * r) >> 64
        if r % 2 == 0:
            return i // d, r // (2 * d)


@pytest.mark.parametrize("n,d,seed", [(1000, 1, 0), (250, 4, 1), (100, 7, 3), (40, 25, 123456789), (16, 64, M64)])
def test_literal_python_generate_edge_equals_c_oracle(n, d, seed):
    E, _ = oracle.bb_generate(n, d, seed)
    for i in range(n * d):
        assert _py_generate_edge(i, d, seed) == (int(E[2 * i]), int(E[2 * i + 1]))


@pytest.mark.parametrize("n,d,seed", [(100000, 4, 1), (4096, 16, 7), (3000, 33, 42), (777, 1, 5), (1, 64, 9)])
def test_per_edge_definition_equals_batagelj_brandes(n, d, seed):
    E, calls_bb = oracle.bb_generate(n, d, seed)
    m = n * d
    assert calls_bb == m
    out, calls = oracle.edges_range(d, seed, 0, m)
    assert np.array_equal(out.astype(np.uint32), E)
    assert calls >= m


def test_large_positions_match_big_integers():
    # 64-bit positions beyond 2^32: the oracle's single-edge path vs big ints
    rng = random.Random(3)
    for _ in range(300):
        d = rng.choice([1, 3, 16, 64])
        i = rng.getrandbits(rng.choice([33, 36, 40, 50]))
        seed = rng.getrandbits(64)
        u, v, _ = oracle.edge(d, seed, i)
        assert (u, v) == _py_generate_edge(i, d, seed)


# ---------------------------------------------------------- special cases


def test_edge_zero_is_a_self_loop_on_node_zero_for_every_seed():
    for seed in list(range(50)) + [M64, 1 << 63]:
        assert oracle.edge(4, seed, 0)[:2] == (0, 0)


def test_first_d_edges_are_self_loops_on_node_zero():
    for d in [1, 2, 5, 16, 64]:
        E, _ = oracle.bb_generate(3, d, 17)
        assert np.all(E[: 2 * d] == 0)


def test_single_node_has_degree_2d():
    for d in [1, 4, 16]:
        E, _ = oracle.bb_generate(1, d, 5)
        assert oracle.count_degrees(E, 1).tolist() == [2 * d]


def test_d_equals_one_sources_are_edge_ids():
    E, _ = oracle.bb_generate(5000, 1, 8)
    assert np.array_equal(E[0::2], np.arange(5000, dtype=np.uint32))


# -------------------------------------------------------------- invariants


@pytest.mark.parametrize("n,d,seed", [(100000, 4, 1), (20000, 16, 7), (5000, 3, 0)])
def test_invariants(n, d, seed):
    E, _ = oracle.bb_generate(n, d, seed)
    u, v = E[0::2].astype(np.int64), E[1::2].astype(np.int64)
    assert np.all(v <= u)
    assert np.array_equal(u, np.arange(n * d) // d)
    deg = oracle.count_degrees(E, n)
    assert int(deg.sum()) == 2 * n * d
    assert np.all(deg >= d)


def test_prefix_stability():
    d, seed = 8, 99
    big, _ = oracle.bb_generate(30000, d, seed)
    for n in [1, 7, 1000, 29999]:
        small, _ = oracle.bb_generate(n, d, seed)
        assert np.array_equal(small, big[: 2 * n * d])


def test_streaming_consumer_agrees_with_stored_array():
    n, d, seed, k = 20000, 5, 3, 1000
    E, _ = oracle.bb_generate(n, d, seed)
    deg_all = oracle.count_degrees(E, n)
    cs_all = oracle.checksum_E(E)
    # whole range in one go
    deg_k, cs, _ = oracle.stream(d, seed, 0, n * d, k)
    assert np.array_equal(deg_k, deg_all[:k])
    assert cs == cs_all
    # in ragged chunks
    deg_k2 = np.zeros(k, dtype=np.uint64)
    cs2, i = 0, 0
    for c in [1, 999, 12345, 7, n * d]:
        c = min(c, n * d - i)
        deg_k2, cs2, _ = oracle.stream(d, seed, i, c, k, deg_k2, cs2)
        i += c
    assert i == n * d
    assert np.array_equal(deg_k2, deg_all[:k]) and cs2 == cs_all


# -------------------------------------------------------- chain statistics


def _ideal_mean_chain_length(m):
    # a(r) = expected hash evaluations from odd position r with h(r) uniform on
    # 0..r-1: a(r) = 1 + (1/r) * sum_{odd s < r} a(s).  Returns mean over r=2i+1.
    s = 0.0
    tot = 0.0
    for i in range(m):
        r = 2 * i + 1
        a = 1.0 + s / r
        tot += a
        s += a
    return tot / m


def test_expected_chain_length_is_about_two():
    # Under one fixed hash, chains that reach the same odd position share the
    # rest of their walk, so the per-graph mean is noisier than sqrt(2/m);
    # average over independent seeds and use their observed spread.
    m = 400000
    expected = _ideal_mean_chain_length(m)
    assert 1.99 < expected < 2.0  # Section 2: bounded by sum 2^-i = 2
    means = np.array([oracle.edges_range(4, s, 0, m)[1] / m for s in range(32)])
    assert np.all(np.abs(means - 2.0) < 0.05)
    sem = means.std(ddof=1) / math.sqrt(means.size)
    assert abs(means.mean() - expected) < 5 * sem


def test_degree_distribution_has_the_barabasi_albert_power_law_tail():
    n, d = 100000, 4
    E, _ = oracle.bb_generate(n, d, 1)
    deg = oracle.count_degrees(E, n).astype(np.float64)
    # mean-field: E[deg v] ~ d * sqrt(n / v)
    v = np.arange(1, 1001)
    ratio = np.mean(deg[1:1001] / (d * np.sqrt(n / v)))
    assert 0.93 < ratio < 1.07
    # CCDF(k) ~ (d/k)^2: log-log slope near -2 over k in [8, 256]
    ks = np.unique(np.round(np.logspace(np.log10(8), np.log10(256), 20)))
    ccdf = np.array([np.mean(deg >= k) for k in ks])
    slope = np.polyfit(np.log(ks), np.log(ccdf), 1)[0]
    assert -2.3 < slope < -1.7
