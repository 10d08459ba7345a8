"""Pins of the oracle's generalized model (paper Section "Generalizations":
a seed graph in front of the edge array, and self-loop-free draws) and of
the paper's CRC-based hash.  Each pin ties the oracle to something other
than itself: published CRC-32C vectors, an independent table-driven CRC,
the plain model (already pinned) as the special case n0 = m0 = 0, brute
force over every choice function, and exact rational probabilities."""
import itertools
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M64 = (1 << 64) - 1


def _vectors():
    msgs = {"zeros32": bytes(32), "ones32": b"\xff" * 32, "inc32": bytes(range(32)), "dec32": bytes(range(31, -1, -1))}
    for line in open(os.path.join(GOLDEN, "crc32c_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "check":
            yield f[1].encode(), int(f[2], 16)
        else:
            yield msgs[f[0]], int(f[1], 16)


@pytest.mark.parametrize("msg,crc", list(_vectors()))
def test_crc32c_published_vectors(msg, crc):
    assert oracle.crc32c_update(0xFFFFFFFF, msg) ^ 0xFFFFFFFF == crc


def _crc_table():
    # an independent, table-driven (byte at a time) CRC-32C built from the polynomial
    t = []
    for b in range(256):
        c = b
        for _ in range(8):
            c = (c >> 1) ^ 0x82F63B78 if c & 1 else c >> 1
        t.append(c)
    return t


_T = _crc_table()


def _crc_table_update(crc, data):
    for byte in data:
        crc = _T[(crc ^ byte) & 0xFF] ^ (crc >> 8)
    return crc


def test_table_crc_matches_the_published_vectors_too():
    for msg, crc in _vectors():
        assert _crc_table_update(0xFFFFFFFF, msg) ^ 0xFFFFFFFF == crc


def test_crc32c_u64_is_the_byte_update_of_the_little_endian_word():
    rng = random.Random(1)
    for _ in range(300):
        x, c = rng.randrange(0, 1 << 64), rng.randrange(0, 1 << 32)
        assert oracle.crc32c_u64(c, x) == _crc_table_update(c, x.to_bytes(8, "little"))
    # CRC registers are affine: the start value and the data contribute by XOR
    for _ in range(100):
        x, y = rng.randrange(0, 1 << 64), rng.randrange(0, 1 << 64)
        assert oracle.crc32c_u64(1, x) == oracle.crc32c_u64(0, x) ^ oracle.crc32c_u64(1, 0)
        assert oracle.crc32c_u64(0, x ^ y) == oracle.crc32c_u64(0, x) ^ oracle.crc32c_u64(0, y)


def test_h_crc_is_the_papers_hash_crc():
    # hash = crc32(0, x) << 32; hash += crc32(1, x); return hash % x  (key 0, bound x)
    rng = random.Random(2)
    for _ in range(300):
        x = rng.choice([rng.randrange(1, 1 << 20), rng.randrange(1, 1 << 40), rng.randrange(1, 1 << 63)])
        b = x.to_bytes(8, "little")
        h = ((_crc_table_update(0, b) << 32) + _crc_table_update(1, b)) % x
        assert oracle.h_crc(0, x, x) == h
    for _ in range(300):  # keyed: the key is XORed into the hashed word
        k, r, bound = rng.randrange(0, 1 << 64), rng.randrange(1, 1 << 50), rng.randrange(1, 1 << 50)
        assert oracle.h_crc(k, r, bound) == oracle.h_crc(0, r ^ k, bound) if (r ^ k) else True
        assert 0 <= oracle.h_crc(k, r, bound) < bound


def test_h_fmix_with_bound_r_is_the_plain_hash():
    rng = random.Random(3)
    for _ in range(500):
        k, r = rng.randrange(0, 1 << 64), rng.randrange(1, 1 << 63)
        assert oracle.h_fmix(k, r, r) == oracle.h(k, r)
        b = rng.randrange(1, 1 << 63)
        assert 0 <= oracle.h_fmix(k, r, b) < b


@pytest.mark.parametrize("n,d,seed", [(50, 3, 1), (200, 1, 9), (31, 7, 123)])
def test_empty_seed_graph_with_loops_is_the_plain_model(n, d, seed):
    E_plain, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(oracle.model_bb_generate(0, 0, None, n, d, seed, 0), E_plain)
    got, _ = oracle.model_edges_range(0, 0, None, d, seed, 0, 0, n * d)
    assert np.array_equal(got.reshape(-1), E_plain)


def _bounds(n0, m0, n, d, flags):
    out = []
    for i in range((n - n0) * d):
        P = 2 * m0 + 2 * i
        out.append(2 * m0 + 2 * d * (i // d) if flags & oracle.NO_LOOPS else P + 1)
    return out


SEEDS = [(1, 1, [0, 0]), (2, 1, [0, 1]), (3, 2, [0, 1, 2, 1])]


@pytest.mark.parametrize("flags", [0, oracle.NO_LOOPS])
@pytest.mark.parametrize("n0,m0,S", SEEDS)
def test_bb_equals_per_edge_chain_for_every_choice_function(n0, m0, S, flags):
    for extra, d in [(1, 2), (2, 1), (2, 2)]:
        n = n0 + extra
        bounds = _bounds(n0, m0, n, d, flags)
        for x in itertools.product(*[range(b) for b in bounds]):
            E = oracle.model_bb_with_choices(n0, m0, S, n, d, flags, x)
            for i in range((n - n0) * d):
                u, v, _ = oracle.model_edge(n0, m0, S, d, 0, flags, i, x=x)
                assert (u, v) == (E[2 * m0 + 2 * i], E[2 * m0 + 2 * i + 1])


@pytest.mark.parametrize("flags", [0, oracle.NO_LOOPS])
def test_bb_with_seed_graph_is_preferential_attachment(flags):
    # exact probabilities: uniform draws over positions == targets chosen in
    # proportion to degree among the allowed earlier nodes
    n0, m0, S = 2, 1, [0, 1]
    n, d = 4, 2
    bounds = _bounds(n0, m0, n, d, flags)
    dist = {}
    for x in itertools.product(*[range(b) for b in bounds]):
        E = tuple(oracle.model_bb_with_choices(n0, m0, S, n, d, flags, x).tolist())
        p = Fraction(1)
        for b in bounds:
            p /= b
        dist[E] = dist.get(E, 0) + p

    def pa(prefix, i):  # sequential preferential attachment, exact
        if i == (n - n0) * d:
            return {tuple(prefix): Fraction(1)}
        u = n0 + i // d
        pool = prefix[:2 * m0 + 2 * d * (i // d)] if flags & oracle.NO_LOOPS else prefix + [u]
        out = {}
        for v in set(pool):
            w = Fraction(pool.count(v), len(pool))
            for e, q in pa(prefix + [u, v], i + 1).items():
                out[e] = out.get(e, 0) + w * q
        return out

    assert dist == pa(list(S), 0)


@pytest.mark.parametrize("flags", [0, oracle.NO_LOOPS, oracle.CRC, oracle.CRC | oracle.NO_LOOPS])
def test_hashed_model_chain_equals_bb_and_keeps_the_invariants(flags):
    rng = np.random.default_rng(flags + 10)
    n0, m0 = 40, 70
    S = rng.integers(0, n0, 2 * m0).astype(np.uint32)
    for n, d, seed in [(2000, 3, 5), (700, 8, 6)]:
        E = oracle.model_bb_generate(n0, m0, S, n, d, seed, flags)
        got, draws = oracle.model_edges_range(n0, m0, S, d, seed, flags, 0, (n - n0) * d)
        new = E[2 * m0:].reshape(-1, 2)
        assert np.array_equal(got, new)
        u, v = new[:, 0].astype(np.int64), new[:, 1].astype(np.int64)
        assert np.array_equal(u, n0 + np.arange(len(u)) // d)
        assert np.all(v <= u) and np.all(v < n)
        if flags & oracle.NO_LOOPS:
            assert np.all(v < u)  # no self-loops
        else:
            assert np.any(v == u)  # self-loops do occur when allowed
        assert int(oracle.count_degrees(E, n).sum()) == len(E)
        assert draws < 2.3 * len(u)  # about two draws per edge on average


def test_no_self_loops_needs_a_seed_edge():
    with pytest.raises(ValueError):
        oracle.model_bb_generate(0, 0, None, 10, 2, 1, oracle.NO_LOOPS)
    with pytest.raises(ValueError):
        oracle.model_bb_generate(5, 0, None, 10, 2, 1, oracle.NO_LOOPS)
    oracle.model_bb_generate(5, 0, None, 10, 2, 1, 0)  # with loops an empty seed graph is fine


def test_crc_hash_draws_are_uniform():
    from scipy import stats
    rng = random.Random(4)
    xs = []
    for _ in range(4000):
        r = rng.randrange(1 << 20, 1 << 40)
        xs.append(oracle.h_crc(oracle.key(7), r, r) / r)
    assert stats.kstest(xs, "uniform").pvalue > 1e-4
