"""Pins of the oracle's edge checksum (the streaming consumer's second output,
modelled on the whole-graph checks of paper Section 3).

The checksum is this project's definition: the XOR over edges i of the word
w_i = (u_i * 2^32 + v_i) * (2i + 1) mod 2^64.  What the definition fixes,
and what these tests check without restating the formula:

* the packed pair u * 2^32 + v is injective for node IDs below 2^32, and the
  multiplier 2i + 1 is odd, hence invertible mod 2^64: the word map is a
  bijection of the pair for every i, so a change of any single edge (either
  endpoint, any bit) always changes the checksum;
* the multiplier depends on the edge's position: two edges of one node that
  exchange their targets change the checksum (a plain XOR of pairs would not
  see it, nor would an order-free word);
* special values: the all-zero edge has word 0, so the d self-loops (0, 0)
  that open every graph contribute nothing; an edge array that is zero except
  edge i = (0, 1) has checksum 2i + 1, and except edge i = (1, 0) has
  checksum (2i + 1) * 2^32 mod 2^64 (the multiplier itself, shifted);
* XOR is associative and self-inverse: the checksum of a graph is the XOR of
  the checksums of any split of its edges, and an edge listed twice cancels.
"""
import random

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1


def _unit_array(m, i, u, v):
    E = np.zeros(2 * m, dtype=np.uint32)
    E[2 * i] = u
    E[2 * i + 1] = v
    return E


@pytest.mark.parametrize("i", [0, 1, 2, 3, 1000, 123457, 299999])
def test_a_lone_unit_edge_gives_the_position_multiplier(i):
    m = 300000
    assert oracle.checksum_E(_unit_array(m, i, 0, 1)) == 2 * i + 1
    assert oracle.checksum_E(_unit_array(m, i, 1, 0)) == ((2 * i + 1) << 32) & M64
    assert oracle.checksum_E(np.zeros(2 * m, dtype=np.uint32)) == 0


def test_word_is_a_bijection_of_the_pair_for_every_position():
    # pairs that differ in a single bit of u or of v, at every bit, including
    # the top bit of u (a packed difference of 2^63: an even multiplier would
    # map both pairs to the same word)
    rng = random.Random(5)
    for _ in range(300):
        i = rng.randrange(0, 1 << 40)
        u, v = rng.randrange(1 << 32), rng.randrange(1 << 32)
        w = oracle.edge_word(i, u, v)
        for b in range(32):
            assert oracle.edge_word(i, u ^ (1 << b), v) != w
            assert oracle.edge_word(i, u, v ^ (1 << b)) != w


def test_changing_any_single_edge_changes_the_checksum():
    n, d, seed = 5000, 4, 11
    E, _ = oracle.bb_generate(n, d, seed)
    cs = oracle.checksum_E(E)
    rng = random.Random(3)
    for _ in range(200):
        j = rng.randrange(n * d)
        for pos, bit in ((2 * j + 1, rng.randrange(32)), (2 * j, 31), (2 * j, rng.randrange(32))):
            F = E.copy()
            F[pos] ^= np.uint32(1 << bit)
            assert oracle.checksum_E(F) != cs


def test_two_edges_that_exchange_their_targets_change_the_checksum():
    n, d, seed = 5000, 8, 2
    E, _ = oracle.bb_generate(n, d, seed)
    cs = oracle.checksum_E(E)
    swaps = 0
    for u in range(1, n, 37):
        a, b = u * d, u * d + d - 1  # first and last edge of node u
        if E[2 * a + 1] == E[2 * b + 1]:
            continue
        F = E.copy()
        F[2 * a + 1], F[2 * b + 1] = E[2 * b + 1], E[2 * a + 1]
        assert oracle.checksum_E(F) != cs
        swaps += 1
    assert swaps > 100


def test_checksum_is_the_xor_of_any_split_and_repeats_cancel():
    n, d, seed = 3000, 3, 9
    m = n * d
    E, _ = oracle.bb_generate(n, d, seed)
    cs = oracle.checksum_E(E)
    # the d opening self-loops (0, 0) contribute nothing
    Z = E.copy()
    Z[: 2 * d] = 0
    assert oracle.checksum_E(Z) == cs
    # stream over a ragged split of the edges (positions keep their index)
    acc, i = 0, 0
    for c in (1, 2, 1000, 77, m):
        c = min(c, m - i)
        _, acc, _ = oracle.stream(d, seed, i, c, 0, None, acc)
        i += c
    assert acc == cs
    # XOR of every edge's word from the per-edge definition
    x = 0
    for j in range(m):
        u, v, _ = oracle.edge(d, seed, j)
        x ^= oracle.edge_word(j, u, v)
    assert x == cs
    # an edge counted twice cancels
    _, twice, _ = oracle.stream(d, seed, 17, 1, 0, None, 0)
    _, twice, _ = oracle.stream(d, seed, 17, 1, 0, None, twice)
    assert twice == 0
