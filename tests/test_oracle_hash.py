"""Pins of the oracle's keyed position hash against facts outside the oracle.

The hash maps an array position r >= 1 to a value in 0..r-1 (paper Section 2,
the paragraph on reproducing random behaviour).  Its pieces are pinned by:

* the published SplitMix64 outputs (tests/golden/splitmix64_outputs.txt): the
  k-th output is fmix64(k * phi64) = fmix64(key(k)), which fixes both the
  output mix (constants and shifts) and the key derivation seed * phi64;
* invertibility of the mix (an inverse built here from the xor-shift and
  modular-inverse identities must undo it);
* big-integer arithmetic for the 64x64 -> high 64 product;
* the range 0 <= h(r) < r and the uniformity of h(r)/r.
"""
import os
import random

import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_outputs.txt")


def _splitmix_vectors():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, hx, dec = line.split()
            assert int(hx, 16) == int(dec)
            out.append((int(k), int(hx, 16)))
    return out


@pytest.mark.parametrize("k,expected", _splitmix_vectors())
def test_splitmix64_published_outputs(k, expected):
    # k-th output of SplitMix64 from state 0 == fmix64(key(k)).
    assert oracle.fmix64(oracle.key(k)) == expected


def test_key_is_seed_times_phi64_wrapping():
    # seed 0 gives key 0; the key is linear in the seed mod 2^64.
    assert oracle.key(0) == 0
    k1 = oracle.key(1)
    for s in [2, 3, 12345, (1 << 63) + 5, M64]:
        assert oracle.key(s) == (s * k1) & M64


def _unxorshift(y, s):
    # inverse of z ^= z >> s on 64-bit words
    z = y
    for _ in range(64 // s + 1):
        z = y ^ (z >> s)
    return z & M64


def _inverse_fmix64(y):
    c1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    c2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    y = _unxorshift(y, 31)
    y = (y * c2) & M64
    y = _unxorshift(y, 27)
    y = (y * c1) & M64
    y = _unxorshift(y, 30)
    return y


def test_fmix64_is_a_bijection():
    rng = random.Random(2016)
    xs = [0, 1, M64, 1 << 63] + [rng.getrandbits(64) for _ in range(2000)]
    for x in xs:
        assert _inverse_fmix64(oracle.fmix64(x)) == x
    # and it really mixes: distinct inputs map to distinct outputs
    assert len({oracle.fmix64(x) for x in range(4096)}) == 4096


@pytest.mark.parametrize(
    "a,b,expected",
    [
        (M64, M64, M64 - 1),  # (2^64-1)^2 = 2^128 - 2^65 + 1
        (M64, 1, 0),
        (1 << 63, 7, 3),  # 2^63 * odd b -> (b-1)/2
        (1 << 63, M64, (M64 - 1) // 2),
        (0, M64, 0),
        (1 << 32, 1 << 32, 1),
    ],
)
def test_umul64hi_edge_cases(a, b, expected):
    assert oracle.umul64hi(a, b) == expected


def test_umul64hi_random_against_big_ints():
    rng = random.Random(7)
    for _ in range(5000):
        a, b = rng.getrandbits(64), rng.getrandbits(rng.choice([8, 31, 32, 33, 37, 64]))
        assert oracle.umul64hi(a, b) == (a * b) >> 64


def test_h_maps_into_0_to_r_minus_1():
    rng = random.Random(11)
    rs = [1, 2, 3, (1 << 31) - 1, 1 << 31, (1 << 32) + 1, (1 << 37) - 1, (1 << 63) + 1, M64]
    rs += [rng.getrandbits(rng.randint(1, 64)) | 1 for _ in range(5000)]
    for seed in [0, 1, 7, 42, M64]:
        key = oracle.key(seed)
        for r in rs:
            x = oracle.h(key, r)
            assert 0 <= x < r
    # h(1) is 0 for every key: the first edge always points to position 0
    for seed in range(100):
        assert oracle.h(oracle.key(seed), 1) == 0


def test_h_is_close_to_uniform_on_0_to_r_minus_1():
    scipy_stats = pytest.importorskip("scipy.stats")
    key = oracle.key(1)
    rs = np.arange(1, 2 * 200000, 2, dtype=np.uint64) + np.uint64(1 << 20)
    u = np.array([oracle.h(key, int(r)) / int(r) for r in rs])
    assert scipy_stats.kstest(u, "uniform").pvalue > 1e-4
    # parity of h(r) is a fair coin: this is what makes chains short
    ev = np.mean([(oracle.h(key, int(r)) & 1) == 0 for r in rs[:50000]])
    assert abs(ev - 0.5) < 0.01
