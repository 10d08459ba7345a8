"""The pins must catch plausible mistakes: plant each one in a private copy of
the oracle's C source (on the CPU), rebuild it, and check that some pin from
test_oracle_hash / test_oracle_model fails against the planted copy."""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_hash as th
from tests import test_oracle_model as tm

SRC = os.path.join(os.path.dirname(oracle.__file__), "bb_oracle.c")

MUTANTS = [
    ("mix constant", "z *= 0xBF58476D1CE4E5B9ull;", "z *= 0xBF58476D1CE4E5B7ull;"),
    ("mix shift", "z ^= z >> 27;", "z ^= z >> 28;"),
    ("key derivation", "return seed * BBO_PHI64;", "return seed + BBO_PHI64;"),
    ("low instead of high product", "return (uint64_t)(p >> 64);", "return (uint64_t)p;"),
    ("choice range 0..2i-1", "uint64_t x = bbo_h(key, 2 * i + 1);", "uint64_t x = bbo_h(key, 2 * i + 1) & ~1ull;"),
    ("source off by one", "E[2 * i] = (uint32_t)(i / d);\n        uint64_t x", "E[2 * i] = (uint32_t)((i + 1) / d);\n        uint64_t x"),
    ("second endpoint r/d", "*v = r / (2 * d);", "*v = r / d;"),
    ("chain start", "uint64_t r = 2 * i + 1;\n    uint64_t k = 0;", "uint64_t r = 2 * i + 3;\n    uint64_t k = 0;"),
    ("stream counts u twice", "if (u < k) deg_k[u] += 1;", "if (u < k) deg_k[u] += 2;"),
]


def _pins():
    yield lambda: [th.test_splitmix64_published_outputs(k, e) for k, e in th._splitmix_vectors()]
    yield th.test_key_is_seed_times_phi64_wrapping
    yield th.test_h_maps_into_0_to_r_minus_1
    yield lambda: tm.test_bb_distribution_is_preferential_attachment(3, 2)
    yield lambda: tm.test_per_edge_definition_equals_batagelj_brandes(4096, 16, 7)
    yield lambda: tm.test_literal_python_generate_edge_equals_c_oracle(250, 4, 1)
    yield tm.test_streaming_consumer_agrees_with_stored_array
    yield tm.test_degree_distribution_has_the_barabasi_albert_power_law_tail


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, monkeypatch):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "m.c")
        so = os.path.join(tmp, "m.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", so, c])
        good = oracle.lib()
        mutant = ctypes.CDLL(so)
        for fname in dir(good):
            if fname.startswith("bbo_"):
                f, g = getattr(mutant, fname), getattr(good, fname)
                f.restype, f.argtypes = g.restype, g.argtypes
        monkeypatch.setattr(oracle, "_lib", mutant)
        caught = []
        for pin in _pins():
            try:
                pin()
            except (AssertionError, ValueError):
                caught.append(pin)
        assert caught, "no pin caught: " + name
