"""The pins must catch plausible mistakes: plant each one in a private copy of
the oracle's C source (on the CPU), rebuild it, and check that some pin from
test_oracle_hash, test_oracle_model, test_oracle_model_ext or
test_oracle_checksum fails against the planted copy."""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_checksum as tc
from tests import test_oracle_hash as th
from tests import test_oracle_model as tm
from tests import test_oracle_model_ext as tx

HERE = os.path.dirname(oracle.__file__)
SRCS = ["bb_oracle.c", "bb_model.c"]

MUTANTS = [
    ("bb_oracle.c", "mix constant", "z *= 0xBF58476D1CE4E5B9ull;", "z *= 0xBF58476D1CE4E5B7ull;"),
    ("bb_oracle.c", "mix shift", "z ^= z >> 27;", "z ^= z >> 28;"),
    ("bb_oracle.c", "key derivation", "return seed * BBO_PHI64;", "return seed + BBO_PHI64;"),
    ("bb_oracle.c", "low instead of high product", "return (uint64_t)(p >> 64);", "return (uint64_t)p;"),
    ("bb_oracle.c", "choice range 0..2i-1", "uint64_t x = bbo_h(key, 2 * i + 1);", "uint64_t x = bbo_h(key, 2 * i + 1) & ~1ull;"),
    ("bb_oracle.c", "source off by one", "E[2 * i] = (uint32_t)(i / d);\n        uint64_t x", "E[2 * i] = (uint32_t)((i + 1) / d);\n        uint64_t x"),
    ("bb_oracle.c", "second endpoint r/d", "*v = r / (2 * d);", "*v = r / d;"),
    ("bb_oracle.c", "chain start", "uint64_t r = 2 * i + 1;\n    uint64_t k = 0;", "uint64_t r = 2 * i + 3;\n    uint64_t k = 0;"),
    ("bb_oracle.c", "stream counts u twice", "if (u < k) deg_k[u] += 1;", "if (u < k) deg_k[u] += 2;"),
    ("bb_oracle.c", "checksum multiplier dropped", "return ((u << 32) + v) * (2 * i + 1);", "return ((u << 32) + v);"),
    ("bb_oracle.c", "checksum multiplier even", "return ((u << 32) + v) * (2 * i + 1);", "return ((u << 32) + v) * (2 * i + 2);"),
    ("bb_oracle.c", "checksum endpoints swapped", "return ((u << 32) + v) * (2 * i + 1);", "return ((v << 32) + u) * (2 * i + 1);"),
    ("bb_oracle.c", "checksum XOR of a partial range", "*cs ^= x;", "*cs ^= x & ~1ull;"),
    ("bb_model.c", "draw bound with loops r + 1", "if (!(M->flags & BBO_NO_LOOPS)) return r;", "if (!(M->flags & BBO_NO_LOOPS)) return r + 1;"),
    ("bb_model.c", "no-loop bound at the edge, not the node", "return 2 * M->m0 + 2 * M->d * (i / M->d);", "return 2 * M->m0 + 2 * i;"),
    ("bb_model.c", "seed offset m0 instead of 2 m0", "return (uint32_t)(M->n0 + (r - 2 * M->m0) / (2 * M->d));", "return (uint32_t)(M->n0 + (r - M->m0) / (2 * M->d));"),
    ("bb_model.c", "crc registers swapped", "((uint64_t)bbo_crc32c_u64(0, z) << 32) + (uint64_t)bbo_crc32c_u64(1, z)", "((uint64_t)bbo_crc32c_u64(1, z) << 32) + (uint64_t)bbo_crc32c_u64(0, z)"),
    ("bb_model.c", "crc-32 polynomial", "crc = (crc >> 1) ^ (0x82F63B78u & (0u - (crc & 1u)));", "crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));"),
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
    yield lambda: [tc.test_a_lone_unit_edge_gives_the_position_multiplier(i) for i in (0, 3, 123457)]
    yield tc.test_word_is_a_bijection_of_the_pair_for_every_position
    yield tc.test_two_edges_that_exchange_their_targets_change_the_checksum
    yield tc.test_checksum_is_the_xor_of_any_split_and_repeats_cancel
    yield lambda: [tx.test_crc32c_published_vectors(msg, c) for msg, c in tx._vectors()]
    yield tx.test_h_crc_is_the_papers_hash_crc
    yield lambda: tx.test_empty_seed_graph_with_loops_is_the_plain_model(50, 3, 1)
    yield lambda: tx.test_bb_equals_per_edge_chain_for_every_choice_function(2, 1, [0, 1], oracle.NO_LOOPS)
    yield lambda: tx.test_bb_equals_per_edge_chain_for_every_choice_function(2, 1, [0, 1], 0)
    yield lambda: tx.test_bb_with_seed_graph_is_preferential_attachment(oracle.NO_LOOPS)
    yield lambda: tx.test_hashed_model_chain_equals_bb_and_keeps_the_invariants(oracle.NO_LOOPS)


@pytest.mark.parametrize("fname,name,old,new", MUTANTS, ids=[m[1] for m in MUTANTS])
def test_pins_catch_planted_mistake(fname, name, old, new, monkeypatch):
    with tempfile.TemporaryDirectory() as tmp:
        cs = []
        for f in SRCS:
            src = open(os.path.join(HERE, f)).read()
            if f == fname:
                assert src.count(old) == 1, name
                src = src.replace(old, new)
            cs.append(os.path.join(tmp, f))
            open(cs[-1], "w").write(src)
        so = os.path.join(tmp, "m.so")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", so] + cs)
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
