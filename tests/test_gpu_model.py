"""GPU parity of the generalized model (seed graph, self-loop-free draws,
the paper's CRC hash) against the CPU oracle, bit-exact: every flag
combination, seed graphs of several shapes, ranges at odd offsets,
misaligned outputs, and 64-bit positions."""
import sys

import numpy as np
import pytest

import oracle

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


FLAGS = [(False, "fmix"), (True, "fmix"), (False, "crc"), (True, "crc")]


def _oflags(no_loops, h):
    return (oracle.NO_LOOPS if no_loops else 0) | (oracle.CRC if h == "crc" else 0)


def _seed_graph(n0, m0, seed):
    S = np.random.default_rng(seed).integers(0, max(n0, 1), 2 * m0).astype(np.uint32)
    return S, torch.from_numpy(S.view(np.int32).copy()).to("cuda")


@pytest.mark.parametrize("no_loops,h", FLAGS)
@pytest.mark.parametrize("n0,m0,n,d,seed", [(1, 1, 3000, 3, 5), (40, 70, 20000, 7, 6), (500, 2000, 9000, 1, 7),
                                             (3, 2, 5000, 16, 0)])
def test_model_matches_the_oracle(no_loops, h, n0, m0, n, d, seed):
    _say("model", no_loops, h, n0, m0, n, d, seed)
    S, St = _seed_graph(n0, m0, seed + 100)
    m = (n - n0) * d
    out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h)
    torch.cuda.synchronize()
    ref, _ = oracle.model_edges_range(n0, m0, S, d, seed, _oflags(no_loops, h), 0, m)
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref)
    if no_loops:
        assert np.all(got[:, 1] != got[:, 0])


@pytest.mark.parametrize("no_loops,h", FLAGS)
def test_model_with_chain_tails_carried_across_tiles(no_loops, h):
    # about 2 tiles per resident wave, so tile tails run into the next tile;
    # whole graph, then a range that starts inside a tile
    n0, m0, n, d, seed = 100, 1000, (1 << 20) + 333, 16, 5
    _say("model carried tails", no_loops, h, n)
    S, St = _seed_graph(n0, m0, seed + 200)
    m = (n - n0) * d
    # the oracle's sequential run lists the seed graph's m0 edges first
    ref = oracle.model_bb_generate(n0, m0, S, n, d, seed, _oflags(no_loops, h)).reshape(-1)[2 * m0 :]
    assert ref.size == 2 * m
    out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32).reshape(-1), ref)
    b, c = 4321, m // 2 + 17
    out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h, begin=b, count=c)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32).reshape(-1), ref[2 * b : 2 * (b + c)])


@pytest.mark.parametrize("no_loops,h", FLAGS)
def test_model_ranges_and_misaligned_outputs(no_loops, h):
    n0, m0, n, d, seed = 30, 45, 40000, 5, 11
    S, St = _seed_graph(n0, m0, 3)
    m = (n - n0) * d
    for b, c in [(1, 7777), (m - 3001, 3001), (12345, 1)]:
        _say("model range", no_loops, h, b, c)
        buf = torch.full((2 * c + 1,), -1, dtype=torch.int32, device="cuda")
        out = buf[1:].view(c, 2)  # 4-byte aligned only
        ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h, begin=b, count=c,
                          out=out)
        torch.cuda.synchronize()
        ref, _ = oracle.model_edges_range(n0, m0, S, d, seed, _oflags(no_loops, h), b, c)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)
        assert int(buf[0]) == -1


def test_trivial_seed_graph_is_the_plain_generator():
    n, d, seed = 50000, 6, 21
    a = ba.generate_model(n, d, seed)
    b, _ = ba.generate(n, d, seed)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("no_loops,h", FLAGS)
def test_model_with_64_bit_positions(no_loops, h):
    n0, m0, d, seed = 7, 1000, 17, 4
    n = (1 << 28) + 5  # positions beyond 2^32
    S, St = _seed_graph(n0, m0, 9)
    m = (n - n0) * d
    for b in [0, (1 << 31) - 500, m - 1000]:
        _say("model wide", no_loops, h, b)
        out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h, begin=b, count=1000)
        torch.cuda.synchronize()
        ref, _ = oracle.model_edges_range(n0, m0, S, d, seed, _oflags(no_loops, h), b, 1000)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)


@pytest.mark.parametrize("m0", [0, 4])
def test_model_at_the_32_bit_position_boundary(m0):
    # 2*m0 + 2*(n-n0)*d = 2^32 exactly (32-bit path) or just past it (64-bit path)
    n0, d, seed = 3, 16, 8
    n = n0 + (1 << 27)
    S, St = _seed_graph(n0, m0, 12)
    m = (n - n0) * d
    for b in [0, m - 2000]:
        _say("model boundary", m0, b)
        out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St if m0 else None, begin=b, count=2000)
        torch.cuda.synchronize()
        ref, _ = oracle.model_edges_range(n0, m0, S, d, seed, 0, b, 2000)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)


@pytest.mark.parametrize("no_loops,h", FLAGS)
def test_model_with_a_large_seed_graph_near_2_32(no_loops, h):
    # 2*m0 = 3*2^23 seed positions and new positions up to just below 2^32:
    # the one-compare stop test at a large P0, chains that end in the seed
    # graph often (first range) and rarely (last range), and seed IDs of
    # every size (IDs >= n0 pass through unchanged)
    n0, m0, d, seed = 1000, 3 << 22, 5, 13
    n = n0 + ((1 << 32) - 2 * m0) // (2 * d)
    rng = np.random.default_rng(17)
    S = rng.integers(0, n0, 2 * m0).astype(np.uint32)
    big = rng.integers(0, 2 * m0, 4096)
    S[big] = rng.integers(0, 1 << 32, big.size, dtype=np.uint64).astype(np.uint32)
    St = torch.from_numpy(S.view(np.int32)).to("cuda")
    m = (n - n0) * d
    assert 2 * m0 + 2 * m <= 1 << 32
    for b, c in [(0, 6000), (m // 2 + 3, 3001), (m - 4097, 4097)]:
        _say("model large seed", no_loops, h, b, c)
        out = ba.generate_model(n, d, seed, n0=n0, seed_edges=St, no_self_loops=no_loops, hash=h, begin=b, count=c)
        torch.cuda.synchronize()
        ref, _ = oracle.model_edges_range(n0, m0, S, d, seed, _oflags(no_loops, h), b, c)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)
