"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element and bit-exact (the method is integer-only, so the
tolerance is zero)."""
import ctypes
import random
import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1602_07106_amd as ba  # noqa: E402

M64 = (1 << 64) - 1


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _u32(t):
    return t.cpu().numpy().view(np.uint32).reshape(-1)


def _u64(t):
    return t.cpu().numpy().view(np.uint64).reshape(-1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ba.lib()
    yield
    torch.cuda.synchronize()


SMALL = [
    (100000, 4, 1),      # the small workload, whole
    (1, 1, 0),
    (1, 64, 9),
    (2, 1, 3),
    (777, 3, 5),         # ragged tail tile
    (5000, 33, 42),      # non-power-of-two d, several tiles
    (4096, 16, 7),
    (30011, 7, M64),
    (65537, 1, 123456789),
]


@pytest.mark.parametrize("n,d,seed", SMALL)
def test_generate_matches_batagelj_brandes(n, d, seed):
    _say("generate", n, d, seed)
    edges, deg = ba.generate(n, d, seed, degrees=True)
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(_u32(edges), E)
    assert np.array_equal(_u32(deg).astype(np.uint64), oracle.count_degrees(E, n))


def test_generate_without_degrees_and_misaligned_output():
    n, d, seed = 12345, 6, 11
    _say("misaligned", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    buf = torch.full((2 * n * d + 4,), -1, dtype=torch.int32, device="cuda")
    for shift in [0, 1, 2, 3]:  # 16-byte, 4-byte, 8-byte, 4-byte aligned
        view = buf[shift : shift + 2 * n * d]
        ba.generate(n, d, seed, out=view)
        torch.cuda.synchronize()
        assert np.array_equal(_u32(view), E), shift


def test_edges_only_with_chain_tails_carried_across_tiles():
    # 2^26 edges: about 8 1024-edge tiles per resident wave, so nearly every
    # tile's chain tail runs into the wave's next tile (and some tails hit
    # the claim cap); whole graph at 16- and 4-byte alignment, then a range
    # that starts inside a tile
    n, d, seed = (1 << 20) + 777, 64, 5
    m = n * d
    _say("carried tails", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    buf = torch.full((2 * m + 4,), -1, dtype=torch.int32, device="cuda")
    for shift in [0, 1]:
        view = buf[shift : shift + 2 * m]
        ba.generate(n, d, seed, out=view)
        torch.cuda.synchronize()
        assert np.array_equal(_u32(view), E), shift
    b, c = 12345, (1 << 24) + 99
    out = ba.generate_range(n, d, seed, b, c)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(out), E[2 * b : 2 * (b + c)])


def test_random_sweep_of_ranges_with_carried_tails():
    # seeded random graphs and ranges of 1e7..4e7 edges (more tiles than
    # resident waves in both generators), d with and without a power of two,
    # ranges starting inside a tile; every other case with degrees (the fused
    # kernel on a range, both endpoints added)
    rng = np.random.default_rng(20261203)
    for k in range(8):
        d = int(rng.choice([1, 2, 3, 5, 7, 12, 16, 31, 33, 64]))
        n = max(2, int(rng.integers(10_000_000, 40_000_000)) // d + int(rng.integers(0, 1000)))
        m = n * d
        b = int(rng.integers(0, m // 4))
        c = int(rng.integers(m // 2, m - b))
        seed = int(rng.integers(0, 1 << 63))
        with_deg = k % 2 == 1
        _say("sweep", k, n, d, seed, b, c, with_deg)
        deg = torch.zeros(n, dtype=torch.int32, device="cuda") if with_deg else None
        out = ba.generate_range(n, d, seed, b, c, deg=deg)
        torch.cuda.synchronize()
        ref, _ = oracle.edges_range(d, seed, b, c)
        ref = ref.astype(np.uint32)
        assert np.array_equal(_u32(out), ref), k
        if with_deg:
            assert np.array_equal(_u32(deg).astype(np.int64), np.bincount(ref, minlength=n)), k


def test_ranges_stitch_to_the_whole_graph_and_accumulate_degrees():
    n, d, seed = 40000, 5, 77
    m = n * d
    _say("ranges", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    deg = torch.zeros(n, dtype=torch.int32, device="cuda")
    rng = random.Random(1)
    cuts = sorted(rng.sample(range(1, m), 25)) + [m]
    order = list(zip([0] + cuts[:-1], cuts))
    rng.shuffle(order)
    got = np.empty(2 * m, dtype=np.uint32)
    for b, e in order:
        out = ba.generate_range(n, d, seed, b, e - b, deg=deg)
        torch.cuda.synchronize()
        got[2 * b : 2 * e] = _u32(out)
    assert np.array_equal(got, E)
    assert np.array_equal(_u32(deg).astype(np.uint64), oracle.count_degrees(E, n))


def test_wide_positions_beyond_2_32():
    # positions >= 2^32 take the 64-bit hash path even for uint32 output
    n, d, seed = 1 << 28, 16, 7
    m = n * d
    for b, c in [(m - 5000, 5000), ((1 << 31) - 2000, 4000), (3 << 30, 12345)]:
        _say("wide", b, c)
        out = ba.generate_range(n, d, seed, b, c)
        torch.cuda.synchronize()
        ref, _ = oracle.edges_range(d, seed, b, c)
        assert np.array_equal(_u32(out), ref.astype(np.uint32))


def test_u64_ids_sampled_across_the_streaming_workload():
    n, d, seed = 1 << 30, 64, 42
    m = n * d
    rng = random.Random(9)
    starts = [0, m - 3000, (1 << 31) - 77] + [rng.randrange(0, m - 3000) for _ in range(6)]
    for b in starts:
        _say("u64 range", b)
        out = ba.generate_range_u64(n, d, seed, b, 3000)
        torch.cuda.synchronize()
        ref, _ = oracle.edges_range(d, seed, b, 3000)
        assert np.array_equal(_u64(out), ref)


@pytest.mark.parametrize("n,d,seed,k", [(20000, 5, 3, 1000), (100000, 4, 1, 100000), (50000, 3, 8, 20000), (1, 2, 0, 1)])
def test_streaming_degrees_and_checksum(n, d, seed, k):
    _say("degrees", n, d, seed, k)
    deg, cs = ba.degrees(n, d, seed, k)
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(_u64(deg), oracle.count_degrees(E, n)[:k])
    assert cs == oracle.checksum_E(E)


def test_streaming_ranges_accumulate_including_wide_positions():
    n, d, seed, k = 1 << 30, 16, 5, 30000
    rng = random.Random(4)
    deg = torch.zeros(k, dtype=torch.int64, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ref = np.zeros(k, dtype=np.uint64)
    rcs = 0
    for b, c in [(0, 200000), ((1 << 31) - 70000, 140000), ((1 << 32) - 100000, 100000),
                 (rng.randrange(1 << 32, n * d - 50000), 50000)]:
        _say("degrees range", b, c)
        ba.degrees_range(n, d, seed, b, c, k, deg, cs)
        ref, rcs, _ = oracle.stream(d, seed, b, c, k, ref, rcs)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(deg), ref)
    assert (int(cs.item()) & M64) == rcs


@pytest.mark.parametrize("tier", [ba.TIER_16K, ba.TIER_64K])
def test_streaming_ranges_with_node_ids_past_2_32(tier):
    # n > 2^32: endpoints at and above 2^32 enter the checksum word
    # (u * 2^32 + v) with their high words; positions near 2^63 and 2^64 make
    # the wide hash's 64x64 high product carry out of its 64-bit partial sum
    k = 1000
    for n, d, seed in [((1 << 33) + 3, 1, 9), (1 << 40, 1 << 21, 13), (1 << 33, (1 << 30) - 1, 21)]:
        m = n * d
        for b, c in [(m - 3000, 3000), (m // 2 - 1500, 3000), (m // 3, 2000)]:
            _say("degrees range past 2^32", n, d, seed, b, c, tier)
            deg = torch.zeros(k, dtype=torch.int64, device="cuda")
            cs = torch.zeros(1, dtype=torch.int64, device="cuda")
            ba.degrees_range(n, d, seed, b, c, k, deg, cs, tier=tier)
            torch.cuda.synchronize()
            ref, rcs, _ = oracle.stream(d, seed, b, c, k)
            assert np.array_equal(_u64(deg), ref)
            assert (int(cs.item()) & M64) == rcs


@pytest.mark.parametrize("tier", [ba.TIER_16K, ba.TIER_64K])
@pytest.mark.parametrize("n,d,seed,k", [(100000, 4, 1, 100000), (20000, 5, 3, 1000), (70001, 9, 77, 65537),
                                        (3000, 2, 5, 3000)])
def test_streaming_degrees_on_either_lds_tier(tier, n, d, seed, k):
    """Both LDS counter tiers give the oracle's counts, whichever holds the
    node (LDS word or global atomic) and at the 65536-node tier edge."""
    _say("degrees tier", tier, n, d, seed, k)
    deg, cs = ba.degrees(n, d, seed, k, tier=tier)
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(_u64(deg), oracle.count_degrees(E, n)[:k])
    assert cs == oracle.checksum_E(E)


@pytest.mark.parametrize("tier", [ba.TIER_16K, ba.TIER_64K])
@pytest.mark.parametrize("begin,d", [(0, 1 << 24), ((1 << 31) - (1 << 12), 1 << 31)])
def test_streaming_degrees_of_two_very_heavy_nodes(tier, begin, d):
    """n = 2 with a huge d: about 2^25 targets land on nodes 0 and 1, so every
    block of the 64K tier takes the 16-bit counters of both halves of one LDS
    word past 0x7FFF several times (up to the 32768-per-round maximum).  The
    second case runs on 64-bit positions (edges straddling 2^31, the
    boundary between nodes 0 and 1)."""
    n, count, k = 2, 1 << 25, 2
    _say("heavy degrees", tier, begin, d)
    deg = torch.zeros(k, dtype=torch.int64, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ba.degrees_range(n, d, seed := 11, begin, count, k, deg, cs, tier=tier)
    torch.cuda.synchronize()
    ref, rcs, _ = oracle.stream(d, seed, begin, count, k)
    got = _u64(deg)
    assert got.sum() == 2 * count
    assert np.array_equal(got, ref)
    assert (int(cs.item()) & M64) == rcs


@pytest.mark.parametrize("d", [16, 12])
@pytest.mark.parametrize("tier", [ba.TIER_16K, ba.TIER_64K])
def test_streaming_tiers_on_wide_positions_accumulate(tier, d):
    """Both tiers on ranges with 64-bit positions (around 2^31 and 2^32 and
    beyond), first_k = 10^5, so LDS counters, the 16-bit wrap moves and the
    global atomics all run on the wide kernels, with d a power of two (shift)
    and not (multiply-high division)."""
    n, seed, k = 1 << 30, 9, 100000
    deg = torch.zeros(k, dtype=torch.int64, device="cuda")
    cs = torch.zeros(1, dtype=torch.int64, device="cuda")
    ref = np.zeros(k, dtype=np.uint64)
    rcs = 0
    for b, c in [((1 << 31) - 70000, 140000), ((1 << 32) - 100000, 300000), (n * d - 250000, 250000)]:
        _say("tier range", tier, d, b, c)
        ba.degrees_range(n, d, seed, b, c, k, deg, cs, tier=tier)
        ref, rcs, _ = oracle.stream(d, seed, b, c, k, ref, rcs)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(deg), ref)
    assert (int(cs.item()) & M64) == rcs


@pytest.mark.parametrize("tier", [ba.TIER_AUTO, ba.TIER_16K, ba.TIER_64K])
def test_streaming_checksum_alone(tier):
    """first_k = 0: no degree is counted, the checksum is still every edge's."""
    n, d, seed = 50000, 7, 13
    _say("checksum only", tier)
    deg, cs = ba.degrees(n, d, seed, 0, tier=tier)
    torch.cuda.synchronize()
    assert deg.numel() == 0
    E, _ = oracle.bb_generate(n, d, seed)
    assert cs == oracle.checksum_E(E)


def _pool_used_high():
    """High-water mark of the device's stream-ordered pool (bytes)."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    v = ctypes.c_uint64(0)
    assert hip.hipMemPoolGetAttribute(pool, 8, ctypes.byref(v)) == 0  # hipMemPoolAttrUsedMemHigh
    return pool, v.value, hip


def test_degrees_without_a_workspace_allocate_nothing():
    # ba_generate / ba_generate_range with deg and no workspace: global
    # atomics from the generator, no device allocation of any kind
    n, d, seed = 70000, 6, 21
    m = n * d
    _say("generate deg no-ws", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    out = torch.empty(2 * m, dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    racc = torch.zeros(n, dtype=torch.int32, device="cuda")
    rout = torch.empty(2 * m, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def run():
        racc.zero_()
        assert ba.lib().ba_generate(n, d, seed, out.data_ptr(), deg.data_ptr(), st) == 0
        for b, c in [(0, 1000), (1000, 12345), (13345, m - 13345)]:
            assert ba.lib().ba_generate_range(n, d, seed, b, c, rout.data_ptr() + 8 * b, racc.data_ptr(), st) == 0
        torch.cuda.synchronize()

    run()  # first launches load the kernels
    pool, _, hip = _pool_used_high()
    zero = ctypes.c_uint64(0)
    assert hip.hipMemPoolSetAttribute(pool, 8, ctypes.byref(zero)) == 0  # reset the high-water mark
    free0 = torch.cuda.mem_get_info()[0]
    run()
    assert _pool_used_high()[1] == 0
    assert torch.cuda.mem_get_info()[0] == free0
    assert np.array_equal(_u32(out), E)
    assert np.array_equal(_u32(rout), E)
    ref = oracle.count_degrees(E, n)
    assert np.array_equal(_u32(deg).astype(np.uint64), ref)
    assert np.array_equal(_u32(racc).astype(np.uint64), ref)


@pytest.mark.parametrize("scale", [0.02, 0.5])
def test_degree_overflow_fallback_is_exact(scale):
    # shrunken region capacities push most second endpoints through the fallback
    n, d, seed = 300000, 5, 8
    m = n * d
    _say("overflow", scale)
    E, _ = oracle.bb_generate(n, d, seed)
    edges = torch.empty(2 * m, dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = ba.workspace(n, d, m)
    st = torch.cuda.current_stream().cuda_stream
    assert ba.lib().ba_test_generate_ws_scaled(n, d, seed, edges.data_ptr(), deg.data_ptr(), ws.data_ptr(),
                                               ws.numel(), scale, st) == 0
    torch.cuda.synchronize()
    assert np.array_equal(_u32(edges), E)
    assert np.array_equal(_u32(deg).astype(np.uint64), oracle.count_degrees(E, n))


def test_degrees_in_several_passes_with_heavy_sub_buckets():
    # a workspace for 2^20 edges forces 32 passes; the lowest 32768-node
    # sub-bucket holds ~3M second endpoints, i.e. several count parts
    n, d, seed = 1 << 22, 8, 13
    m = n * d
    _say("multi-pass", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    ref = oracle.count_degrees(E, n)
    ws = ba.workspace(n, d, 1 << 20)
    deg = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = ba.generate_range(n, d, seed, 0, m, deg=deg, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(out), E)
    assert np.array_equal(_u32(deg).astype(np.uint64), ref)
    edges, deg2 = ba.generate(n, d, seed, degrees=True)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(deg2).astype(np.uint64), ref)
    # the whole graph through the same small workspace: the first pass stores
    # single-part counts directly over the filled first endpoints, the other
    # 31 read-modify-write
    edges, deg3 = ba.generate(n, d, seed, degrees=True, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(edges), E)
    assert np.array_equal(_u32(deg3).astype(np.uint64), ref)


def test_extreme_parameters_sampled():
    # the largest uint32 graph (IDs up to 2^32 - 1), a huge d (one divisor
    # for 2^31 - 1 edges per node), d = 1 with 64-bit positions, extreme seeds
    # d = 2^31 with n = 1: the largest power-of-two divisor on 32-bit positions;
    # n = 3, d = 715827882: a large odd-factor divisor with edge indices up to
    # 2^31 - 3 on 32-bit positions (the 31-bit-numerator division)
    # positions near 2^63 and 2^64 (n = 2^40, d = 2^21; n = 2^33, d = 2^30 - 1):
    # the wide hash's high product carries out of its 64-bit partial sum
    cases = [((1 << 32), 2, 5), ((1 << 32), 1, M64), (3, (1 << 31) - 1, 0), (5, (1 << 30) + 7, 77),
             ((1 << 33) + 3, 1, 9), (1, 1 << 31, 3), (3, 715827882, 11), (1 << 40, 1 << 21, 13),
             (1 << 33, (1 << 30) - 1, 21)]
    for n, d, seed in cases:
        m = n * d
        for b in [0, m // 2 - 1000, m - 2000]:
            _say("extreme", n, d, seed, b)
            ref, _ = oracle.edges_range(d, seed, b, 2000)
            if n <= (1 << 32):
                out = ba.generate_range(n, d, seed, b, 2000)
                torch.cuda.synchronize()
                assert np.array_equal(_u32(out), ref.astype(np.uint32).reshape(-1))
            out64 = ba.generate_range_u64(n, d, seed, b, 2000)
            torch.cuda.synchronize()
            assert np.array_equal(_u64(out64), ref.reshape(-1))


def test_range_degrees_starting_and_ending_inside_a_node():
    # a range whose first and last edges are not node boundaries: the first
    # endpoints of the partial nodes count only the edges in the range
    n, d, seed = 20000, 7, 3
    m = n * d
    E, _ = oracle.bb_generate(n, d, seed)
    for b, c in [(3, 1000), (12345, 54321), (m - 5, 5), (6, 1)]:
        _say("partial-node range degrees", b, c)
        deg = torch.zeros(n, dtype=torch.int32, device="cuda")
        out = ba.generate_range(n, d, seed, b, c, deg=deg)
        torch.cuda.synchronize()
        assert np.array_equal(_u32(out), E[2 * b:2 * (b + c)])
        ref = np.bincount(E[2 * b:2 * (b + c)].astype(np.int64), minlength=n)
        assert np.array_equal(_u32(deg).astype(np.int64), ref)


def test_degrees_past_one_window_take_the_partition_kernel():
    # n just above 2^26: 2049 sub-buckets of 32768 nodes, two windows, so the
    # generator writes the target list and the partition kernel sorts it
    n, d, seed = (1 << 26) + 12345, 2, 19
    _say("unfused pipeline", n, d, seed)
    edges, deg = ba.generate(n, d, seed, degrees=True)
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(_u32(edges), E)
    assert np.array_equal(_u32(deg).astype(np.uint64), oracle.count_degrees(E, n))


def test_fused_degrees_on_wide_positions_and_misaligned_output():
    # n <= 2^26 with positions beyond 2^32 (the fused kernel's 64-bit hash),
    # a range across edge 2^31 with accumulated degrees; then a graph whose
    # edge buffer is only 4-byte aligned (the fused kernel's scalar stores)
    n, d, seed = 1 << 21, 1100, 5
    b, c = (1 << 31) - 777777, 1555555
    _say("fused wide range", n, d, seed, b, c)
    deg = torch.zeros(n, dtype=torch.int32, device="cuda")
    ws = ba.workspace(n, d, c)
    out = ba.generate_range(n, d, seed, b, c, deg=deg, ws=ws)
    torch.cuda.synchronize()
    ref, _ = oracle.edges_range(d, seed, b, c)
    ref = ref.astype(np.uint32).reshape(-1)
    assert np.array_equal(_u32(out), ref)
    assert np.array_equal(_u32(deg).astype(np.int64), np.bincount(ref.astype(np.int64), minlength=n))
    n, d, seed = 200003, 7, 31
    _say("fused misaligned", n, d, seed)
    E, _ = oracle.bb_generate(n, d, seed)
    buf = torch.full((2 * n * d + 1,), -1, dtype=torch.int32, device="cuda")
    view = buf[1:]
    _, deg2 = ba.generate(n, d, seed, degrees=True, out=view)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(view), E)
    assert np.array_equal(_u32(deg2).astype(np.uint64), oracle.count_degrees(E, n))


@pytest.mark.parametrize("n,d,seed", [(3, 1 << 20, 4), (100, 100000, 6), (70000, 300, 2)])
def test_stored_degrees_of_very_heavy_nodes(n, d, seed):
    # nodes with far more than 65535 second endpoints in one histogram part:
    # the packed 16-bit counters wrap and the block's counter sum differs
    # from its entry count, so the part goes to deg by global atomics
    _say("heavy stored degrees", n, d, seed)
    edges, deg = ba.generate(n, d, seed, degrees=True)
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(_u32(edges), E)
    ref = oracle.count_degrees(E, n)
    assert ref.max() > 65536
    assert np.array_equal(_u32(deg).astype(np.uint64), ref)
