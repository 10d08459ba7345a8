"""ba_generate_static (the whole graph and its degrees with the degree
pipeline's workspace in the library's static device scratch, no allocation)
against ba_generate_ws with a caller workspace: bit-exact, on two calls in a
row, the second with a smaller graph, and without any device allocation;
then captured into a HIP graph and replayed, with eager calls on the same
scratch between the replays."""
import ctypes
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


def _pool():
    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    return hip, pool


def _pool_high(hip, pool):
    v = ctypes.c_uint64(0)
    assert hip.hipMemPoolGetAttribute(pool, 8, ctypes.byref(v)) == 0  # hipMemPoolAttrUsedMemHigh
    return v.value


def _reference(n, d, seed):
    """Edges and degrees from ba_generate_ws with a whole workspace."""
    m = n * d
    edges = torch.empty(2 * m, dtype=torch.int32, device="cuda")
    deg = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = ba.workspace(n, d, m)
    st = torch.cuda.current_stream().cuda_stream
    assert ba.lib().ba_generate_ws(n, d, seed, edges.data_ptr(), deg.data_ptr(), ws.data_ptr(), ws.numel(), st) == 0
    torch.cuda.synchronize()
    del ws
    return edges, deg


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ba.lib()
    yield
    torch.cuda.synchronize()


def test_static_scratch_matches_the_workspace_call_twice_in_a_row():
    L = ba.lib()
    st = torch.cuda.current_stream().cuda_stream
    hip, pool = _pool()
    # first the 2^26-node, d = 16 graph (48 passes through the scratch), then
    # a smaller one with a ragged tail: the second call runs over what the
    # first left in the scratch
    for n, d, seed in [(1 << 26, 16, 7), (100003, 5, 3)]:
        _say("static scratch", n, d, seed)
        ref_e, ref_deg = _reference(n, d, seed)
        m = n * d
        edges = torch.full((2 * m,), -1, dtype=torch.int32, device="cuda")
        deg = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        zero = ctypes.c_uint64(0)
        assert hip.hipMemPoolSetAttribute(pool, 8, ctypes.byref(zero)) == 0  # reset the high-water mark
        free0 = torch.cuda.mem_get_info()[0]
        assert L.ba_generate_static(n, d, seed, edges.data_ptr(), deg.data_ptr(), st) == 0
        torch.cuda.synchronize()
        assert _pool_high(hip, pool) == 0
        assert torch.cuda.mem_get_info()[0] == free0
        assert torch.equal(edges, ref_e)
        assert torch.equal(deg, ref_deg)
        if m <= 1_000_000:
            E, _ = oracle.bb_generate(n, d, seed)
            assert np.array_equal(edges.cpu().numpy().view(np.uint32), E)
            assert np.array_equal(deg.cpu().numpy().view(np.uint32).astype(np.uint64), oracle.count_degrees(E, n))
        del ref_e, ref_deg, edges, deg


def test_static_without_degrees_and_refusals():
    L = ba.lib()
    st = torch.cuda.current_stream().cuda_stream
    n, d, seed = 50000, 3, 11
    _say("static no deg", n, d, seed)
    edges = torch.empty(2 * n * d, dtype=torch.int32, device="cuda")
    assert L.ba_generate_static(n, d, seed, edges.data_ptr(), None, st) == 0
    torch.cuda.synchronize()
    E, _ = oracle.bb_generate(n, d, seed)
    assert np.array_equal(edges.cpu().numpy().view(np.uint32), E)
    # a graph whose single smallest pass exceeds the scratch: refused on the
    # host, nothing launched, outputs untouched
    small = torch.full((16,), 7, dtype=torch.int32, device="cuda")
    assert L.ba_generate_static(1 << 28, 1, 0, small.data_ptr(), small.data_ptr(), st) == ba.BA_ENOMEM
    torch.cuda.synchronize()
    assert int((small != 7).sum()) == 0


def test_static_entry_point_replays_from_a_captured_graph():
    L = ba.lib()
    # 2^28 edges: the degree pipeline needs several passes through the
    # 256 MiB scratch, so the graph holds every pass's launches
    n, d, seed = (1 << 24) + 77, 16, 13
    m = n * d
    _say("static graph capture", n, d, seed)
    ref_e = torch.empty(2 * m, dtype=torch.int32, device="cuda")
    ref_d = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = ba.workspace(n, d, m)
    st = torch.cuda.current_stream().cuda_stream
    assert L.ba_generate_ws(n, d, seed, ref_e.data_ptr(), ref_d.data_ptr(), ws.data_ptr(), ws.numel(), st) == 0
    torch.cuda.synchronize()
    del ws
    edges = torch.full((2 * m,), -1, dtype=torch.int32, device="cuda")
    deg = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    # an eager call first: the scratch's address is looked up once per device
    assert L.ba_generate_static(n, d, seed, edges.data_ptr(), deg.data_ptr(), st) == 0
    torch.cuda.synchronize()
    assert torch.equal(edges, ref_e) and torch.equal(deg, ref_d)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rc = L.ba_generate_static(n, d, seed, edges.data_ptr(), deg.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    other_e = torch.empty(2 * 99991 * 7, dtype=torch.int32, device="cuda")
    other_d = torch.empty(99991, dtype=torch.int32, device="cuda")
    for rep in range(3):
        _say("replay", rep)
        edges.fill_(-1)
        deg.fill_(-1)
        # eager work on the same scratch between replays
        assert L.ba_generate_static(99991, 7, rep, other_e.data_ptr(), other_d.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream) == 0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(edges, ref_e), rep
        assert torch.equal(deg, ref_d), rep
    del g
