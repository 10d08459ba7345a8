"""GPU parity of batched generation (many graphs in one persistent launch)
against the CPU oracle, bit-exact: ragged tables, every kernel shape,
misaligned outputs, a wide instance, the full 4096-instance workload in
rounds as bench.py runs it (every instance sampled, 256 of them, the 16
largest among them, compared whole), and replays of a captured HIP graph."""
import random
import sys

import numpy as np
import pytest

import oracle
import workloads
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32).reshape(-1)


def _ragged_table(seed, count):
    rng = random.Random(seed)
    n, d, s = [], [], []
    for j in range(count):
        kind = rng.random()
        if kind < 0.1:
            n.append(0); d.append(rng.randrange(0, 5))
        elif kind < 0.2:
            n.append(1); d.append(rng.randrange(1, 40))
        else:
            n.append(rng.randrange(1, 4000)); d.append(rng.randrange(1, 12))
        s.append(rng.randrange(0, 1 << 64))
    d[3] = 0  # an instance with d = 0 (no edges)
    return n, d, s


def _check_instances(out, n, d, s, off):
    flat = _u32(out)
    for j in range(len(n)):
        m = n[j] * d[j]
        if m == 0:
            continue
        ref, _ = oracle.edges_range(d[j], s[j], 0, m)
        got = flat[int(off[j]):int(off[j]) + 2 * m]
        assert np.array_equal(got, ref.astype(np.uint32).reshape(-1)), "instance %d (n=%d d=%d)" % (j, n[j], d[j])


def test_ragged_batch_every_shape():
    n, d, s = _ragged_table(1, 61)
    b = ba.Batch(n, d, s)
    out = b.empty_output()
    for shape in range(ba.BATCH_SHAPES):
        _say("ragged batch, shape", ba.batch_shape(shape))
        out.fill_(-1)
        b.launch(out, shape=shape)
        torch.cuda.synchronize()
        _check_instances(out, n, d, s, b.out_offset)


def test_batch_with_unaligned_and_reordered_outputs():
    n, d, s = _ragged_table(2, 23)
    m2 = [2 * a * c for a, c in zip(n, d)]
    order = list(range(len(n)))
    random.Random(3).shuffle(order)
    off = [0] * len(n)
    pos = 1  # odd start: 4-byte aligned only
    for j in order:
        off[j] = pos
        pos += m2[j] + 1
    _say("unaligned outputs")
    out = torch.full((pos + 3,), -1, dtype=torch.int32, device="cuda")
    b = ba.Batch(n, d, s, out_offset=off)
    b.launch(out)
    torch.cuda.synchronize()
    _check_instances(out, n, d, s, off)
    flat = _u32(out)
    gaps = [off[j] + m2[j] for j in range(len(n))]
    assert all(flat[g] == 0xFFFFFFFF for g in gaps)  # nothing written between instances


def test_batch_with_a_wide_instance():
    # 2m > 2^32: the 64-bit hash path inside the batch kernel
    n = [5000, (1 << 27) + 3, 17]
    d = [3, 17, 2]
    s = [11, 12, 13]
    b = ba.Batch(n, d, s)
    out = b.empty_output()
    _say("batch with a wide instance", n, d)
    b.launch(out)
    torch.cuda.synchronize()
    flat = out.view(-1)
    m = [a * c for a, c in zip(n, d)]
    for j in (0, 2):
        ref, _ = oracle.edges_range(d[j], s[j], 0, m[j])
        got = flat[int(b.out_offset[j]):int(b.out_offset[j]) + 2 * m[j]].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref.astype(np.uint32).reshape(-1))
    for b0 in [0, (1 << 31) - 1000, m[1] - 4000, 1 << 31]:
        ref, _ = oracle.edges_range(d[1], s[1], b0, 4000)
        lo = int(b.out_offset[1]) + 2 * b0
        got = flat[lo:lo + 8000].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref.astype(np.uint32).reshape(-1))


def test_full_batched_workload_in_rounds():
    n, d, s = workloads.batch_instances()
    round_elems = 1 << 34  # 64 GiB of uint32 per round
    r, off, rounds = ba.batch_plan_rounds(n, d, round_elems)
    assert rounds >= 8
    out = torch.empty(round_elems, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(5)
    # compared whole: the 16 largest instances and 240 others
    m_all = n.astype(np.int64) * d.astype(np.int64)
    largest = np.argsort(-m_all)[:16]
    rest = np.setdiff1d(np.arange(n.size), largest)
    whole = set(largest.tolist()) | set(np.random.default_rng(17).choice(rest, 240, replace=False).tolist())
    assert len(whole) == 256
    compared = 0
    total = 0
    for k in range(rounds):
        js = np.flatnonzero(r == k)
        _say("round", k, "instances", len(js))
        b = ba.Batch(n[js], d[js], s[js], out_offset=off[js])
        if k == 0:
            b.autotune(out)  # as bench.py: the tuned shape for every round
        b.launch(out)
        for j in js:
            if int(j) in whole:
                m = int(m_all[j])
                got = out[int(off[j]):int(off[j]) + 2 * m].cpu().numpy().view(np.uint32)
                ref = oracle_par.edges_u32(int(d[j]), int(s[j]), 0, m)
                if not np.array_equal(got, ref):
                    x = int(np.flatnonzero(got != ref)[0])
                    pytest.fail("instance %d (n=%d d=%d) differs first at element %d" % (j, n[j], d[j], x))
                compared += 1
        # samples: first 32, last 32 and 64 random edges of every instance
        idx, refs = [], []
        for j in js:
            m = int(n[j]) * int(d[j])
            total += m
            for b0 in (0, m - 32):
                ref, _ = oracle.edges_range(int(d[j]), int(s[j]), b0, 32)
                idx.append(int(off[j]) + 2 * b0 + np.arange(64))
                refs.append(ref.astype(np.uint32).reshape(-1))
            for e in rng.integers(0, m, 64):
                u, v, _ = oracle.edge(int(d[j]), int(s[j]), int(e))
                idx.append(int(off[j]) + 2 * int(e) + np.arange(2))
                refs.append(np.array([u, v], dtype=np.uint32))
        sel = torch.from_numpy(np.concatenate(idx).astype(np.int64)).to("cuda")
        got = out[sel].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, np.concatenate(refs)), "round %d" % k
    assert total == int((n.astype(np.float64) * d).sum())
    assert compared == 256


def test_batch_launch_replays_from_a_captured_graph():
    n, d, s = _ragged_table(4, 40)
    b = ba.Batch(n, d, s)
    ref_out = b.empty_output().fill_(-7)  # the padding between instances stays -7 as in the replays
    b.launch(ref_out)
    torch.cuda.synchronize()
    out = b.empty_output()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.launch(out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        b.launch(out)
    for rep in range(3):
        _say("graph replay", rep)
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out)
    _check_instances(out, n, d, s, b.out_offset)
