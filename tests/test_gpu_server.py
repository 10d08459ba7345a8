"""GPU parity of served generation (continuous batching): every result of a
mixed request stream equals the CPU oracle's for that request alone,
bit-exact, under an arena small enough to force many steps, admission waits
and out-of-arena failures; and a slice of the real served trace at full
size (an n=2^27 edge list, first-10^5 degrees on both LDS tiers, 64-bit
positions in edge and degree requests), every result compared whole."""
import sys
import time

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


def _deadline(seconds):
    """A callable that fails the test once `seconds` have passed (a server
    that stops making progress must not hang the run)."""
    end = time.monotonic() + seconds

    def check(srv):
        if time.monotonic() > end:
            pytest.fail("server made no progress for %d s: queued/in flight/arena bytes = %s" % (seconds, srv.stats()))

    return check


def _check_result(srv, t, n, d, seed, kind, k):
    res = srv.result(t)
    m = n * d
    if kind == ba.REQ_EDGES:
        got = res.view(torch.int32).cpu().numpy().view(np.uint32)
        ref, _ = oracle.edges_range(d, seed, 0, m)
        assert np.array_equal(got, ref.astype(np.uint32).reshape(-1)), "edges request %d" % t
    else:
        got = res.view(torch.int64).cpu().numpy().view(np.uint64)
        rdeg, rcs, _ = oracle.stream(d, seed, 0, m, k)
        assert np.array_equal(got[:k], rdeg) and int(got[k]) == rcs, "degrees request %d" % t


def test_served_requests_match_the_oracle_under_a_small_arena():
    tr = workloads.served_trace(count=90, n_lo=1e3, n_hi=3e4, big_frac=0.0, seed=3)
    tr["d"] = np.minimum(tr["d"], 8).astype(np.uint32)
    tr["first_k"] = np.where(tr["kind"] == 1, np.minimum(tr["n"], 700), 0).astype(np.uint64)
    srv = ba.Server(4 << 20)  # 4 MiB: a few requests at a time
    tickets = []
    for j in range(len(tr["n"])):
        n, d, s, kind, k = (int(tr["n"][j]), int(tr["d"][j]), int(tr["seed"][j]), int(tr["kind"][j]),
                            int(tr["first_k"][j]))
        t = srv.submit_edges(n, d, s) if kind == 0 else srv.submit_degrees(n, d, s, k)
        tickets.append((t, n, d, s, kind, k))
    big = srv.submit_edges(1 << 20, 4, 1)  # 32 MiB of edges: never fits
    tail = srv.submit_degrees(5000, 3, 77, 100)  # queued behind the failing one
    _say("served", len(tickets), "requests")
    done, steps, order, times_seen = set(), 0, [], []
    pending = [x[0] for x in tickets] + [big, tail]
    late = _deadline(120)
    while len(done) < len(pending):
        late(srv)
        steps += srv.pump(max_inflight=2) > 0
        for t in srv.completed():
            order.append(t)
            st, ms, _, _ = srv.poll(t)
            if st == ba.JOB_READY:
                if t < len(tickets):
                    times_seen.append(ms)
                if t != tail:
                    _check_result(srv, *tickets[t])
                else:
                    _check_result(srv, tail, 5000, 3, 77, ba.REQ_DEGREES, 100)
                srv.release(t)
            else:
                assert st == ba.JOB_FAILED and t == big
                srv.release(t)  # drops the failed request
            done.add(t)
    assert sorted(order) == sorted(pending) and len(order) == len(pending)
    assert steps >= 3  # the arena forced several continuous-batching steps
    assert srv.stats() == (0, 0, 0)  # nothing queued, in flight or held
    with pytest.raises(ba.BAError):
        srv.poll(tickets[0][0])  # released tickets are gone
    srv.close()


def test_server_validation():
    srv = ba.Server(1 << 20)
    with pytest.raises(ba.BAError):
        srv.submit_edges((1 << 32) + 1, 1, 0)  # uint32 IDs need n <= 2^32
    with pytest.raises(ba.BAError):
        srv.submit_degrees(10, 2, 0, 11)  # first_k > n
    # result sizes that do not fit 64 bits are refused, not wrapped
    with pytest.raises(ba.BAError):
        srv.submit_edges(1 << 32, 1 << 30, 0)  # 8 * 2^62 bytes
    with pytest.raises(ba.BAError):
        srv.submit_degrees(1 << 62, 1, 0, 1 << 61)  # 8 * (2^61 + 1) bytes
    # representable but larger than the arena: fails at admission, launches nothing
    big = srv.submit_degrees(1 << 40, 1, 0, 1 << 40)
    late = _deadline(60)
    while srv.poll(big)[0] != ba.JOB_FAILED:
        late(srv)
        srv.pump()
    srv.release(big)
    t = srv.submit_edges(100, 2, 5)
    with pytest.raises(ba.BAError):
        srv.release(t)  # not ready yet
    while srv.poll(t)[0] != ba.JOB_READY:
        late(srv)
        srv.pump()
    srv.release(t)
    srv.close()


def test_served_trace_slice_at_full_size():
    tr = workloads.served_trace()
    n = tr["n"].astype(np.int64)
    d = tr["d"].astype(np.int64)
    m = n * d
    kind, k = tr["kind"], tr["first_k"].astype(np.int64)

    def first(mask):
        return int(np.flatnonzero(mask)[0])

    picks = {
        "n=2^27 edges": first((n == 1 << 27) & (kind == 0)),
        "n=2^27 degrees (16K tier)": first((n == 1 << 27) & (kind == 1)),
        "degrees, 64-bit positions": first((kind == 1) & (2 * m > 1 << 32) & (m <= 4e9) & (n != 1 << 27)),
        "degrees, 64K tier": first((kind == 1) & (k == 100000) & (n < 5e7) & (n > 2e5)),
        "degrees, first_k = n": first((kind == 1) & (n < 100000)),
        "edges, 64-bit positions": first((kind == 0) & (2 * m > 1 << 32) & (m <= 3e9) & (n != 1 << 27)),
    }
    sel = sorted(set(picks.values()) | set([j for j in range(60) if m[j] <= 1e9][:40]))
    srv = ba.Server(48 << 30)
    ticket_of = {}
    for j in sel:  # arrival order
        if kind[j] == 0:
            t = srv.submit_edges(int(n[j]), int(d[j]), int(tr["seed"][j]))
        else:
            t = srv.submit_degrees(int(n[j]), int(d[j]), int(tr["seed"][j]), int(k[j]))
        ticket_of[t] = j
    _say("served slice", len(sel), "requests", {name: int(j) for name, j in picks.items()})
    done = 0
    late = _deadline(300)
    while done < len(sel):
        late(srv)
        srv.pump(max_inflight=2)
        for t in srv.completed():
            j = ticket_of[t]
            st, _, _, _ = srv.poll(t)
            assert st == ba.JOB_READY, "request %d failed" % j
            res = srv.result(t)
            dj, sj = int(d[j]), int(tr["seed"][j])
            if kind[j] == 0:
                got = res.view(torch.int32).cpu().numpy().view(np.uint32)
                ref = oracle_par.edges_u32(dj, sj, 0, int(m[j]))
                assert np.array_equal(got, ref), "edges request %d (n=%d d=%d)" % (j, n[j], dj)
            else:
                got = res.view(torch.int64).cpu().numpy().view(np.uint64)
                kj = int(k[j])
                rdeg, rcs = oracle_par.stream(dj, sj, 0, int(m[j]), kj)
                assert np.array_equal(got[:kj], rdeg) and int(got[kj]) == rcs, "degrees request %d" % j
            srv.release(t)
            done += 1
    assert srv.stats() == (0, 0, 0)
    srv.close()
