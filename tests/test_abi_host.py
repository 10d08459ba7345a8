"""Host-side checks of libba (no GPU needed): the library loads, exports every
function include/ba.h declares, validates arguments before touching the
device, and its exact divider (used by the kernels for floor(i/d) and
floor(r/(2d))) agrees with integer division."""
import ctypes
import os
import random
import re

import numpy as np
import pytest

import paper_1602_07106_amd as ba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ba.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_\w+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = ba.lib()
    names = _declared()
    assert "ba_generate" in names and "ba_degrees" in names and len(names) >= 8
    for name in names:
        assert hasattr(L, name), name


def test_strerror_covers_every_status():
    L = ba.lib()
    for st in [ba.BA_OK, ba.BA_EINVAL, ba.BA_ERANGE, ba.BA_ENOMEM, ba.BA_EDEVICE, 12345]:
        assert L.ba_strerror(st)
    assert L.ba_strerror(12345) == b"unknown status"


def _host_divide(d, xs):
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
    q = np.zeros_like(x)
    rc = ba.lib().ba_host_divide(d, x.ctypes.data, q.ctypes.data, x.size)
    assert rc == 0
    return [int(v) for v in q]


def _boundary_values(d):
    M = (1 << 64) - 1
    vals = {0, 1, 2, d - 1, d, d + 1, 2 * d - 1, 2 * d, (1 << 31) - 1, 1 << 31, (1 << 32) - 1, 1 << 32,
            (1 << 32) + 1, (1 << 37) - 1, (1 << 63) - 1, 1 << 63, M - 1, M}
    for k in [1, 2, 3, 1000, (1 << 31) // d, (1 << 32) // d, (1 << 63) // d, M // d]:  # tops of both forms
        for delta in (-1, 0, 1):
            vals.add(k * d + delta)
    return sorted(v for v in vals if 0 <= v <= M)


@pytest.mark.parametrize("d", list(range(1, 65)) + [100, 127, 641, 1000003, (1 << 31) - 1, (1 << 31) + 1, (1 << 32) - 1])
def test_exact_division_on_boundaries(d):
    xs = _boundary_values(d)
    assert _host_divide(d, xs) == [x // d for x in xs]


def test_exact_division_random():
    rng = random.Random(5)
    for _ in range(200):
        d = rng.randint(1, (1 << 32) - 1) if rng.random() < 0.5 else rng.randint(1, 200)
        xs = [rng.getrandbits(rng.choice([16, 30, 31, 31, 32, 33, 40, 62, 63, 63, 64])) for _ in range(200)]
        assert _host_divide(d, xs) == [x // d for x in xs]


def test_divide_rejects_zero_divisor():
    x = np.zeros(1, dtype=np.uint64)
    assert ba.lib().ba_host_divide(0, x.ctypes.data, x.ctypes.data, 1) == ba.BA_EINVAL


def _host_mod(xs, bs):
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
    b = np.ascontiguousarray(np.asarray(bs, dtype=np.uint32))
    r = np.zeros(x.size, dtype=np.uint32)
    assert ba.lib().ba_host_mod64(x.ctypes.data, b.ctypes.data, r.ctypes.data, x.size) == 0
    return [int(v) for v in r]


def test_exact_remainder_on_boundaries():
    """x mod b for the CRC hash (64-bit x, 32-bit b): divisors from 1 to
    2^32 - 1, among them those whose float rounding is coarsest (2^24 + 1,
    2^32 - 2^7 - 1: the reciprocal seed's largest error), dividends at
    multiples of b, around 2^53 and up to 2^64 - 1.  The host runs the
    device's algorithm with a seed error larger than the device's."""
    M = (1 << 64) - 1
    divs = [1, 2, 3, 7, 4095, 4096, 4097, (1 << 21) - 1, 1 << 21, (1 << 21) + 1, 1000003, (1 << 24) - 1,
            (1 << 24) + 1, (1 << 24) + 3, (3 << 23) + 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1,
            (1 << 32) - (1 << 7) - 1, (1 << 32) - 3, (1 << 32) - 1]
    xs, bs = [], []
    for b in divs:
        vals = {0, 1, b - 1, b, b + 1, (1 << 32) - 1, 1 << 32, (1 << 53) - 1, 1 << 53, (1 << 53) + 1, M - 1, M}
        for k in [1, 2, (1 << 32) - 1, M // b, (M // b) - 1, ((1 << 53) // b)]:
            for delta in (-1, 0, 1):
                vals.add(k * b + delta)
        for v in sorted(v for v in vals if 0 <= v <= M):
            xs.append(v)
            bs.append(b)
    assert _host_mod(xs, bs) == [x % b for x, b in zip(xs, bs)]


def test_exact_remainder_random():
    rng = random.Random(11)
    xs = [rng.getrandbits(rng.choice([32, 40, 53, 54, 63, 64])) for _ in range(200000)]
    bs = [rng.randint(1, (1 << 32) - 1) if rng.random() < 0.6 else rng.randint(1, 1 << rng.randint(1, 31))
          for _ in range(200000)]
    assert _host_mod(xs, bs) == [x % b for x, b in zip(xs, bs)]


def test_remainder_rejects_zero_divisor():
    x = np.ones(2, dtype=np.uint64)
    b = np.array([3, 0], dtype=np.uint32)
    r = np.zeros(2, dtype=np.uint32)
    assert ba.lib().ba_host_mod64(x.ctypes.data, b.ctypes.data, r.ctypes.data, 2) == ba.BA_EINVAL


# Argument validation returns before any HIP call, so it runs without a GPU.
# Pointer values below are never dereferenced.
FAKE = 1 << 20


def test_generate_rejects_graphs_that_do_not_fit():
    L = ba.lib()
    assert L.ba_generate((1 << 32) + 1, 1, 0, FAKE, None, None) == ba.BA_ERANGE
    assert L.ba_generate(1 << 62, 4, 0, FAKE, None, None) == ba.BA_ERANGE
    assert L.ba_generate_range_u64(1 << 62, 4, 0, 0, 1, FAKE, None) == ba.BA_ERANGE
    assert L.ba_degrees(1 << 62, 4, 0, 1, FAKE, None, None) == ba.BA_ERANGE


def test_generate_rejects_bad_buffers():
    L = ba.lib()
    assert L.ba_generate(10, 2, 0, None, None, None) == ba.BA_EINVAL
    assert L.ba_generate(10, 2, 0, FAKE + 2, None, None) == ba.BA_EINVAL
    assert L.ba_generate(10, 2, 0, FAKE, FAKE + 1, None) == ba.BA_EINVAL
    assert L.ba_generate_range_u64(10, 2, 0, 0, 5, FAKE + 4, None) == ba.BA_EINVAL
    assert L.ba_degrees(10, 2, 0, 5, None, None, None) == ba.BA_EINVAL
    assert L.ba_degrees(10, 2, 0, 5, FAKE + 4, None, None) == ba.BA_EINVAL


def test_ranges_and_first_k_are_checked():
    L = ba.lib()
    assert L.ba_generate_range(10, 2, 0, 15, 6, FAKE, None, None) == ba.BA_EINVAL
    assert L.ba_generate_range(10, 2, 0, 21, 0, FAKE, None, None) == ba.BA_EINVAL
    assert L.ba_generate_range(10, 2, 0, (1 << 64) - 1, 2, FAKE, None, None) == ba.BA_EINVAL
    assert L.ba_degrees(10, 2, 0, 11, FAKE, None, None) == ba.BA_EINVAL
    assert L.ba_degrees_range(10, 2, 0, 0, 21, 5, FAKE, None, None) == ba.BA_EINVAL


def test_empty_work_is_a_no_op():
    L = ba.lib()
    # m = 0 and no degree output: nothing to launch
    assert L.ba_generate(0, 4, 0, None, None, None) == ba.BA_OK
    assert L.ba_generate(10, 0, 0, None, None, None) == ba.BA_OK
    assert L.ba_generate_range(10, 2, 0, 20, 0, None, None, None) == ba.BA_OK
    assert L.ba_generate_range_u64(10, 2, 0, 3, 0, None, None) == ba.BA_OK
    assert L.ba_degrees_range(10, 2, 0, 0, 0, 0, None, None, None) == ba.BA_OK


def test_binding_refuses_cpu_tensors():
    import torch

    with pytest.raises(ValueError):
        ba.generate(10, 2, 0, device="cpu")


def test_timing_kinds_match_header_and_read_empty():
    src = open(HEADER).read()
    kinds = dict((k, int(v)) for k, v in re.findall(r"\bBA_KT_(\w+)\s*=\s*(\d+)", src))
    assert kinds.pop("COUNT") == len(ba.KERNEL_KINDS)
    assert sorted(kinds.values()) == list(range(len(ba.KERNEL_KINDS)))
    for name, idx in kinds.items():
        assert ba.KERNEL_KINDS[idx] == name.lower()
    ba.kernel_timing(True)
    got = ba.kernel_timing_read()  # nothing launched: every kind reads zero
    ba.kernel_timing(False)
    assert got == {k: (0.0, 0) for k in ba.KERNEL_KINDS}
    assert ba.lib().ba_kernel_timing_read(None, None) == ba.BA_EINVAL


def test_batch_round_planning():
    n = [1000, 5, 0, 7, 300, 2]
    d = [3, 2, 4, 1, 2, 9]
    r, o, k = ba.batch_plan_rounds(n, d, 7000)
    m2 = [2 * a * b for a, b in zip(n, d)]
    assert k == 2 and r.tolist() == [0, 0, 0, 0, 1, 1]
    assert all(int(x) % 4 == 0 for x in o)  # 16-byte aligned starts
    for rr in range(k):  # inside a round: in order, disjoint, within the budget
        js = [j for j in range(len(n)) if r[j] == rr]
        for a, b in zip(js, js[1:]):
            assert int(o[a]) + m2[a] <= int(o[b])
        assert int(o[js[-1]]) + m2[js[-1]] <= 7000
    with pytest.raises(ba.BAError):
        ba.batch_plan_rounds([1000], [3], 5999)  # one instance bigger than a round
    with pytest.raises(ba.BAError):
        ba.batch_plan_rounds([(1 << 32) + 1], [1], 1 << 40)  # uint32 IDs need n <= 2^32
    assert ba.batch_plan_rounds([], [], 10)[2] == 0


def test_batch_host_validation_without_gpu():
    L = ba.lib()
    info = ba.BatchInfo()
    assert L.ba_batch_upload(0, None, None, None, None, None, 0, ctypes.addressof(info), None) == ba.BA_OK
    assert info.count == 0 and info.edges_len == 0
    assert L.ba_batch_launch(ctypes.addressof(info), None, None, 0, None) == ba.BA_OK  # empty batch: no-op
    assert L.ba_batch_upload(1, None, None, None, None, None, 0, ctypes.addressof(info), None) == ba.BA_EINVAL
    nn = np.array([(1 << 32) + 1], dtype=np.uint64)
    dd = np.array([1], dtype=np.uint32)
    ss = np.array([0], dtype=np.uint64)
    oo = np.array([0], dtype=np.uint64)
    # a workspace that is too small is refused before any device work
    assert L.ba_batch_upload(1, nn.ctypes.data, dd.ctypes.data, ss.ctypes.data, oo.ctypes.data, 256, 1,
                             ctypes.addressof(info), None) == ba.BA_EINVAL
    assert L.ba_batch_workspace_bytes(4096) >= 4096 * 64 + 3 * 4097 * 8
    assert L.ba_batch_launch_shape(ctypes.addressof(info), None, None, 0, 5, None) == ba.BA_EINVAL
    assert [ba.batch_shape(k)[1:] for k in range(ba.BATCH_SHAPES)] == [(1024, 4), (2048, 4), (4096, 4), (1024, 8),
                                                                       (2048, 8)]


def test_model_argument_checks_without_gpu():
    L = ba.lib()
    # unknown flag, n0 > n, no-self-loops without a seed edge, range past the new edges
    assert L.ba_generate_model(100, 2, 1, 0, 0, None, 4, 0, 1, 16, None) == ba.BA_EINVAL
    assert L.ba_generate_model(100, 2, 1, 101, 0, None, 0, 0, 0, None, None) == ba.BA_EINVAL
    assert L.ba_generate_model(100, 2, 1, 0, 0, None, ba.NO_SELF_LOOPS, 0, 1, 16, None) == ba.BA_EINVAL
    assert L.ba_generate_model(100, 2, 1, 10, 0, None, 0, 180, 1, 16, None) == ba.BA_EINVAL
    assert L.ba_generate_model(100, 2, 1, 10, 3, None, 0, 0, 1, 16, None) == ba.BA_EINVAL  # seed edges missing
    assert L.ba_generate_model((1 << 32) + 1, 1, 1, 0, 0, None, 0, 0, 0, None, None) == ba.BA_ERANGE
    assert L.ba_generate_model(100, 2, 1, 10, 0, None, 0, 5, 0, None, None) == ba.BA_OK  # empty range


def test_streaming_tier_is_checked_per_call():
    L = ba.lib()
    for bad in (1, 32, -1, 65):
        assert L.ba_degrees_range_tier(10, 2, 0, 0, 20, 5, FAKE, None, bad, None) == ba.BA_EINVAL
    # valid tiers on empty work: nothing to launch
    for t in (ba.TIER_AUTO, ba.TIER_16K, ba.TIER_64K):
        assert L.ba_degrees_range_tier(10, 2, 0, 0, 0, 0, None, None, t, None) == ba.BA_OK


def test_uint32_degrees_that_could_wrap_are_refused():
    # node v holds d first endpoints plus at most m - d*v second endpoints:
    # counts stay below 2^32 only while n*d + d < 2^32
    L = ba.lib()
    assert L.ba_generate(1, 1 << 31, 0, FAKE, FAKE, None) == ba.BA_ERANGE
    assert L.ba_generate(3, (1 << 31) - 1, 0, FAKE, FAKE, None) == ba.BA_ERANGE
    assert L.ba_generate_range(3, (1 << 31) - 1, 0, 0, 1, FAKE, FAKE, None) == ba.BA_ERANGE
    assert L.ba_generate_ws(1 << 20, 1 << 12, 0, FAKE, FAKE, FAKE, 1 << 40, None) == ba.BA_ERANGE


def test_workspace_too_small_is_enomem_and_bad_pointers_einval():
    L = ba.lib()
    n, d = 1 << 20, 4
    need = ba.workspace_bytes(n, d, n * d)
    assert need > 0
    assert L.ba_generate_ws(n, d, 0, FAKE, FAKE, FAKE, 1000, None) == ba.BA_ENOMEM
    assert L.ba_generate_range_ws(n, d, 0, 5, 1 << 20, FAKE, FAKE, FAKE, 1000, None) == ba.BA_ENOMEM
    assert L.ba_generate_ws(n, d, 0, FAKE, FAKE, None, need, None) == ba.BA_EINVAL
    assert L.ba_generate_ws(n, d, 0, FAKE, FAKE, FAKE + 4, need, None) == ba.BA_EINVAL


def test_static_scratch_too_small_is_enomem_before_any_device_call():
    # n = 2^28 needs more than the static scratch for a single 2^20-edge pass
    # (every region of its 8192 sub-buckets costs slack); without deg no
    # scratch is used, and argument errors come first
    L = ba.lib()
    assert L.ba_generate_static(1 << 28, 1, 0, FAKE, FAKE, None) == ba.BA_ENOMEM
    assert L.ba_generate_static(240_000_000, 2, 0, FAKE, FAKE, None) == ba.BA_ENOMEM
    assert L.ba_generate_static(1, 1 << 31, 0, FAKE, FAKE, None) == ba.BA_ERANGE
    assert L.ba_generate_static(10, 2, 0, None, FAKE, None) == ba.BA_EINVAL
    assert L.ba_generate_static(10, 2, 0, FAKE, FAKE + 2, None) == ba.BA_EINVAL
    assert L.ba_generate_static(0, 4, 0, None, None, None) == ba.BA_OK
