"""Barabasi-Albert graph generation by per-edge recomputation on MI355X.

Thin Python binding over libba.so (C ABI in include/ba.h).  Every step of the
generator runs in the library's HIP kernels; this module only allocates torch
device tensors, passes their pointers and the current HIP stream, and turns
status codes into exceptions.  There is no CPU fallback: without the built
library every call raises.

The graph (Sanders & Schulz, arXiv:1602.07106, Section 2): n nodes, d edges
per node, empty seed graph, self-loops and parallel edges allowed.  Edge i is
(floor(i/d), E[2i+1]) where E[2i+1] follows r = 2i+1, r = h(r), ... until r is
even and is floor(r/(2d)); h(r) = umul64hi(fmix64(r ^ seed*phi64), r).

Tensors: node IDs of the uint32 paths are returned in int32 tensors holding
the uint32 bit patterns (identical values for n <= 2^31); uint64 results
(64-bit IDs, degrees, checksums) are returned in int64 tensors holding the
uint64 bit patterns.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

from . import build as _build

__all__ = [
    "BAError",
    "KERNEL_KINDS",
    "workspace",
    "workspace_bytes",
    "generate",
    "generate_range",
    "generate_range_u64",
    "kernel_timing",
    "kernel_timing_read",
    "degrees",
    "degrees_range",
    "Batch",
    "batch_plan_rounds",
    "batch_shape",
    "generate_batch",
    "Server",
    "generate_model",
    "lib",
    "library_path",
]

BA_OK, BA_EINVAL, BA_ERANGE, BA_ENOMEM, BA_EDEVICE = 0, -1, -2, -3, -4
# kernel kinds of the timing hook (BA_KT_* in include/ba.h)
KERNEL_KINDS = ("gen", "part", "hist", "stream", "other")


class BAError(RuntimeError):
    def __init__(self, fn: str, status: int):
        L = lib()
        msg = L.ba_strerror(status).decode()
        if status == BA_EDEVICE:
            msg += " (hipError_t %d)" % L.ba_last_hip_error()
        super().__init__("%s: %s" % (fn, msg))
        self.status = status


_u64, _u32, _p, _int = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
_SIGS = {
    "ba_generate": (_int, [_u64, _u32, _u64, _p, _p, _p]),
    "ba_generate_range": (_int, [_u64, _u32, _u64, _u64, _u64, _p, _p, _p]),
    "ba_generate_ws": (_int, [_u64, _u32, _u64, _p, _p, _p, _u64, _p]),
    "ba_generate_range_ws": (_int, [_u64, _u32, _u64, _u64, _u64, _p, _p, _p, _u64, _p]),
    "ba_generate_workspace_bytes": (_u64, [_u64, _u32, _u64]),
    "ba_generate_static": (_int, [_u64, _u32, _u64, _p, _p, _p]),
    "ba_test_generate_ws_scaled": (_int, [_u64, _u32, _u64, _p, _p, _p, _u64, ctypes.c_double, _p]),
    "ba_generate_range_u64": (_int, [_u64, _u32, _u64, _u64, _u64, _p, _p]),
    "ba_degrees": (_int, [_u64, _u32, _u64, _u64, _p, _p, _p]),
    "ba_degrees_range": (_int, [_u64, _u32, _u64, _u64, _u64, _u64, _p, _p, _p]),
    "ba_degrees_range_tier": (_int, [_u64, _u32, _u64, _u64, _u64, _u64, _p, _p, _int, _p]),
    "ba_strerror": (ctypes.c_char_p, [_int]),
    "ba_last_hip_error": (_int, []),
    "ba_host_divide": (_int, [_u32, _p, _p, _u64]),
    "ba_host_mod64": (_int, [_p, _p, _p, _u64]),
    "ba_kernel_timing": (_int, [_int]),
    "ba_kernel_timing_read": (_int, [_p, _p]),
    "ba_batch_workspace_bytes": (_u64, [_u32]),
    "ba_batch_upload": (_int, [_u32, _p, _p, _p, _p, _p, _u64, _p, _p]),
    "ba_batch_launch": (_int, [_p, _p, _p, _u64, _p]),
    "ba_batch_autotune": (_int, [_p, _p, _p, _u64, _p, _p]),
    "ba_batch_launch_shape": (_int, [_p, _p, _p, _u64, _int, _p]),
    "ba_batch_current_shape": (_int, [_p]),
    "ba_batch_shape_dims": (_int, [_int, _p, _p]),
    "ba_batch_plan_rounds": (_int, [_u32, _p, _p, _u64, _p, _p, _p]),
    "ba_generate_model": (_int, [_u64, _u32, _u64, _u64, _u64, _p, _u32, _u64, _u64, _p, _p]),
    "ba_server_create": (_int, [_p, _u64, _p, _p]),
    "ba_server_destroy": (_int, [_p]),
    "ba_server_submit": (_int, [_p, _p, _p]),
    "ba_server_pump": (_int, [_p, _u32, _p]),
    "ba_server_poll": (_int, [_p, _u64, _p, _p, _p, _p]),
    "ba_server_completed": (_int, [_p, _p, _u32, _p]),
    "ba_server_release": (_int, [_p, _u64]),
    "ba_server_stats": (_int, [_p, _p, _p, _p]),
}

_lib = None


def library_path() -> str:
    return _build.LIB


def lib() -> ctypes.CDLL:
    """The loaded libba.so (built first if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(fn: str, status: int) -> None:
    if status != BA_OK:
        raise BAError(fn, status)


def _ptr(t: Optional[torch.Tensor], dev: Optional[torch.device] = None) -> Optional[int]:
    """t's device address; t must be a contiguous device tensor (on dev, when given)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dev is not None:
        want = dev.index if dev.index is not None else torch.cuda.current_device()
        if t.device.index != want:
            raise ValueError(f"expected a tensor on cuda:{want}, got one on {t.device}")
    return t.data_ptr()


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _device(device) -> torch.device:
    dev = torch.device("cuda" if device is None else device)
    if dev.type != "cuda":
        raise ValueError("the generator runs on the GPU only")
    return dev


def workspace_bytes(n: int, d: int, edge_count: int) -> int:
    """Device workspace the degree pipeline needs for edge_count edges."""
    return int(lib().ba_generate_workspace_bytes(n, d, edge_count))


def workspace(n: int, d: int, edge_count: int, device=None) -> torch.Tensor:
    """A uint8 device tensor large enough for :func:`workspace_bytes`."""
    return torch.empty(max(1, workspace_bytes(n, d, edge_count)), dtype=torch.uint8, device=_device(device))


def _ws_arg(ws: Optional[torch.Tensor], n: int, d: int, count: int, dev: torch.device):
    if ws is None:
        ws = workspace(n, d, count, dev)
    if ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor")
    return ws, ws.numel()


def generate(
    n: int,
    d: int,
    seed: int,
    *,
    degrees: bool = False,
    out: Optional[torch.Tensor] = None,
    deg_out: Optional[torch.Tensor] = None,
    ws: Optional[torch.Tensor] = None,
    device=None,
) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    """Whole edge list of (n, d, seed) as int32[n*d, 2] (uint32 IDs), and the
    degree array int32[n] (uint32 counts) when ``degrees``.  ``out`` /
    ``deg_out`` may supply preallocated contiguous int32 tensors, ``ws`` the
    degree pipeline's workspace (see :func:`workspace`)."""
    dev = _device(device if out is None else out.device)
    m = n * d
    if out is None:
        out = torch.empty((m, 2), dtype=torch.int32, device=dev)
    elif out.dtype != torch.int32 or out.numel() != 2 * m:
        raise ValueError("out must be int32 with 2*n*d elements")
    deg = None
    if degrees:
        deg = deg_out if deg_out is not None else torch.empty(n, dtype=torch.int32, device=dev)
        if deg.dtype != torch.int32 or deg.numel() != n:
            raise ValueError("deg_out must be int32 with n elements")
    with torch.cuda.device(dev):
        if deg is None:
            _check("ba_generate", lib().ba_generate(n, d, seed, _ptr(out, dev), None, _stream(dev)))
        else:
            w, wb = _ws_arg(ws, n, d, m, dev)
            _check(
                "ba_generate_ws",
                lib().ba_generate_ws(n, d, seed, _ptr(out, dev), _ptr(deg, dev), _ptr(w, dev), wb, _stream(dev)),
            )
    return out, deg


def generate_range(
    n: int,
    d: int,
    seed: int,
    begin: int,
    count: int,
    *,
    deg: Optional[torch.Tensor] = None,
    out: Optional[torch.Tensor] = None,
    ws: Optional[torch.Tensor] = None,
    device=None,
) -> torch.Tensor:
    """Edges begin..begin+count-1 as int32[count, 2].  When ``deg`` (int32[n])
    is given, both endpoints of every edge in the range are added to it."""
    dev = _device(device if out is None else out.device)
    if out is None:
        out = torch.empty((count, 2), dtype=torch.int32, device=dev)
    elif out.dtype != torch.int32 or out.numel() != 2 * count:
        raise ValueError("out must be int32 with 2*count elements")
    if deg is not None and (deg.dtype != torch.int32 or deg.numel() != n):
        raise ValueError("deg must be int32 with n elements")
    with torch.cuda.device(dev):
        if deg is None:
            _check(
                "ba_generate_range",
                lib().ba_generate_range(n, d, seed, begin, count, _ptr(out, dev), None, _stream(dev)),
            )
        else:
            w, wb = _ws_arg(ws, n, d, count, dev)
            _check(
                "ba_generate_range_ws",
                lib().ba_generate_range_ws(n, d, seed, begin, count, _ptr(out, dev), _ptr(deg, dev), _ptr(w, dev), wb,
                                           _stream(dev)),
            )
    return out


def kernel_timing(enable: bool) -> None:
    """Start (or stop) recording HIP events around every kernel launched by
    this thread's calls (see ba_kernel_timing)."""
    _check("ba_kernel_timing", lib().ba_kernel_timing(1 if enable else 0))


def kernel_timing_read() -> Dict[str, Tuple[float, int]]:
    """{kind: (summed kernel milliseconds, launches)} since the last read,
    for every kind in KERNEL_KINDS."""
    k = len(KERNEL_KINDS)
    ms, n = (ctypes.c_double * k)(), (ctypes.c_uint64 * k)()
    _check("ba_kernel_timing_read", lib().ba_kernel_timing_read(ctypes.addressof(ms), ctypes.addressof(n)))
    return {name: (ms[i], n[i]) for i, name in enumerate(KERNEL_KINDS)}


def generate_range_u64(n: int, d: int, seed: int, begin: int, count: int, *, device=None) -> torch.Tensor:
    """Edges begin..begin+count-1 with 64-bit IDs as int64[count, 2]."""
    dev = _device(device)
    out = torch.empty((count, 2), dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _check(
            "ba_generate_range_u64",
            lib().ba_generate_range_u64(n, d, seed, begin, count, _ptr(out, dev), _stream(dev)),
        )
    return out


TIER_AUTO, TIER_16K, TIER_64K = 0, 16, 64


def degrees(n: int, d: int, seed: int, first_k: int, *, tier: int = TIER_AUTO,
            device=None) -> Tuple[torch.Tensor, int]:
    """Streaming degrees of nodes 0..first_k-1 (int64[first_k]) and the edge
    XOR checksum (a Python int in 0..2^64-1); no edge is stored.  ``tier``
    picks the streaming kernel's LDS counter tier (TIER_AUTO, TIER_16K or
    TIER_64K; the result is the same on every tier)."""
    dev = _device(device)
    with torch.cuda.device(dev):
        if tier == TIER_AUTO:
            deg = torch.empty(first_k, dtype=torch.int64, device=dev)
            cs = torch.empty(1, dtype=torch.int64, device=dev)
            _check("ba_degrees", lib().ba_degrees(n, d, seed, first_k, _ptr(deg, dev), _ptr(cs, dev), _stream(dev)))
        else:
            deg = torch.zeros(first_k, dtype=torch.int64, device=dev)
            cs = torch.zeros(1, dtype=torch.int64, device=dev)
            _check("ba_degrees_range_tier",
                   lib().ba_degrees_range_tier(n, d, seed, 0, n * d, first_k, _ptr(deg, dev), _ptr(cs, dev), tier,
                                               _stream(dev)))
    return deg, int(cs.item()) & ((1 << 64) - 1)


def degrees_range(
    n: int,
    d: int,
    seed: int,
    begin: int,
    count: int,
    first_k: int,
    deg: torch.Tensor,
    cs: Optional[torch.Tensor] = None,
    *,
    tier: int = TIER_AUTO,
) -> None:
    """Accumulating form of :func:`degrees` over edges begin..begin+count-1:
    adds endpoint counts into ``deg`` (int64[first_k]) and XORs the edge words
    into ``cs`` (int64[1]) when given."""
    dev = deg.device
    if deg.dtype != torch.int64 or deg.numel() != first_k:
        raise ValueError("deg must be int64 with first_k elements")
    if cs is not None and (cs.dtype != torch.int64 or cs.numel() != 1):
        raise ValueError("cs must be int64 with one element")
    with torch.cuda.device(dev):
        _check(
            "ba_degrees_range_tier",
            lib().ba_degrees_range_tier(n, d, seed, begin, count, first_k, _ptr(deg, dev), _ptr(cs, dev), tier,
                                        _stream(dev)),
        )


class BatchInfo(ctypes.Structure):
    """ba_batch_info of include/ba.h."""

    _fields_ = [
        ("count", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("tiles", ctypes.c_uint64 * 3),
        ("edges_len", ctypes.c_uint64),
    ]


def _table(n: Sequence[int], d: Sequence[int], seed: Optional[Sequence[int]] = None):
    nn = np.ascontiguousarray(np.asarray(n, dtype=np.uint64))
    dd = np.ascontiguousarray(np.asarray(d, dtype=np.uint32))
    if nn.shape != dd.shape or nn.ndim != 1:
        raise ValueError("n and d must be 1-D and of equal length")
    ss = None
    if seed is not None:
        ss = np.ascontiguousarray(np.asarray(seed, dtype=np.uint64))
        if ss.shape != nn.shape:
            raise ValueError("seed must match n")
    return nn, dd, ss


def batch_plan_rounds(n: Sequence[int], d: Sequence[int], round_elems: int) -> Tuple[np.ndarray, np.ndarray, int]:
    """(round_of, offset_of, rounds): the instances, in order, packed into
    rounds whose edge outputs fit round_elems uint32 each (see
    ba_batch_plan_rounds).  Also the packed layout of a single round."""
    nn, dd, _ = _table(n, d)
    r = np.zeros(nn.size, dtype=np.uint32)
    o = np.zeros(nn.size, dtype=np.uint64)
    k = ctypes.c_uint32(0)
    _check("ba_batch_plan_rounds", lib().ba_batch_plan_rounds(nn.size, nn.ctypes.data, dd.ctypes.data, round_elems,
                                                                r.ctypes.data, o.ctypes.data, ctypes.addressof(k)))
    return r, o, k.value


class Batch:
    """A table of instances (n[j], d[j], seed[j]) uploaded to the device.
    Instance j writes its uint32 edge pairs at out_offset[j] (uint32
    elements) of the output; by default the instances are packed in order,
    each 16-byte aligned."""

    def __init__(self, n, d, seed, out_offset=None, device=None):
        nn, dd, ss = _table(n, d, seed)
        if out_offset is None:
            _, out_offset, _ = batch_plan_rounds(nn, dd, (1 << 64) - 1)
        oo = np.ascontiguousarray(np.asarray(out_offset, dtype=np.uint64))
        if oo.shape != nn.shape:
            raise ValueError("out_offset must match n")
        self.count = nn.size
        self.out_offset = oo
        self.ws = torch.empty(max(1, int(lib().ba_batch_workspace_bytes(self.count))), dtype=torch.uint8,
                              device=_device(device))
        self.device = self.ws.device  # with its index
        self.info = BatchInfo()
        with torch.cuda.device(self.device):
            _check("ba_batch_upload",
                   lib().ba_batch_upload(self.count, nn.ctypes.data, dd.ctypes.data, ss.ctypes.data, oo.ctypes.data,
                                         self.ws.data_ptr(), self.ws.numel(), ctypes.addressof(self.info),
                                         _stream(self.device)))
        self.edges_len = int(self.info.edges_len)

    def empty_output(self) -> torch.Tensor:
        return torch.empty(max(1, self.edges_len), dtype=torch.int32, device=self.device)

    def _out(self, out: torch.Tensor) -> Tuple[int, int]:
        if out.dtype != torch.int32 or out.device != self.device or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor on the batch's device")
        return out.data_ptr(), out.numel()

    def launch(self, out: torch.Tensor, shape: Optional[int] = None) -> torch.Tensor:
        """Every instance's edges into out (int32, at least edges_len), with
        the device's tuned kernel shape or an explicit one."""
        p, ln = self._out(out)
        with torch.cuda.device(self.device):
            if shape is None:
                _check("ba_batch_launch", lib().ba_batch_launch(ctypes.addressof(self.info), self.ws.data_ptr(), p, ln,
                                                                _stream(self.device)))
            else:
                _check("ba_batch_launch_shape",
                       lib().ba_batch_launch_shape(ctypes.addressof(self.info), self.ws.data_ptr(), p, ln, shape,
                                                   _stream(self.device)))
        return out

    def autotune(self, out: torch.Tensor) -> int:
        """Time every kernel shape on this batch and keep the fastest for the
        device (see ba_batch_autotune); returns the chosen shape index."""
        p, ln = self._out(out)
        shape = ctypes.c_int(-1)
        with torch.cuda.device(self.device):
            _check("ba_batch_autotune", lib().ba_batch_autotune(ctypes.addressof(self.info), self.ws.data_ptr(), p, ln,
                                                                ctypes.addressof(shape), _stream(self.device)))
        return shape.value


BATCH_SHAPES = 5


def batch_shape(shape: Optional[int] = None) -> Tuple[int, int, int]:
    """(index, tile edges, waves per block) of a kernel shape; by default the
    one ba_batch_launch uses on the current device."""
    if shape is None:
        k = ctypes.c_int(0)
        _check("ba_batch_current_shape", lib().ba_batch_current_shape(ctypes.addressof(k)))
        shape = k.value
    t, w = ctypes.c_int(0), ctypes.c_int(0)
    _check("ba_batch_shape_dims", lib().ba_batch_shape_dims(shape, ctypes.addressof(t), ctypes.addressof(w)))
    return shape, t.value, w.value


def generate_batch(n, d, seed, *, out_offset=None, out: Optional[torch.Tensor] = None, device=None):
    """(edges, out_offset): every instance's uint32 edge pairs in one int32
    tensor, instance j at out_offset[j] (packed by default)."""
    b = Batch(n, d, seed, out_offset, device if out is None else out.device)
    if out is None:
        out = b.empty_output()
    b.launch(out)
    return out, b.out_offset


REQ_EDGES, REQ_DEGREES = 0, 1
JOB_QUEUED, JOB_RUNNING, JOB_READY, JOB_FAILED, JOB_RELEASED = 0, 1, 2, 3, 4


class Request(ctypes.Structure):
    """ba_request of include/ba.h."""

    _fields_ = [
        ("n", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("first_k", ctypes.c_uint64),
        ("d", ctypes.c_uint32),
        ("kind", ctypes.c_uint32),
    ]


class Server:
    """Continuous batching of generation requests (see ba_server_* in
    include/ba.h): edge batches on `stream`, degree batches on a stream of
    the server's own.  Results live in a device arena of arena_bytes until
    released, and are valid once their ticket is ready."""

    def __init__(self, arena_bytes: int, device=None, stream: Optional[torch.cuda.Stream] = None):
        dev = _device(device)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
        self.device = self.arena.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check("ba_server_create", lib().ba_server_create(self.arena.data_ptr(), arena_bytes,
                                                              self.stream.cuda_stream, ctypes.addressof(h)))
        self._h = h

    def close(self) -> None:
        if self._h:
            _check("ba_server_destroy", lib().ba_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_edges(self, n: int, d: int, seed: int) -> int:
        return self._submit(Request(n, seed, 0, d, REQ_EDGES))

    def submit_degrees(self, n: int, d: int, seed: int, first_k: int) -> int:
        return self._submit(Request(n, seed, first_k, d, REQ_DEGREES))

    def _submit(self, r: Request) -> int:
        t = ctypes.c_uint64(0)
        _check("ba_server_submit", lib().ba_server_submit(self._h, ctypes.addressof(r), ctypes.addressof(t)))
        return t.value

    def pump(self, max_inflight: int = 2) -> int:
        """Retire finished steps; launch one more when fewer than max_inflight
        are in flight.  Returns the number of requests admitted."""
        k = ctypes.c_uint32(0)
        with torch.cuda.device(self.device):
            _check("ba_server_pump", lib().ba_server_pump(self._h, max_inflight, ctypes.addressof(k)))
        return k.value

    def poll(self, ticket: int):
        """(state, done_ms, offset, bytes) of a ticket."""
        st, ms, off, nb = ctypes.c_int(0), ctypes.c_double(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check("ba_server_poll", lib().ba_server_poll(self._h, ticket, ctypes.addressof(st), ctypes.addressof(ms),
                                                      ctypes.addressof(off), ctypes.addressof(nb)))
        return st.value, ms.value, off.value, nb.value

    def completed(self, capacity: int = 4096):
        """Tickets that became ready or failed since the last call."""
        buf = (ctypes.c_uint64 * capacity)()
        k = ctypes.c_uint32(0)
        _check("ba_server_completed", lib().ba_server_completed(self._h, ctypes.addressof(buf), capacity,
                                                                ctypes.addressof(k)))
        return [buf[i] for i in range(k.value)]

    def result(self, ticket: int) -> torch.Tensor:
        """A ready result as a view into the arena: int32[2m] edge pairs or
        int64[first_k + 1] (degrees, then the checksum)."""
        st, _, off, nb = self.poll(ticket)
        if st != JOB_READY:
            raise BAError("ba_server_poll", BA_EINVAL)
        return self.arena[off:off + nb]

    def release(self, ticket: int) -> None:
        _check("ba_server_release", lib().ba_server_release(self._h, ticket))

    def stats(self):
        q, i, u = ctypes.c_uint64(0), ctypes.c_uint32(0), ctypes.c_uint64(0)
        _check("ba_server_stats", lib().ba_server_stats(self._h, ctypes.addressof(q), ctypes.addressof(i),
                                                        ctypes.addressof(u)))
        return q.value, i.value, u.value


NO_SELF_LOOPS, HASH_CRC = 1, 2


def generate_model(n: int, d: int, seed: int, *, n0: int = 0, seed_edges: Optional[torch.Tensor] = None,
                   no_self_loops: bool = False, hash: str = "fmix", begin: int = 0, count: Optional[int] = None,
                   out: Optional[torch.Tensor] = None, device=None) -> torch.Tensor:
    """New edges begin..begin+count-1 of the generalized model (see
    ba_generate_model) as int32[count, 2]: a seed graph of n0 nodes whose
    edges are the int32 device tensor seed_edges (2*m0 IDs), optional
    self-loop-free draws, and the fmix or the paper's crc hash."""
    if hash not in ("fmix", "crc"):
        raise ValueError("hash must be 'fmix' or 'crc'")
    m0 = 0
    sp = None
    if seed_edges is not None:
        if seed_edges.dtype != torch.int32 or seed_edges.numel() % 2:
            raise ValueError("seed_edges must be int32 with 2*m0 elements")
        m0 = seed_edges.numel() // 2
        device = seed_edges.device if device is None else device
    if count is None:
        count = (n - n0) * d - begin
    dev = _device(device if out is None else out.device)
    if out is None:
        out = torch.empty((count, 2), dtype=torch.int32, device=dev)
    elif out.dtype != torch.int32 or out.numel() != 2 * count:
        raise ValueError("out must be int32 with 2*count elements")
    sp = _ptr(seed_edges, dev)
    flags = (NO_SELF_LOOPS if no_self_loops else 0) | (HASH_CRC if hash == "crc" else 0)
    with torch.cuda.device(dev):
        _check("ba_generate_model", lib().ba_generate_model(n, d, seed, n0, m0, sp, flags, begin, count,
                                                            _ptr(out, dev) if count else None, _stream(dev)))
    return out
