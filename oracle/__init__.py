"""CPU oracle for the Barabasi-Albert edge generator (arXiv:1602.07106).

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the library in
``paper_1602_07106_amd/`` never does.  The arithmetic lives in the plain C
file ``bb_oracle.c`` next to this one (compiled with gcc, loaded through
ctypes); this module only marshals numpy arrays.

Functions follow the paper section by section:

* ``key``, ``fmix64``, ``umul64hi``, ``h`` -- the keyed position hash: a
  function of the array position that returns a value in 0..r-1 (Section 2,
  the paragraph on reproducing random behaviour).  The hash itself is the
  SplitMix64 output mix of ``r XOR seed*phi64`` scaled into 0..r-1 by a
  64x64->128 high product.
* ``bb_generate`` -- the sequential Batagelj-Brandes algorithm (Section 2,
  second paragraph): E[2i] = floor(i/d), E[2i+1] = E[x] with x in 0..2i.
* ``bb_with_choices`` -- the same with the choices x given explicitly.
* ``edge`` / ``edges_range`` -- one edge at a time from the definition of E
  (Section 2, figure generateEdge).
* ``stream`` -- the streaming degree consumer of Section 3 (degrees of the
  first k nodes) plus the edge checksum.
* ``count_degrees`` / ``checksum_E`` -- occurrence counts and the checksum of
  a stored edge array.
* ``model_*`` (``bb_model.c``) -- the generalizations of Section
  "Generalizations": a seed graph of n0 nodes and m0 edges in front of the
  edge array, and draws that avoid self-loops; ``crc32c_*`` / ``h_crc`` --
  the paper's CRC-based hash (figure with hash_crc) as an alternative
  keyed hash.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bb_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "bb_model.c")]
_LIB = os.path.join(_HERE, "libbb_oracle.so")

_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile bb_oracle.c and bb_model.c into libbb_oracle.so with gcc (plain -O2)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp] + _SRCS
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()  # no-op unless the library is missing or older than its source
        L = ctypes.CDLL(_LIB)
        for name, res, args in [
            ("bbo_key", _u64, [_u64]),
            ("bbo_fmix64", _u64, [_u64]),
            ("bbo_umul64hi", _u64, [_u64, _u64]),
            ("bbo_h", _u64, [_u64, _u64]),
            ("bbo_edge_word", _u64, [_u64, _u64, _u64]),
            ("bbo_bb_generate", ctypes.c_int, [_u64, _u64, _u64, _p, _p]),
            ("bbo_bb_with_choices", ctypes.c_int, [_u64, _u64, _p, _p]),
            ("bbo_count_degrees", ctypes.c_int, [_p, _u64, _u64, _p]),
            ("bbo_checksum_E", _u64, [_p, _u64]),
            ("bbo_edge", None, [_u64, _u64, _u64, _p, _p, _p]),
            ("bbo_edges_range", None, [_u64, _u64, _u64, _u64, _p, _p]),
            ("bbo_stream", None, [_u64, _u64, _u64, _u64, _u64, _p, _p, _p]),
            ("bbo_crc32c_update", ctypes.c_uint32, [ctypes.c_uint32, _p, _u64]),
            ("bbo_crc32c_u64", ctypes.c_uint32, [ctypes.c_uint32, _u64]),
            ("bbo_h_crc", _u64, [_u64, _u64, _u64]),
            ("bbo_h_fmix", _u64, [_u64, _u64, _u64]),
            ("bbo_model_bb_generate", ctypes.c_int, [_u64, _u64, _p, _u64, _u64, _u64, ctypes.c_uint, _p, _p]),
            ("bbo_model_bb_with_choices", ctypes.c_int, [_u64, _u64, _p, _u64, _u64, ctypes.c_uint, _p, _p]),
            ("bbo_model_edge", None, [_u64, _u64, _p, _u64, _u64, ctypes.c_uint, _p, _u64, _p, _p, _p]),
            ("bbo_model_edges_range", None, [_u64, _u64, _p, _u64, _u64, ctypes.c_uint, _u64, _u64, _p, _p]),
        ]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def key(seed: int) -> int:
    return lib().bbo_key(seed)


def fmix64(z: int) -> int:
    return lib().bbo_fmix64(z)


def umul64hi(a: int, b: int) -> int:
    return lib().bbo_umul64hi(a, b)


def h(key_: int, r: int) -> int:
    return lib().bbo_h(key_, r)


def edge_word(i: int, u: int, v: int) -> int:
    return lib().bbo_edge_word(i, u, v)


def bb_generate(n: int, d: int, seed: int):
    """Sequential Batagelj-Brandes. Returns (E as uint32[2nd], hash calls)."""
    E = np.empty(2 * n * d, dtype=np.uint32)
    calls = _u64(0)
    rc = lib().bbo_bb_generate(n, d, seed, _ptr(E), ctypes.addressof(calls))
    if rc == -1:
        raise ValueError("bb_generate: node IDs must fit 32 bits")
    if rc != 0:
        raise ValueError("bb_generate: hash left the range 0..2i")
    return E, calls.value


def bb_with_choices(n: int, d: int, x) -> np.ndarray:
    """Batagelj-Brandes with explicit choices x[i] in 0..2i."""
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    assert xs.shape == (n * d,)
    E = np.empty(2 * n * d, dtype=np.uint32)
    if lib().bbo_bb_with_choices(n, d, _ptr(xs), _ptr(E)) != 0:
        raise ValueError("choice out of range")
    return E


def count_degrees(E: np.ndarray, n: int) -> np.ndarray:
    E = np.ascontiguousarray(E, dtype=np.uint32)
    deg = np.empty(n, dtype=np.uint64)
    if lib().bbo_count_degrees(_ptr(E), E.size, n, _ptr(deg)) != 0:
        raise ValueError("count_degrees: entry is not a node ID below n")
    return deg


def checksum_E(E: np.ndarray) -> int:
    E = np.ascontiguousarray(E, dtype=np.uint32)
    return lib().bbo_checksum_E(_ptr(E), E.size // 2)


def edge(d: int, seed: int, i: int):
    """(u, v, hash evaluations) of edge i."""
    u, v, s = _u64(0), _u64(0), _u64(0)
    lib().bbo_edge(d, seed, i, ctypes.addressof(u), ctypes.addressof(v), ctypes.addressof(s))
    return u.value, v.value, s.value


def edges_range(d: int, seed: int, i0: int, count: int):
    """Edges i0..i0+count-1 as uint64[2*count] (u, v interleaved), and hash calls."""
    out = np.empty(2 * count, dtype=np.uint64)
    calls = _u64(0)
    lib().bbo_edges_range(d, seed, i0, count, _ptr(out), ctypes.addressof(calls))
    return out, calls.value


def stream(d: int, seed: int, i0: int, count: int, k: int, deg_k=None, cs: int = 0):
    """Streaming degrees of nodes 0..k-1 and checksum over edges i0..i0+count-1.

    Accumulates into ``deg_k`` (uint64[k], created zeroed when None) and XORs
    into ``cs``.  Returns (deg_k, cs, hash calls).
    """
    if deg_k is None:
        deg_k = np.zeros(k, dtype=np.uint64)
    assert deg_k.dtype == np.uint64 and deg_k.size == k
    c = _u64(cs)
    calls = _u64(0)
    lib().bbo_stream(d, seed, i0, count, k, _ptr(deg_k), ctypes.addressof(c), ctypes.addressof(calls))
    return deg_k, c.value, calls.value


NO_LOOPS, CRC = 1, 2


def crc32c_update(crc: int, data: bytes) -> int:
    buf = np.frombuffer(bytes(data), dtype=np.uint8)
    return int(lib().bbo_crc32c_update(crc, buf.ctypes.data if buf.size else None, buf.size))


def crc32c_u64(crc: int, x: int) -> int:
    return int(lib().bbo_crc32c_u64(crc, x))


def h_crc(key_: int, r: int, bound: int) -> int:
    return int(lib().bbo_h_crc(key_, r, bound))


def h_fmix(key_: int, r: int, bound: int) -> int:
    return int(lib().bbo_h_fmix(key_, r, bound))


def _seed_arr(S, m0):
    S = np.ascontiguousarray(np.asarray(S if S is not None else [], dtype=np.uint32))
    assert S.size == 2 * m0
    return S


def model_bb_generate(n0: int, m0: int, S, n: int, d: int, seed: int, flags: int = 0) -> np.ndarray:
    """Batagelj-Brandes with a seed graph: all 2*m0 + 2*(n-n0)*d positions."""
    S = _seed_arr(S, m0)
    E = np.empty(2 * m0 + 2 * (n - n0) * d, dtype=np.uint32)
    calls = _u64(0)
    rc = lib().bbo_model_bb_generate(n0, m0, S.ctypes.data if S.size else None, n, d, seed, flags,
                                     E.ctypes.data if E.size else None, ctypes.addressof(calls))
    if rc != 0:
        raise ValueError("model_bb_generate: rc %d" % rc)
    return E


def model_bb_with_choices(n0: int, m0: int, S, n: int, d: int, flags: int, x) -> np.ndarray:
    S = _seed_arr(S, m0)
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    E = np.empty(2 * m0 + 2 * (n - n0) * d, dtype=np.uint32)
    rc = lib().bbo_model_bb_with_choices(n0, m0, S.ctypes.data if S.size else None, n, d, flags,
                                         xs.ctypes.data if xs.size else None, E.ctypes.data if E.size else None)
    if rc != 0:
        raise ValueError("model_bb_with_choices: rc %d" % rc)
    return E


def model_edge(n0: int, m0: int, S, d: int, seed: int, flags: int, i: int, x=None):
    """(u, v, draws) of new edge i; with x given, the draws come from it."""
    S = _seed_arr(S, m0)
    xs = None if x is None else np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    u, v, s = _u64(0), _u64(0), _u64(0)
    lib().bbo_model_edge(n0, m0, S.ctypes.data if S.size else None, d, seed, flags,
                         None if xs is None else xs.ctypes.data, i, ctypes.addressof(u), ctypes.addressof(v),
                         ctypes.addressof(s))
    return u.value, v.value, s.value


def model_edges_range(n0: int, m0: int, S, d: int, seed: int, flags: int, i0: int, count: int):
    """(uint32[count, 2] new edges i0.., total draws)."""
    S = _seed_arr(S, m0)
    out = np.empty((count, 2), dtype=np.uint32)
    steps = _u64(0)
    lib().bbo_model_edges_range(n0, m0, S.ctypes.data if S.size else None, d, seed, flags, i0, count,
                                out.ctypes.data if count else None, ctypes.addressof(steps))
    return out, steps.value
