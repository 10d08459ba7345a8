"""The oracle's per-edge recomputation over disjoint edge ranges on several
host threads (test infrastructure only).  Each piece is one sequential
oracle call (edges_range / stream); the pieces are merged exactly (edge
arrays concatenated, degree counts added, checksums XORed), so the result is
the sequential oracle's over the whole range, in a fraction of the time.
The foreign calls release the GIL, so the threads run in parallel."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

# worker threads: the host cores granted to one GPU (at most 16)
THREADS = max(1, min(16, os.cpu_count() or 1))


def _pieces(b: int, c: int, piece: int):
    return [(b + o, min(piece, c - o)) for o in range(0, c, piece)]


def edges_u32(d: int, seed: int, b: int, c: int) -> np.ndarray:
    """Edges b .. b+c-1 as uint32[2c] (u, v interleaved; IDs below 2^32)."""
    out = np.empty(2 * c, dtype=np.uint32)
    oracle.lib()

    def work(p):
        b0, c0 = p
        ref, _ = oracle.edges_range(d, seed, b0, c0)
        out[2 * (b0 - b):2 * (b0 - b + c0)] = ref.astype(np.uint32)

    with ThreadPoolExecutor(THREADS) as ex:
        list(ex.map(work, _pieces(b, c, 1 << 22)))
    return out


def stream(d: int, seed: int, b: int, c: int, k: int):
    """(uint64[k] degrees of nodes 0..k-1, XOR checksum) over edges b .. b+c-1."""
    oracle.lib()
    piece = max(1 << 20, -(-c // (4 * THREADS)))

    def work(p):
        dk, cs, _ = oracle.stream(d, seed, p[0], p[1], k)
        return dk, cs

    deg = np.zeros(k, dtype=np.uint64)
    cs = 0
    with ThreadPoolExecutor(THREADS) as ex:
        for dk, x in ex.map(work, _pieces(b, c, piece)):
            deg += dk
            cs ^= x
    return deg, cs
