"""Benchmark: Barabasi-Albert generation by per-edge recomputation on one MI355X.

One step = the whole hot path on the 2^26-node, d=16, seed=7 graph
(1,073,741,824 edges): every edge computed by its own hash chain, the full
uint32 edge array (8 GiB) written to HBM and the full uint32 degree array of
all 2^26 nodes.  Outputs and the degree workspace stay allocated across steps
(the inputs are three integers), so a timed step is pure GPU work.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is edges per second of the timed steps.
Every kernel of a step is timed live with HIP events on the stream it runs
on (the library's timing hook); `roofline` is that of the kernel with the
largest share of the step, against its algorithmic work (ALU lane-cycles
priced by the frozen per-instruction costs below, and 8 bytes per edge);
`kernels` gives every kernel's share and roofline fraction, `path` the whole
step against the method's 8.25 bytes per edge.  The other two parts of the
metric follow: `batched_over_single` (the 4096-instance batch against the
single-graph chain kernel, both edge pairs only) and `served_p50_ms` /
`served_p99_ms` (the 4000-request trace through the continuous-batching
server).  `cpu_baseline` times the CPU oracle (sequential Batagelj-Brandes
plus the degree count) on a bounded prefix of the same graph;
`cpu_recompute` times the oracle's per-edge recomputation on every granted
host core (the paper's own parallel method on the CPU), edges only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, D, SEED = 1 << 26, 16, 7
M = N * D
HBM_PEAK = 8.0e12                          # MI355X HBM3E, bytes/s
VALU_PEAK = 256 * 64 * 2.4e9               # 32-bit lane-cycles/s: 256 CUs x 64 lanes x 2.4 GHz
# Algorithmic work, frozen: the VALU instructions of a
# plain 32-bit lowering of the hash and of the per-edge work, priced at the
# issue costs `bench.py --workload rates` measured on the MI355X (lane-cycles
# at 2.4 GHz: multiplies 1.151, alignbit 1.041, add3 1.046, simple 0.634):
#   narrow hash (r < 2^32): 11 multiplies + 3 alignbit + 2 add3 + 15 simple = 27.38
#   wide hash (any r):      15 multiplies + 3 alignbit + 2 add3 + 20 simple = 35.15
#   per edge besides its hash evaluations: 2 multiplies + 13 simple       = 10.54
# Hash evaluations per edge of this graph: 2,147,478,402 over its 2^30 edges
# (counted by the CPU oracle).  Bytes: the edge pairs (8 per edge) and the
# degree array (4 per node); region entries of the degree pipeline (2 bytes
# per edge, written by the fused generator and read by the histogram) are
# the implementation's own traffic, not the method's.
ALU_NARROW_HASH = 27.38
ALU_WIDE_HASH = 35.15
ALU_FIXED = 10.54
HASH_PER_EDGE = 2147478402 / M
ALU_PER_EDGE = HASH_PER_EDGE * ALU_NARROW_HASH + ALU_FIXED
EDGE_BYTES = 8.0
DEG_BYTES = 4.0 * N
HIST_IMPL_BYTES = 2.0 * M + 4.0 * N
KERNEL_NAMES = {
    "gen": "k_gen_part (chain + edge pairs + partition of second endpoints)",
    "hist": "k_deg_hist16 (LDS histograms into deg)",
}
PROFILE = os.path.join(ROOT, "profiles", "pipeline_n2e26_d16_hbm_traffic.md")
# Files holding the pipeline's kernels and the host code that launches them:
# the committed counter summary counts only while they are unchanged.
KERNEL_SOURCES = [
    os.path.join(ROOT, "paper_1602_07106_amd", "csrc", f)
    for f in ("ba.hip", "ba_device.h", "ba_degree.h", "ba_genpart.h")
]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic() -> dict:
    """HBM bytes per launch of each kernel kind from the committed rocprofv3
    counter summary; empty when absent or taken on different kernel source."""
    try:
        txt = open(PROFILE).read()
    except OSError:
        return {}
    m_src = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    if not m_src or m_src.group(1) != kernel_source_hash():
        return {}
    return {k: float(v) for k, v in re.findall(r"hbm_bytes_per_launch\[(\w+)\]:\s*([0-9.eE+]+)", txt)}


def cpu_baseline():
    """The CPU oracle as it stands, on the first 2^29 edges of the same graph
    (the graph is prefix-stable: they are the whole 2^25-node graph)."""
    import oracle

    n_s = 1 << 25
    t0 = time.perf_counter()
    E, _ = oracle.bb_generate(n_s, D, SEED)
    oracle.count_degrees(E, n_s)
    dt = time.perf_counter() - t0
    return {
        "value": n_s * D / dt,
        "unit": "edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first 2^29 edges (n=2^25, d=16, seed=7): sequential Batagelj-Brandes + degree count, %.1f s" % dt,
    }


def cpu_recompute_threads():
    """A second CPU figure: the paper's own parallel method on the host.  The
    oracle's per-edge recomputation (no edge array read) runs on disjoint
    edge ranges in one thread per host core granted (at most 16), on the
    first 2^29 edges of the headline graph; edges only."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    threads = max(1, min(16, os.cpu_count() or 1))
    total, piece = 1 << 29, 1 << 22
    oracle.lib()

    def work(b):
        oracle.edges_range(D, SEED, b, piece)  # the foreign call releases the GIL

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(0, total, piece)))
    dt = time.perf_counter() - t0
    return {
        "value": total / dt,
        "unit": "edges/s",
        "cores": threads,
        "kind": "oracle per-edge recomputation, one thread per core over disjoint edge ranges (edges only)",
        "sample": "first 2^29 edges (n=2^26, d=16, seed=7) in pieces of 2^22, %.1f s" % dt,
    }


def copy_calibration(nbytes: int) -> int:
    """A plain device copy of known size: under rocprofv3 --pmc FETCH_SIZE /
    WRITE_SIZE it gives the counter reading for nbytes read and written."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)
    return 0


def kernel_rooflines(per_launch_s: dict) -> dict:
    """Roofline of each main kernel of the step from its measured mean launch
    time, against its algorithmic work (the binding bound is the longer of
    the ALU and HBM times at peak)."""
    out = {}
    t = per_launch_s.get("gen")
    if t:
        cyc, nbytes = ALU_PER_EDGE * M, EDGE_BYTES * M
        alu, hbm = cyc / t, nbytes / t
        if nbytes / HBM_PEAK >= cyc / VALU_PEAK:
            out["gen"] = {"bound": "hbm", "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                          "frac": hbm / HBM_PEAK, "alu_frac": alu / VALU_PEAK}
        else:
            out["gen"] = {"bound": "alu", "achieved": alu / 1e12, "peak": VALU_PEAK / 1e12, "unit": "Tlane-cycles/s",
                          "frac": alu / VALU_PEAK, "hbm_frac": hbm / HBM_PEAK}
        out["gen"].update({"alg_bytes": nbytes, "alg_cycles": cyc})
    t = per_launch_s.get("hist")
    if t:
        bw = DEG_BYTES / t
        out["hist"] = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                       "frac": bw / HBM_PEAK, "alg_bytes": DEG_BYTES, "impl_bytes": HIST_IMPL_BYTES,
                       "impl_frac": HIST_IMPL_BYTES / t / HBM_PEAK}
    return out


def batch_roofline(cyc: float, nbytes: float, t: float, ms_per_step: float, launches: int) -> dict:
    """Binding roofline (the longer of the ALU and HBM times) of one pass of
    the batched kernel over all rounds."""
    alu, hbm = cyc / t / VALU_PEAK, nbytes / t / HBM_PEAK
    if nbytes / HBM_PEAK >= cyc / VALU_PEAK:
        r = {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
             "frac": round(hbm, 4), "alu_frac": round(alu, 4)}
    else:
        r = {"bound": "alu", "achieved": round(cyc / t / 1e12, 2), "peak": round(VALU_PEAK / 1e12, 2),
             "unit": "Tlane-cycles/s", "frac": round(alu, 4), "hbm_frac": round(hbm, 4)}
    r.update({"traffic": None, "kernel": "k_gen_batch", "kernel_ms_per_step": round(ms_per_step, 3),
              "launches": launches, "alg_bytes_per_step": nbytes, "alg_lane_cycles_per_step": cyc})
    return r


def batch_line(args) -> dict:
    """The batched workload: 4096 independent graphs (workloads.batch_instances,
    7.64e10 edges, 611 GB of edge pairs) in HBM-budgeted rounds of 64 GiB,
    one persistent launch per round into the same round buffer.  A step is a
    pass over all instances.  Also times the single-graph chain kernel on the
    n=2^26, d=16 graph (edge pairs only) for the batched / single ratio."""
    import numpy as np
    import torch

    import paper_1602_07106_amd as ba
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, d, s = workloads.batch_instances()
    total = int((n.astype(np.uint64) * d.astype(np.uint64)).sum())
    round_elems = 1 << 34
    r, off, rounds = ba.batch_plan_rounds(n, d, round_elems)
    out = torch.empty(round_elems, dtype=torch.int32, device=dev)
    batches = []
    for k in range(rounds):
        js = np.flatnonzero(r == k)
        batches.append(ba.Batch(n[js], d[js], s[js], out_offset=off[js], device=dev))
    shape = batches[0].autotune(out)

    def step():
        for b in batches:
            b.launch(out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ba.kernel_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    kt = ba.kernel_timing_read()
    ba.kernel_timing(False)
    ms = e0.elapsed_time(e1)
    value = total * args.steps / (ms / 1e3)
    # single graph, chain kernel only (same edge-pair output)
    single = out[: 2 * M].view(M, 2)
    for _ in range(2):
        ba.generate(N, D, SEED, out=single)
    torch.cuda.synchronize()
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    f0.record()
    for _ in range(5):
        ba.generate(N, D, SEED, out=single)
    f1.record()
    torch.cuda.synchronize()
    single_rate = M * 5 / (f0.elapsed_time(f1) / 1e3)
    # ALU roofline with the ideal-hash expectation of evaluations per edge
    # (2 - 1.77/sqrt(m) per instance; the oracle cannot count 7.6e10 edges)
    m = n.astype(np.float64) * d
    hashes = float((m * (2.0 - 1.77 / np.sqrt(m))).sum())
    gen_ms, gen_n = kt["gen"]
    t_launch = gen_ms / 1e3 / args.steps  # kernel time of one pass (all rounds)
    cyc = hashes * ALU_NARROW_HASH + total * ALU_FIXED  # every instance's positions are below 2^32
    line = {
        "metric": "edges/s, 4096-instance batch (batched vs single)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded instance table: n log-uniform 1e3..1e7, d uniform 1..32)",
        "config": {"workload": "4096 plain BA graphs, uint32 edge pairs, rounds of 64 GiB", "instances": int(n.size),
                   "edges": total, "rounds": rounds, "shape": list(ba.batch_shape(shape))},
        "single_graph_edges_per_s": single_rate,
        "batched_over_single": value / single_rate,
        "roofline": batch_roofline(cyc, 8.0 * total, t_launch, gen_ms / args.steps, gen_n),
    }
    return line


def bench_batch(args) -> int:
    print(json.dumps(batch_line(args)), flush=True)
    return 0


def served_line(args) -> dict:
    """The served workload: the 4000-request trace of workloads.served_trace
    (Poisson arrivals at 2000/s; half edge lists, half first-10^5 degrees)
    replayed in real time against a continuous-batching server with a
    160 GiB arena; each result is released as soon as it is ready.  Latency
    is arrival to GPU completion of the request's step."""
    import numpy as np
    import torch

    import paper_1602_07106_amd as ba
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tr = workloads.served_trace()
    count = len(tr["n"])
    m = tr["n"].astype(np.float64) * tr["d"]
    # warm-up: load every kernel the server launches
    w = ba.Server(1 << 30, device=dev)
    ts = [w.submit_edges(5000, 4, 1), w.submit_edges(1 << 22, 2, 1), w.submit_degrees(5000, 4, 1, 100),
          w.submit_degrees(1 << 31, 2, 1, 100)]
    left = set(ts)
    t_end = time.perf_counter() + 60
    while left:
        if time.perf_counter() > t_end:
            raise RuntimeError("served warm-up made no progress in 60 s")
        w.pump()
        for t in w.completed():
            w.release(t)
            left.discard(t)
    w.close()
    del w
    torch.cuda.synchronize()

    srv = ba.Server(160 << 30, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()  # the server's time origin has just run on the GPU
    arrival = tr["arrival_s"]
    lat = np.zeros(count)
    ticket_of = {}
    i = done = 0
    while done < count:
        now = time.perf_counter() - t0
        if now > arrival[-1] + 120:
            raise RuntimeError("served trace not finished 120 s after its last arrival (%d of %d done)" % (done, count))
        while i < count and arrival[i] <= now:
            if tr["kind"][i] == 0:
                t = srv.submit_edges(int(tr["n"][i]), int(tr["d"][i]), int(tr["seed"][i]))
            else:
                t = srv.submit_degrees(int(tr["n"][i]), int(tr["d"][i]), int(tr["seed"][i]), int(tr["first_k"][i]))
            ticket_of[t] = i
            i += 1
        admitted = srv.pump(max_inflight=args.served_inflight)
        fin = srv.completed()
        for t in fin:
            st, ms, _, _ = srv.poll(t)
            if st != ba.JOB_READY:
                raise RuntimeError("request %d failed" % ticket_of[t])
            j = ticket_of[t]
            lat[j] = ms - arrival[j] * 1e3
            srv.release(t)
            done += 1
        if not admitted and not fin:
            time.sleep(0.0002)
    makespan = time.perf_counter() - t0
    srv.close()
    total = float(m.sum())
    line = {
        "metric": "served p99 ms (4000-request trace)",
        "value": float(np.percentile(lat, 99)),
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": makespan * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded request trace: Poisson 2000/s, n log-uniform 1e4..1e8, 2% n=2^27 d=16)",
        "config": {"workload": "continuous batching, 4000 requests, half edge lists / half first-1e5 degrees, "
                               "160 GiB arena", "requests": count, "edges": total},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "arrival_span_s": float(arrival[-1]),
        "makespan_s": makespan,
        "inflight_steps": args.served_inflight,
        "served_edges_per_s": total / makespan,
        "offered_edges_per_s": total / float(arrival[-1]),
    }
    return line


def bench_served(args) -> int:
    print(json.dumps(served_line(args)), flush=True)
    return 0


# Streaming workload: n=2^30, d=64, seed=42, degrees of nodes 0..10^5-1 and
# the edge checksum over all 2^36 edges (64-bit positions, nothing stored).
# Algorithmic work: the frozen wide-hash price (positions reach 2^37) at the
# ideal-hash mean of evaluations per edge, plus the per-edge price.
STREAM = (1 << 30, 64, 42, 100000)


def bench_stream(args) -> int:
    import torch

    import paper_1602_07106_amd as ba

    n, d, seed, k = STREAM
    m = n * d
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    for _ in range(args.warmup):
        ba.degrees(n, d, seed, k)
    torch.cuda.synchronize()
    ba.kernel_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ba.degrees(n, d, seed, k)
    e1.record()
    torch.cuda.synchronize()
    kt = ba.kernel_timing_read()
    ba.kernel_timing(False)
    ms = e0.elapsed_time(e1) / args.steps
    st_ms, st_n = kt["stream"]
    t = st_ms / st_n / 1e3
    hashes = m * (2.0 - 1.77 / m ** 0.5)
    cyc = hashes * ALU_WIDE_HASH + m * ALU_FIXED
    line = {
        "metric": "edges/s, streamed first-10^5 degrees at n=2^30, d=64",
        "value": m / (ms / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (the generator is the workload: n, d, seed)",
        "config": {"workload": "streamed degrees of nodes 0..99999 + edge checksum, n=2^30, d=64, seed=42, "
                               "2^36 edges, nothing stored", "edges": m},
        "roofline": {"bound": "alu", "achieved": round(cyc / t / 1e12, 2), "peak": round(VALU_PEAK / 1e12, 2),
                     "unit": "Tlane-cycles/s", "frac": round(cyc / t / VALU_PEAK, 4), "traffic": None,
                     "kernel": "k_stream (64-bit positions)", "kernel_ms": round(t * 1e3, 3), "launches": st_n,
                     "alg_lane_cycles_per_launch": cyc},
    }
    if not args.no_cpu_baseline:
        import time as _t

        import oracle

        c = 1 << 28
        t0 = _t.perf_counter()
        oracle.stream(d, seed, 0, c, k)
        dt = _t.perf_counter() - t0
        line["cpu_baseline"] = {"value": c / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
                                "sample": "first 2^28 edges of the same graph, streamed degrees + checksum, %.1f s" % dt}
    print(json.dumps(line), flush=True)
    return 0


# Generalized-model workload: n=2^26, d=16, seed=7 with a seed graph of
# n0=100 nodes and m0=1000 edges (workloads.seed_graph) in front of the new
# edges; the four variants of the hash (fmix, the paper's CRC) and the
# draw bound (self-loops allowed or not).
MODEL = (1 << 26, 16, 7, 100, 1000)


def bench_model(args) -> int:
    import numpy as np
    import torch

    import paper_1602_07106_amd as ba
    import workloads

    n, d, seed, n0, m0 = MODEL
    m = (n - n0) * d
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S_host = workloads.seed_graph(n0, m0)
    S = torch.from_numpy(S_host.astype(np.int32)).to(dev)
    out = torch.empty((m, 2), dtype=torch.int32, device=dev)
    variants = {}
    for h in ("fmix", "crc"):
        for nl in (False, True):
            def f():
                ba.generate_model(n, d, seed, n0=n0, seed_edges=S, no_self_loops=nl, hash=h, out=out)

            for _ in range(args.warmup):
                f()
            torch.cuda.synchronize()
            ba.kernel_timing(True)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                f()
            e1.record()
            torch.cuda.synchronize()
            kt = ba.kernel_timing_read()
            ba.kernel_timing(False)
            ms = e0.elapsed_time(e1) / args.steps
            g_ms, g_n = kt["gen"]
            name = h + (", no self-loops" if nl else "")
            variants[name] = {"edges_per_s": m / (ms / 1e3), "ms_per_step": round(ms, 4),
                              "kernel_ms": round(g_ms / g_n, 4)}
    main = variants["fmix"]
    t = main["kernel_ms"] / 1e3
    hashes = m * (2.0 - 1.77 / m ** 0.5)
    cyc = hashes * ALU_NARROW_HASH + m * ALU_FIXED
    byts = 8.0 * m
    line = {
        "metric": "edges/s, generalized model (100-node, 1000-edge seed graph) at n=2^26, d=16",
        "value": main["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded seed graph from workloads.seed_graph; the generator is the workload)",
        "config": {"workload": "generalized model: seed graph n0=100, m0=1000, then n=2^26, d=16, seed=7; "
                               "uint32 edge pairs of the new edges", "edges": m, "variants": variants},
        "roofline": {"bound": "hbm", "achieved": round(byts / t / 1e9, 2), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": round(byts / t / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_gen_model (fmix, 32-bit positions)", "kernel_ms": main["kernel_ms"],
                     "alg_bytes_per_launch": byts, "alu_frac": round(cyc / t / VALU_PEAK, 4)},
    }
    if not args.no_cpu_baseline:
        import time as _t

        import oracle

        c = 1 << 26
        t0 = _t.perf_counter()
        oracle.model_edges_range(n0, m0, S_host, d, seed, 0, 0, c)
        dt = _t.perf_counter() - t0
        line["cpu_baseline"] = {"value": c / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
                                "sample": "first 2^26 new edges, fmix hash, per-edge chains, %.1f s" % dt}
    print(json.dumps(line), flush=True)
    return 0


# Issue-rate microbenchmark (libba_rates.so): lane-cycles one VALU
# instruction of each kind costs at 2.4 GHz when every lane runs 8
# independent chains of it (8 waves per SIMD), and the 16-byte fill rate.
RATE_OPS = ("mul_lo_u32", "mul_hi_u32", "mad_u64_u32", "alignbit_b32", "add3_u32", "xor_b32", "lshrrev_b32",
            "add_u32")


def bench_rates(args) -> int:
    import ctypes

    import torch

    from paper_1602_07106_amd import build as _b

    L = ctypes.CDLL(_b.RATES_LIB)
    L.ba_rate_run.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_float)]
    L.ba_rate_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_float)]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks, iters = cus * 8, 4096
    sink = torch.zeros(blocks, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    lane_cycles_per_s = VALU_PEAK  # 256 CUs x 64 lanes x 2.4 GHz
    ops = {}
    for k, name in enumerate(RATE_OPS):
        best = None
        for _ in range(max(2, args.steps // 4)):
            ms = ctypes.c_float(0)
            rc = L.ba_rate_run(k, blocks, iters, sink.data_ptr(), st, ctypes.byref(ms))
            if rc:
                raise RuntimeError("ba_rate_run(%s) failed: %d" % (name, rc))
            best = ms.value if best is None else min(best, ms.value)
        n_ops = blocks * 256 * iters * L.ba_rate_ops_per_iter(k)
        rate = n_ops / (best / 1e3)
        ops[name] = {"lane_ops_per_s": rate, "lane_cycles_per_op": round(lane_cycles_per_s / rate, 3),
                     "ms": round(best, 3)}
    nbytes = 4 << 30
    buf = torch.empty(nbytes // 4, dtype=torch.int32, device=dev)
    fill = None
    for _ in range(max(3, args.steps // 4)):
        ms = ctypes.c_float(0)
        rc = L.ba_rate_fill(buf.data_ptr(), nbytes // 16, cus * 8, st, ctypes.byref(ms))
        if rc:
            raise RuntimeError("ba_rate_fill failed: %d" % rc)
        fill = ms.value if fill is None else min(fill, ms.value)
    line = {"metric": "VALU issue cost and 16-byte fill rate", "unit": "lane-cycles per instruction at 2.4 GHz",
            "cus": cus, "blocks": blocks, "threads_per_block": 256, "chains_per_lane": 8, "iters": iters,
            "ops": ops, "fill_bytes": nbytes, "fill_ms": round(fill, 4),
            "fill_GB_per_s": round(nbytes / (fill / 1e3) / 1e9, 1)}
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["graph", "batch", "served", "stream", "model", "rates"], default="graph",
                    help="graph: the n=2^26, d=16 graph with degrees (default); batch: 4096 graphs; "
                         "served: a 4000-request trace through the continuous-batching server; "
                         "stream: streamed first-10^5 degrees at n=2^30, d=64; "
                         "model: the generalized model (seed graph, no-self-loop draws, CRC hash); "
                         "rates: VALU issue-rate and 16-byte fill microbenchmarks (the ALU roofline's prices)")
    ap.add_argument("--served-inflight", type=int, default=2, metavar="STEPS",
                    help="steps the served workload keeps in flight (server pump's max_inflight)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="graph workload only: skip the batched and served parts of the metric")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the generator here has no multi-GPU path "
              "(GPUs would take contiguous edge-ID ranges, with no exchange but one reduction "
              "of the degree counts); use --gpus 1", file=sys.stderr)
        return 2
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "model":
        return bench_model(args)
    if args.workload == "stream":
        return bench_stream(args)
    if args.workload == "rates":
        return bench_rates(args)

    import torch

    import paper_1602_07106_amd as ba

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    out = torch.empty((M, 2), dtype=torch.int32, device=dev)
    deg = torch.empty(N, dtype=torch.int32, device=dev)
    ws = ba.workspace(N, D, M, device=dev)

    def step():
        ba.generate(N, D, SEED, degrees=True, out=out, deg_out=deg, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the library launches on torch's current stream, where these events sit
    ba.kernel_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    kt = ba.kernel_timing_read()
    ba.kernel_timing(False)

    ms_per_step = gpu_ms / args.steps
    value = M * args.steps / (gpu_ms / 1e3)

    per_launch_s = {k: ms / n / 1e3 for k, (ms, n) in kt.items() if n}
    roofs = kernel_rooflines(per_launch_s)
    traffic = committed_traffic()
    kernels = {}
    for k, (ms, n) in kt.items():
        if not n:
            continue
        e = {"ms_per_launch": round(ms / n, 4), "launches": n, "share_of_step": round(ms / gpu_ms, 4)}
        if k in roofs:
            e.update({"bound": roofs[k]["bound"], "frac": round(roofs[k]["frac"], 4)})
            for f in ("hbm_frac", "alu_frac", "impl_frac"):
                if f in roofs[k]:
                    e[f] = round(roofs[k][f], 4)
            e["traffic"] = traffic.get(k)
        kernels[k] = e
    dom = max(roofs, key=lambda k: kt[k][0])
    r = roofs[dom]
    roof = {"bound": r["bound"], "achieved": round(r["achieved"], 2), "peak": round(r["peak"], 2), "unit": r["unit"],
            "frac": round(r["frac"], 4), "traffic": traffic.get(dom),
            "kernel": KERNEL_NAMES[dom], "kernel_ms": round(per_launch_s[dom] * 1e3, 4), "launches": kt[dom][1],
            "alg_bytes_per_launch": r["alg_bytes"]}
    if "alg_cycles" in r:
        roof["alg_lane_cycles_per_launch"] = r["alg_cycles"]
        for f in ("hbm_frac", "alu_frac"):
            if f in r:
                roof[f] = round(r[f], 4)
    # the whole step against the method's own bytes (edge pairs + degree
    # array: 8 B per edge + 4 B per node) and its frozen ALU work
    step_s = ms_per_step / 1e3
    path = {"alg_bytes_per_edge": (EDGE_BYTES * M + DEG_BYTES) / M,
            "hbm_frac": round((EDGE_BYTES * M + DEG_BYTES) / step_s / HBM_PEAK, 4),
            "alg_lane_cycles_per_edge": round(ALU_PER_EDGE, 2),
            "alu_frac": round(ALU_PER_EDGE * M / step_s / VALU_PEAK, 4)}

    line = {
        "metric": "edges/s at n=2^26,d=16 (bit-exact)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (the generator is the workload: n, d, seed)",
        "config": {"workload": "plain BA, empty seed graph: n=2^26, d=16, seed=7, uint32 edge pairs + full "
                               "uint32 degree array", "edges": M, "n": N, "d": D, "seed": SEED},
        "roofline": roof,
        "kernels": kernels,
        "path": path,
        "wall_s": round(wall, 3),
    }
    if not args.no_extras:
        # the other two parts of the metric: batched vs single-graph edges/s
        # (4096-instance table, 3 timed passes) and the served trace's p50/p99
        del out, deg, ws
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        b = batch_line(argparse.Namespace(steps=3, warmup=1))
        line["batched_edges_per_s"] = b["value"]
        line["single_graph_edges_per_s"] = b["single_graph_edges_per_s"]
        line["batched_over_single"] = b["batched_over_single"]
        line["batch_roofline"] = b["roofline"]
        torch.cuda.empty_cache()
        sv = served_line(args)
        line["served_p50_ms"] = sv["p50_ms"]
        line["served_p99_ms"] = sv["p99_ms"]
        line["served_edges_per_s"] = sv["served_edges_per_s"]
        line["served_trace"] = {"requests": sv["config"]["requests"], "arrival_span_s": sv["arrival_span_s"],
                                "makespan_s": sv["makespan_s"], "offered_edges_per_s": sv["offered_edges_per_s"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
        line["cpu_recompute"] = cpu_recompute_threads()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
