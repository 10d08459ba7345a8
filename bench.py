"""Benchmark: Barabasi-Albert generation by per-edge recomputation on one MI355X.

One step = the whole hot path on the 2^26-node, d=16, seed=7 graph
(1,073,741,824 edges): every edge computed by its own hash chain, the full
uint32 edge array (8 GiB) written to HBM and the fused uint32 degree array of
all 2^26 nodes.  Outputs and the degree workspace stay allocated across steps
(the inputs are three integers), so a timed step is pure GPU work.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is edges per second of the timed steps.
`roofline` is that of the dominant kernel (the per-edge chain kernel with
its fused coarse partition of second endpoints), timed live with HIP events
on its own stream; `cpu_baseline` times the CPU oracle (sequential
Batagelj-Brandes plus the degree count) on a bounded prefix of the same graph.
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
HBM_PEAK_GBPS = 8000.0                    # MI355X HBM3E
VALU_PEAK = 256 * 64 * 2.4e9              # 32-bit lane-ops/s, one per lane per clock
# Algorithmic work of the chain kernel per edge (derivation in the design doc):
# hash evaluations per edge for this graph (2,147,478,402 over its 2^30
# edges, counted by the CPU oracle), VALU issue cycles per evaluation of the
# narrow (r < 2^32) hash, and fixed cycles per edge.
HASH_PER_EDGE = 2147478402 / M
CYCLES_PER_HASH = 17.0
CYCLES_PER_EDGE = 2.0
BYTES_PER_EDGE = 8.0                      # the uint32 (u, v) pair written per edge
PROFILE = os.path.join(ROOT, "profiles", "gen_partition_n2e26_d16_traffic.md")
KERNEL_SOURCES = [
    os.path.join(ROOT, "paper_1602_07106_amd", "csrc", f) for f in ("ba.hip", "ba_device.h", "ba_degree.h")
]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per launch of the chain kernel from the committed rocprofv3
    counter summary, or None when absent or taken on different kernel source."""
    try:
        txt = open(PROFILE).read()
    except OSError:
        return None
    m_src = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_src or not m_b or m_src.group(1) != kernel_source_hash():
        return None
    return float(m_b.group(1))


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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        return 2

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
    kern_ms, launches = ba.kernel_timing_read()
    ba.kernel_timing(False)
    kern_avg = kern_ms / max(1, launches)

    ms_per_step = gpu_ms / args.steps
    value = M * args.steps / (gpu_ms / 1e3)

    # roofline of the chain kernel: both bounds, the binding one reported
    t_hbm = BYTES_PER_EDGE * M / (HBM_PEAK_GBPS * 1e9)
    t_alu = (HASH_PER_EDGE * CYCLES_PER_HASH + CYCLES_PER_EDGE) * M / VALU_PEAK
    kern_s = kern_avg / 1e3
    hbm_achieved = BYTES_PER_EDGE * M / kern_s / 1e9
    alu_achieved = (HASH_PER_EDGE * CYCLES_PER_HASH + CYCLES_PER_EDGE) * M / kern_s / 1e12
    traffic = committed_traffic()
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(hbm_achieved / HBM_PEAK_GBPS, 4), "traffic": traffic}
    else:
        roof = {"bound": "alu", "achieved": round(alu_achieved, 2), "peak": round(VALU_PEAK / 1e12, 2),
                "unit": "Tlane-cycles/s", "frac": round(alu_achieved * 1e12 / VALU_PEAK, 4), "traffic": traffic}
    roof.update({
        "kernel": "k_gen_u32 (chain + coarse partition)",
        "kernel_ms": round(kern_avg, 4),
        "launches": launches,
        "alu_frac": round(alu_achieved * 1e12 / VALU_PEAK, 4),
        "hbm_frac": round(hbm_achieved / HBM_PEAK_GBPS, 4),
    })

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
        "config": {"workload": "plain BA, empty seed graph: n=2^26, d=16, seed=7, uint32 edge pairs + fused "
                               "uint32 degree array", "edges": M, "n": N, "d": D, "seed": SEED},
        "roofline": roof,
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
