"""Benchmark of the sketch Y = A * Omega(seed) with a generated operand on one MI355X.

Default workload (one step): A 32768 x 32768 FP32 N(0,1), k = 5, P = 8 shares
of the paper's 1D layouts emulated on one GPU:
  * row layout, no reduction: 8 calls of sketch_gen_matmul on 4096-row blocks;
  * column layout with reduction: 1 call of sketch_gen_matmul_reduce on 8
    column blocks of 4096 (strided views of A), partial products summed on the
    device in FP64.
Each step streams A twice (8 GiB).  value = A bytes / wall time of the timed
steps (GB/s).  The roofline object covers the streaming kernel: algorithmic
bytes (A bytes; Omega is generated, never read) per launch / launch duration,
measured with HIP events recorded on the launch stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "A-stream GB/s (% HBM peak) for Y=A·Ω(seed) at k=5; p50/p99 latency served"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="target duration of the oracle's timed sample")
    return p.parse_args()


def cpu_baseline(A, k, seed, target_s):
    """Time the CPU oracle on a bounded row sample of the same share workload."""
    import numpy as np

    import oracle

    n = A.shape[1]
    rows = 256
    sample = A[:rows].cpu().numpy()
    t0 = time.perf_counter()
    oracle.gen_matmul(sample, seed, 0, 0, k)
    t_small = time.perf_counter() - t0
    rows = int(min(A.shape[0], max(256, rows * target_s / max(t_small, 1e-3))))
    rows = (rows // 256) * 256
    sample = np.ascontiguousarray(A[:rows].cpu().numpy())
    t0 = time.perf_counter()
    oracle.gen_matmul(sample, seed, 0, 0, k)
    dt = time.perf_counter() - t0
    return {"value": rows * n * 4 / dt / 1e9, "unit": "GB/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"rows 0..{rows} of A x all {n} columns (row layout, k={k}, Omega generated "
                      f"from the seed), {rows * n * 4 / 2**20:.0f} MiB, {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2603_20966_amd as sk
    from sketch_inputs import normal_matrix_device

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, P, k, seed = 32768, 8, 5, 1
    w = N // P
    A = normal_matrix_device(N, N, seed=0, device=dev)
    Yrows = torch.empty((N, k), dtype=torch.float32, device=dev)
    Yred = torch.empty((N, k), dtype=torch.float32, device=dev)
    shares = [A[i * w:(i + 1) * w] for i in range(P)]
    blocks = [A[:, b * w:(b + 1) * w] for b in range(P)]
    row0s = [b * w for b in range(P)]
    stream = torch.cuda.current_stream(dev)
    share_bytes = w * N * 4
    red_bytes = N * N * 4

    launches = []  # (start_event, end_event, bytes, kind)

    def step(record):
        for i in range(P):
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            sk.sketch_gen_matmul(shares[i], seed, k, Y=Yrows[i * w:(i + 1) * w], stream=stream)
            if record:
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(stream)
                launches.append((e0, e1, share_bytes, "row"))
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        sk.sketch_gen_matmul_reduce(blocks, row0s, seed, k, Y=Yred, stream=stream)
        if record:
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record(stream)
            launches.append((e0, e1, red_bytes, "col"))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    same = bool(torch.equal(Yrows, Yred))
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        step(True)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    step_bytes = P * share_bytes + red_bytes
    value = step_bytes * args.steps / (total_ms * 1e-3) / 1e9

    dur = {"row": [], "col": []}
    for e0, e1, nb, kind in launches:
        dur[kind].append((e0.elapsed_time(e1), nb))
    tot_b = sum(nb for v in dur.values() for _, nb in v)
    tot_ms = sum(ms for v in dur.values() for ms, _ in v)
    achieved = tot_b / (tot_ms * 1e-3) / 1e9
    n_launch = sum(len(v) for v in dur.values())
    rate = {kd: sum(b for _, b in v) / (sum(ms for ms, _ in v) * 1e-3) / 1e9
            for kd, v in dur.items()}
    avg_us = {kd: 1e3 * sum(ms for ms, _ in v) / len(v) for kd, v in dur.items()}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "A 32768x32768 fp32 N(0,1) (torch generator, seed 0), Omega "
                               "N(0,1) Philox4x32-10 seed 1, k=5; P=8 shares on one GPU: "
                               "row layout (8 x sketch_gen_matmul on 4096-row blocks) + column "
                               "layout (sketch_gen_matmul_reduce on 8 4096-column blocks, "
                               "FP64 device sum)",
                   "m": N, "n": N, "k": k, "P": P, "bytes_per_step": step_bytes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None,
                     "kernel": "k_gemm_stream<5,f32,gen>",
                     "launches": n_launch,
                     "avg_launch_us": round(1e3 * tot_ms / n_launch, 2)},
        "extra": {"hbm_frac_of_value": round(value / HBM_PEAK_GBPS, 4),
                  "row_layout_GBps": round(rate["row"], 1),
                  "col_layout_GBps": round(rate["col"], 1),
                  "row_launch_us": round(avg_us["row"], 2),
                  "col_launch_us": round(avg_us["col"], 2),
                  "row_equals_col_bitwise": same,
                  "tflops": round(2 * N * N * k * 2 * args.steps / (total_ms * 1e-3) / 1e12, 3)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, k, seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
