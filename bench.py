#!/usr/bin/env python3
"""Benchmark of the MI355X augmentation path (one GPU).

Default workload (the batched ragged pipeline): 2048 RGB u8 images with
H, W ~ U{128..1024}, 21-label blob masks and 0..16 boxes each; per image a
random Dih4 element + brightness/contrast, bilinear resize to 224x224 and
per-channel normalisation into float32 NCHW, masks nearest, boxes
transformed -- one persistent launch replayed from a hipGraph, launch variant
chosen by the autotuner.  A step is one pass over the whole batch; inputs are
resident in HBM before timing starts.

Prints ONE JSON line: images/s of the batched form (value), the per-image
launch form for comparison, the roofline of the dominant kernel (algorithmic
bytes per launch / average launch time, HIP events on the launch stream), and
the oracle's CPU throughput on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ragged|d4bc|c2|wc|elastic]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="ragged")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def resize_rows_touched(L: int, out: int = 224) -> int:
    """Distinct source lines the bilinear taps of a resize L -> out read
    (positions ((2j+1)L - out)/(2 out), clamped taps floor and floor + 1)."""
    j = np.arange(out, dtype=np.int64)
    num = ((2 * j + 1) * L - out) * 1024
    q = np.floor_divide(num, 2 * out)
    r = num - q * 2 * out
    q = q + ((2 * r > 2 * out) | ((2 * r == 2 * out) & (q % 2 == 1)))
    f = np.floor_divide(q, 1024)
    return len(np.unique(np.clip(np.concatenate([f, f + 1]), 0, L - 1)))


def resize_rows_nearest(L: int, out: int = 224) -> int:
    j = np.arange(out, dtype=np.int64)
    return len(np.unique(np.minimum(((2 * j + 1) * L) // (2 * out), L - 1)))


def ragged_algorithmic_bytes(hw, nboxes, out=224):
    """Bytes the method must move for one batch: every source row a tap reads
    (whole rows: bilinear taps at downscale factors up to 4.6 touch every
    64-byte line of a row), the mask rows the nearest taps read, boxes, and the
    float32 NCHW images, u8 masks and boxes written."""
    total = 0
    for H, W in hw:
        # source rows are resized to `out` lines (output rows, or output columns when the
        # Dih4 element swaps axes; both are `out` long, so the element does not matter)
        total += resize_rows_touched(int(H), out) * int(W) * 3
        total += resize_rows_nearest(int(H), out) * int(W)
    total += len(hw) * out * out * (3 * 4 + 1)
    total += 2 * nboxes * 16
    return total


def cpu_baseline_ragged(b, flags, ab, seconds):
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    done = 0
    while done < b.n:
        oracle.pipe_ragged_one(b.image(done), b.mask_of(done), flags[done], ab[done], b.boxes_of(done), 224, 224)
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": "first %d images of the same 2048-image batch, single-threaded C oracle, %.1f s" % (done, dt)}


def bench_ragged(args, torch, m):
    dev = torch.device("cuda:0")
    n = 2048
    print("# generating 2048-image ragged batch on the GPU", file=sys.stderr, flush=True)
    import synth
    b = synth.ragged_batch(1809068393, n, device=dev)
    flags, ab = m.sample_d4bc(1809068393, 0, n)
    ctx = m.Context(0)
    r = m.Ragged.from_host(b, flags, ab, device=dev)
    torch.cuda.synchronize()
    variant, tune_ms = m.ragged_autotune(ctx, r, reps=3)
    variants = m.ragged_variants()
    print("# autotuner chose variant %d (%s), %.3f ms" % (variant, variants[variant], tune_ms), file=sys.stderr,
          flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = m.Graph(ctx, r, s)
        for _ in range(args.warmup):
            g.launch(s)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s)
        for _ in range(args.steps):
            g.launch(s)
        e1.record(s)
        s.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        # comparison form: the same kernels launched once per image
        pe_steps = max(1, min(5, args.steps))
        m.ragged_apply_per_image(ctx, r, s)
        s.synchronize()
        e0.record(s)
        for _ in range(pe_steps):
            m.ragged_apply_per_image(ctx, r, s)
        e1.record(s)
        s.synchronize()
        ms_pi = e0.elapsed_time(e1) / pe_steps
    g.close()
    alg = ragged_algorithmic_bytes(b.hw, len(b.boxes))
    achieved = alg / (ms * 1e-3) / 1e9
    res = {
        "metric": "images/sec and HBM GB/s (% peak) for batched augment pipeline; batched vs per-image",
        "value": n / (ms * 1e-3), "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "ragged_d4_bc_resize224_normalize_f32", "global_batch": n,
                   "sizes": "H,W~U{128..1024}", "masks": "21 labels", "boxes": "0-16 per image",
                   "launch": "persistent kernel in hipGraph, autotuned: %s" % variants[variant],
                   "parallelism": "single GPU"},
        "per_image_launches": {"value": n / (ms_pi * 1e-3), "unit": "images/s", "ms_per_step": ms_pi,
                               "batched_speedup": ms_pi / ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_ragged_persistent", "algorithmic_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_ragged(b, flags, ab, args.cpu_seconds)
    return res


WORKLOADS = {"ragged": bench_ragged}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (shards would be independent "
              "per-GPU batches); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_1809_06839_amd as m
    m.lib()
    if args.workload not in WORKLOADS:
        print("unknown workload %s (have %s)" % (args.workload, sorted(WORKLOADS)), file=sys.stderr)
        sys.exit(2)
    res = WORKLOADS[args.workload](args, torch, m)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
