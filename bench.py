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

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ragged|d4bc|c2|wc|elastic|elastic_f32|table1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# exact elastic field: both passes run their multiply-adds two per lane and clock (v_dot2c_i32_i16)
# when the taps fit 16 bits (sigma 50 here)
INT32_MAC_TMACS = 256 * 64 * 2.4e9 / 1e12
FIELD_PEAK_TMACS = 2 * INT32_MAC_TMACS
FP32_PEAK_TFLOPS = 157.3


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--min-warmup-s", type=float, default=1.0,
                   help="after the W warm-up steps, keep running untimed steps until this much time has passed "
                        "(GPU clocks reach their working level only after some back-to-back work)")
    p.add_argument("--workload", default="ragged")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--variant", type=int, default=-1,
                   help="ragged launch variant; -1 runs the autotuner (outside the timed region)")
    return p.parse_args()


def profiled_traffic(profile: str, variant_name: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary of
    a kernel, or None when the kernel source or the launch variant has changed
    since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(" "))
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1809_06839_amd", "csrc")
    h = hashlib.sha256()
    for f in ("k_ragged.hip", "k_rows.hip", "k_gather.hip", "ragged_common.h", "dev_common.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    if fields.get("kernel_source_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    # one entry per launch variant the counters were taken on: variant / traffic_bytes_per_launch,
    # variant_1 / traffic_bytes_per_launch_1, ...
    for sfx in [""] + ["_%d" % i for i in range(1, 8)]:
        if fields.get("variant" + sfx, "").strip() == variant_name:
            try:
                return int(fields["traffic_bytes_per_launch" + sfx].split()[0])
            except (KeyError, ValueError):
                return None
    return None


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


def ragged_kernel_name(variant_name: str) -> str:
    """Kernel that a ragged launch variant runs."""
    if "row bands" in variant_name:
        return "k_rows"
    if "row gathers" in variant_name:
        return "k_gather"
    if "double-buffered" in variant_name:
        return "k_ragged_pipe6"
    if "planning wave" in variant_name:
        return "k_ragged_pipe5"
    if "next pass planned" in variant_name:
        return "k_ragged_pipe"
    if "streaming" in variant_name:
        return "k_ragged_stream"
    if "flat" in variant_name:
        return "k_ragged_flat"
    return "k_ragged_persistent"


def cpu_baseline_ragged(b, flags, ab, seconds):
    import oracle
    oracle.lib()

    def one(i):
        oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), 224, 224)
    return cpu_oracle_rates(one, b.n, seconds, "images of the same 2048-image batch, C oracle")


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
    variants = m.ragged_variants()
    if args.variant >= 0:
        variant = args.variant
        ctx.set_variant(variant)
        print("# variant %d (%s) forced" % (variant, variants[variant]), file=sys.stderr, flush=True)
    else:
        variant, tune_ms, tune_times = m.ragged_autotune(ctx, r, reps=3, return_times=True)
        for i, t in enumerate(tune_times):
            print("#   variant %d (%s): %.3f ms" % (i, variants[i], t), file=sys.stderr, flush=True)
        print("# autotuner chose variant %d (%s), %.3f ms" % (variant, variants[variant], tune_ms), file=sys.stderr,
              flush=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = m.Graph(ctx, r, s)
        warm_up(lambda st: g.launch(st), args, s)
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
        # the op-list form: the same chain compiled from an op list, replayed through
        # miaug_pipeline_graph_launch with fresh records every step (sampled on the
        # host while the previous step runs)
        pipe = m.Pipeline(ctx, [m.op("HFLIP", 0.5), m.op("VFLIP", 0.5), m.op("ROT90", 1, (0,), (3,)),
                                m.op("TRANSPOSE", 0.5), m.op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)),
                                m.op("RESIZE", out=(224, 224)), m.op("NORMALIZE", 1, m.IMAGENET_MEAN, m.IMAGENET_STD)])
        bi, bo, _ = pipe.batch(ragged=r)
        pg = pipe.graph(bi, bo, s)
        for j in range(max(2, args.warmup)):
            pg.launch(pipe.sample(1809068393, j * n, n), s)
        s.synchronize()
        e0.record(s)
        for j in range(args.steps):
            pg.launch(pipe.sample(1809068393, (j + 1000) * n, n), s)
        e1.record(s)
        s.synchronize()
        ms_pg = e0.elapsed_time(e1) / args.steps
        pg.close()
        pipe.close()
    g.close()
    alg = ragged_algorithmic_bytes(b.hw, len(b.boxes))
    achieved = alg / (ms * 1e-3) / 1e9
    res = {
        "metric": "images/sec and HBM GB/s (% peak) for batched augment pipeline; batched vs per-image",
        "value": n / (ms * 1e-3), "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "min_warmup_s": args.min_warmup_s,
        "ms_per_step": ms, "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "ragged_d4_bc_resize224_normalize_f32", "global_batch": n,
                   "sizes": "H,W~U{128..1024}", "masks": "21 labels", "boxes": "0-16 per image",
                   "launch": "one launch in a hipGraph, %s: %s" % ("forced" if args.variant >= 0 else "autotuned",
                                                                   variants[variant]),
                   "parallelism": "single GPU"},
        "per_image_launches": {"value": n / (ms_pi * 1e-3), "unit": "images/s", "ms_per_step": ms_pi,
                               "batched_speedup": ms_pi / ms},
        "pipeline_graph": {"value": n / (ms_pg * 1e-3), "unit": "images/s", "ms_per_step": ms_pg,
                           "form": "op-list pipeline, miaug_pipeline_graph_launch, fresh records per step"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("k_gather_2048img_ragged_to_224_f32.md", variants[variant]),
                     "kernel": ragged_kernel_name(variants[variant]), "algorithmic_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_ragged(b, flags, ab, args.cpu_seconds)
    return res


def warm_up(fn, args, s):
    """W untimed calls of fn(s), then more until --min-warmup-s seconds have passed."""
    for _ in range(args.warmup):
        fn(s)
    s.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < args.min_warmup_s:
        for _ in range(4):
            fn(s)
        s.synchronize()


MIN_WARMUP_S = 1.0  # set from --min-warmup-s


def time_on_stream(torch, fn, steps, warmup, s, min_warmup_s=None):
    """Average ms of fn(s) over `steps` calls on stream s, HIP events around the loop, after
    `warmup` untimed calls and more until min_warmup_s (default --min-warmup-s) seconds have passed."""
    if min_warmup_s is None:
        min_warmup_s = MIN_WARMUP_S
    with torch.cuda.stream(s):
        for _ in range(warmup):
            fn(s)
        s.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < min_warmup_s:
            for _ in range(4):
                fn(s)
            s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(steps):
            fn(s)
        e1.record(s)
        s.synchronize()
    return e0.elapsed_time(e1) / steps


def line(metric, n, ms, args, dtype, config, roofline, extra=None):
    res = {"metric": metric, "value": n / (ms * 1e-3), "unit": "images/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "min_warmup_s": args.min_warmup_s, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline}
    if extra:
        res.update(extra)
    return res


ROTATE_BYTES = 1 << 30  # inputs + outputs cycled per step, so no step finds its data in the 256 MB MALL


def n_sets(set_bytes):
    """Copies of a workload's buffers that together reach ROTATE_BYTES."""
    return max(1, -(-ROTATE_BYTES // int(set_bytes)))


def time_rotating(torch, fn, sets, steps, warmup, s):
    """time_on_stream over fn(st, k): call i uses buffer set i mod `sets`."""
    i = [0]

    def call(st):
        fn(st, i[0] % sets)
        i[0] += 1
    return time_on_stream(torch, call, steps, warmup, s)


def host_cpu():
    """Model name and logical CPU count of the host."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def pool_threads():
    """Threads for the all-core oracle timing: the host's CPUs, at most the 16
    that a one-GPU share of the machine gets (OMP_NUM_THREADS when set)."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    n = int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    return max(1, min(n, os.cpu_count() or 1, 16))


def cpu_oracle_rates(one, n_items, seconds, what):
    """The oracle's throughput on a bounded sample: one(i) processes item i
    (a call into the C oracle, which releases the GIL); items cycle through
    0 .. n_items - 1.  First single-threaded for about seconds / 2, then on a
    thread pool for about seconds / 2; returns the cpu_baseline record
    (value: all cores)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    done1 = 0
    while time.perf_counter() - t0 < seconds / 2:
        one(done1 % n_items)
        done1 += 1
    dt1 = time.perf_counter() - t0
    th = pool_threads()
    t0 = time.perf_counter()
    doneN = 0
    with ThreadPoolExecutor(th) as ex:
        while time.perf_counter() - t0 < seconds / 2:
            list(ex.map(lambda i: one(i % n_items), range(doneN, doneN + 4 * th)))
            doneN += 4 * th
    dtN = time.perf_counter() - t0
    model, nproc = host_cpu()
    return {"value": doneN / dtN, "unit": "images/s", "cores": th, "kind": "oracle",
            "sample": "%s, cycled: %d on %d threads in %.1f s (single thread: %d in %.1f s)"
                      % (what, doneN, th, dtN, done1, dt1),
            "single_thread": {"value": done1 / dt1, "unit": "images/s", "cores": 1},
            "cpu_model": model, "nproc": nproc}


def hbm_roof(alg_bytes, ms, kernel):
    a = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernel, "algorithmic_bytes_per_launch": alg_bytes}


def bench_d4bc(args, torch, m):
    """64 RGB 256x256 u8 images: random Dih4 element + brightness/contrast.  The
    batch is 25 MB, so a step replays a hipGraph of 40 batch launches, each on
    its own copy of the buffers (41 copies, 1 GiB, cycled)."""
    import synth
    n, H, W = 64, 256, 256
    img = synth.uniform_u8(1809068391, n, H, W).cuda()
    flags, ab = m.sample_d4bc(1809068391, 0, n)
    fl, abt = torch.from_numpy(flags).cuda(), torch.from_numpy(ab).cuda()
    alg = 2 * n * H * W * 3
    K = n_sets(alg)
    imgs = [img] + [img.clone() for _ in range(K - 1)]
    outs = [torch.empty_like(img) for _ in range(K)]
    per_graph = 40
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for k in range(K):
            m.d4_bc_u8(imgs[k], fl, abt, outs[k], s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for j in range(per_graph):
            m.d4_bc_u8(imgs[j % K], fl, abt, outs[j % K], torch.cuda.current_stream())
    ms_graph = time_on_stream(torch, lambda st: g.replay(), args.steps, args.warmup, s)
    ms = ms_graph / per_graph
    ms_eager = time_rotating(torch, lambda st, k: m.d4_bc_u8(imgs[k], fl, abt, outs[k], st), K, args.steps,
                             args.warmup, s)
    res = line("images/sec and HBM GB/s (% peak), plain Dih4 + brightness/contrast", n, ms, args, "u8",
               {"workload": "d4_brightness_contrast_64x256x256x3",
                "timing": "%d batch launches per hipGraph replay, %d buffer copies (%.2f GB) cycled"
                          % (per_graph, K, K * alg / 1e9)},
               hbm_roof(alg, ms, "k_d4_bc<3>"), {"eager_ms_per_batch": ms_eager})
    if not args.no_cpu_baseline:
        import oracle
        x = img.cpu().numpy()
        res["cpu_baseline"] = cpu_oracle_rates(
            lambda i: oracle.pipe_d4bc(x[i:i + 1], flags[i:i + 1], ab[i:i + 1]), n, args.cpu_seconds,
            "images of the 64-image batch, C oracle")
    return res


def bench_c2(args, torch, m):
    """256 smooth-noise RGB 512x512 u8 images: shift-scale-rotate -> crop 448 -> 224 -> HSV -> gamma -> blur."""
    import synth
    n = 256
    img = synth.smooth_u8_hwc(1809068392, n, 512, 512, device="cuda")
    f, k = m.sample_c2(1809068392, 0, n)
    rec = torch.from_numpy(m.compile_c2(f, k, 512, 512, 448)).cuda()
    alg = n * (512 * 512 * 3 + 224 * 224 * 3)
    K = n_sets(alg)
    imgs = [img] + [img.clone() for _ in range(K - 1)]
    outs = [torch.empty((n, 224, 224, 3), dtype=torch.uint8, device="cuda") for _ in range(K)]
    s = torch.cuda.Stream()
    ms = time_rotating(torch, lambda st, j: m.ssr_crop_resize_hsv_gamma_blur_u8(imgs[j], rec, 448, 224, outs[j], st),
                       K, args.steps, args.warmup, s)
    res = line("images/sec and HBM GB/s (% peak), full u8 pipeline", n, ms, args, "u8",
               {"workload": "ssr_crop448_resize224_hsv_gamma_blur_256x512x512x3",
                "timing": "%d buffer copies (%.2f GB) cycled" % (K, K * alg / 1e9)}, hbm_roof(alg, ms, "k_c2"))
    if not args.no_cpu_baseline:
        import oracle
        x = img.cpu().numpy()
        res["cpu_baseline"] = cpu_oracle_rates(lambda i: oracle.pipe_c2_one(x[i], f[i], k[i]), n, args.cpu_seconds,
                                               "images of the 256-image batch, C oracle")
    return res


def bench_wc(args, torch, m):
    """128 x 3 x 224 x 224 float32: differentiable warp + colour, forward + backward."""
    import synth
    n, C, H, W = 128, 3, 224, 224
    x = synth.smooth_noise(1809068394, n, H, W, C, device="cuda")
    p = torch.from_numpy(m.sample_wc(1809068394, 0, n)).cuda()
    g = torch.Generator().manual_seed(5)
    w = (torch.rand((n, C, H, W), generator=g) * 2 - 1).cuda()
    plane = n * C * H * W * 4
    K = n_sets(4 * plane)  # x, y, dL/dy, grad_x per copy
    xs = [x] + [x.clone() for _ in range(K - 1)]
    ws_ = [w] + [w.clone() for _ in range(K - 1)]
    ys = [torch.empty_like(x) for _ in range(K)]
    gxs = [torch.empty_like(x) for _ in range(K)]
    gp = torch.empty_like(p)
    ws = torch.empty(m.lib().miaug_warpcolor_workspace_bytes(n, C, H, W), dtype=torch.uint8, device="cuda")
    L = m.lib()

    def fwd(st, k):
        m._check(L.miaug_warpcolor_fwd(m._p(xs[k]), n, C, H, W, m._p(p), m._p(ys[k]), m._stream(st)))

    def bwd(st, k):
        m._check(L.miaug_warpcolor_bwd(m._p(xs[k]), n, C, H, W, m._p(p), m._p(ws_[k]), m._p(gxs[k]), m._p(gp),
                                       m._p(ws), ws.numel(), m._stream(st)))

    s = torch.cuda.Stream()
    ms = time_rotating(torch, lambda st, k: (fwd(st, k), bwd(st, k)), K, args.steps, args.warmup, s)
    ms_f = time_rotating(torch, fwd, K, args.steps, args.warmup, s)
    ms_b = time_rotating(torch, bwd, K, args.steps, args.warmup, s)
    alg = 2 * plane + 3 * plane  # forward x, y; backward gy, x, grad_x
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        xh, ph, wh = x.cpu().numpy(), p.cpu().numpy().astype(np.float64), w.cpu().numpy().astype(np.float64)

        def one(i):
            oracle.wc_forward(xh[i], ph[i])
            oracle.wc_backward(xh[i], ph[i], wh[i])
        cpu = cpu_oracle_rates(one, n, args.cpu_seconds, "images of the 128-image batch, fp64 C oracle forward + "
                                                          "backward")
    res = line("images/sec and HBM GB/s (% peak), differentiable warp + colour fwd+bwd", n, ms, args, "f32",
                {"workload": "warpcolor_fwd_bwd_128x3x224x224_f32",
                 "timing": "%d buffer copies (%.2f GB) cycled" % (K, K * 4 * plane / 1e9)},
                hbm_roof(alg, ms, "k_wc_* (fwd + bwd)"),
                {"forward_ms": ms_f, "forward_roofline": hbm_roof(2 * plane, ms_f, "k_wc_fwd"),
                 "backward_ms": ms_b, "backward_roofline": hbm_roof(3 * plane, ms_b, "k_wc_bwd + k_wc_reduce")})
    if cpu:
        res["cpu_baseline"] = cpu
    return res


def bench_elastic(args, torch, m):
    """16 RGB 4096x4096 u8 images + 8-label masks: elastic (sigma 50, alpha 1000) + 5x5 grid (0.3)."""
    import synth
    n, H, W = 16, 4096, 4096
    img = torch.cat([synth.smooth_u8_hwc(1809068395 + i, 1, H, W, 3, device="cuda") for i in range(n)])
    mask = torch.cat([synth.blob_masks(1809068396 + i, 1, H, W, 8, 512, device="cuda") for i in range(n)])
    grid = torch.from_numpy(m.sample_grid(1809068395, 0, n)).cuda()
    off = torch.empty((n, 2, H, W), dtype=torch.int32, device="cuda")
    ws = torch.empty(m.lib().miaug_elastic_workspace_bytes(n, H, W), dtype=torch.uint8, device="cuda")
    mapx = torch.empty((n, W), dtype=torch.int32, device="cuda")
    mapy = torch.empty((n, H), dtype=torch.int32, device="cuda")
    out = torch.empty_like(img)
    om = torch.empty_like(mask)
    L = m.lib()

    def fields(st):
        m._check(L.miaug_elastic_fields(1809068395, 0, n, H, W, 50.0, 1000, 150, m._p(off), m._p(ws), ws.numel(),
                                         m._stream(st)))
        m._check(L.miaug_grid_tables(m._p(grid), n, H, W, m._p(mapx), m._p(mapy), m._stream(st)))

    def remap(st, per_image=0):
        m._check(L.miaug_elastic_grid_u8(m._p(img), m._p(mask), n, H, W, 3, m._p(off), m._p(mapx), m._p(mapy),
                                         m._p(out), m._p(om), per_image, m._stream(st)))

    ws_box = torch.empty(m.lib().miaug_elastic_box_workspace_bytes(n, H, W), dtype=torch.uint8, device="cuda")

    def fields_box(st):
        m._check(L.miaug_elastic_fields_box(1809068395, 0, n, H, W, 50.0, 1000, m._p(off), m._p(ws_box),
                                             ws_box.numel(), m._stream(st)))

    s = torch.cuda.Stream()
    steps = max(1, args.steps // 4)
    ms_fb = time_on_stream(torch, fields_box, steps, 1, s)
    ms_f = time_on_stream(torch, fields, steps, 1, s)
    ms_r = time_on_stream(torch, remap, args.steps, args.warmup, s)
    ms_ri = time_on_stream(torch, lambda st: remap(st, 1), steps, 1, s)
    macs = n * 2 * H * W * 301 * 2
    alg = n * H * W * (3 + 1) * 2
    ms = ms_f + ms_r
    res = line("images/sec, large-tile elastic + grid distortion (fields + remap)", n, ms, args, "u8",
               {"workload": "elastic_grid_16x4096x4096x3_masks"}, hbm_roof(alg, ms_r, "k_remap_chain_u8"),
               {"field_ms": ms_f, "remap_ms": ms_r, "remap_per_image_launch_ms": ms_ri,
                "field_roofline": {"bound": "alu", "achieved": macs / (ms_f * 1e-3) / 1e12,
                                   "peak": FIELD_PEAK_TMACS,
                                   "unit": "Tmac/s (packed 16-bit multiply-adds into int32)",
                                   "frac": macs / (ms_f * 1e-3) / 1e12 / FIELD_PEAK_TMACS},
                "box_field_ms": ms_fb, "box_field_speedup": ms_f / ms_fb,
                "box_field_roofline": hbm_roof(n * 2 * H * W * 4, ms_fb, "k_box_rows + 3 x k_box_cols2")})
    return res


def bench_elastic_f32(args, torch, m):
    """Float copy of the elastic + grid chain (the training-time form, backward on a
    float32 copy): 16 x 3 x 4096 x 4096 float32, fields sigma 50 / alpha 1000 and a
    5x5 grid (0.3), forward and backward timed apart."""
    import synth
    n, C, H, W = 16, 3, 4096, 4096
    x = torch.cat([synth.smooth_noise(1809068395 + i, 1, H, W, C, device="cuda") for i in range(n)])
    g = torch.Generator(device="cuda").manual_seed(1809068399)
    gy = torch.rand((n, C, H, W), generator=g, device="cuda") * 2 - 1
    grid = torch.from_numpy(m.sample_grid(1809068395, 0, n)).cuda()
    off = torch.empty((n, 2, H, W), dtype=torch.int32, device="cuda")
    wsf = torch.empty(m.lib().miaug_elastic_workspace_bytes(n, H, W), dtype=torch.uint8, device="cuda")
    mapx = torch.empty((n, W), dtype=torch.int32, device="cuda")
    mapy = torch.empty((n, H), dtype=torch.int32, device="cuda")
    L = m.lib()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        m._check(L.miaug_elastic_fields(1809068395, 0, n, H, W, 50.0, 1000, 150, m._p(off), m._p(wsf), wsf.numel(),
                                         m._stream(s)))
        m._check(L.miaug_grid_tables(m._p(grid), n, H, W, m._p(mapx), m._p(mapy), m._stream(s)))
    s.synchronize()
    del wsf
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    ws = torch.empty(L.miaug_chain_f32_workspace_bytes(n, C, H, W), dtype=torch.uint8, device="cuda")

    def fwd(st):
        m._check(L.miaug_elastic_grid_f32_fwd(m._p(x), n, C, H, W, m._p(off), m._p(mapx), m._p(mapy), m._p(y),
                                               m._p(ws), ws.numel(), m._stream(st)))

    def bwd(st):
        m._check(L.miaug_elastic_grid_f32_bwd(m._p(gy), n, C, H, W, m._p(off), m._p(mapx), m._p(mapy), m._p(gx),
                                               m._p(ws), ws.numel(), m._stream(st)))

    steps = max(2, args.steps // 4)
    ms_f = time_on_stream(torch, fwd, steps, 1, s)
    ms_b = time_on_stream(torch, bwd, steps, 1, s)
    plane = n * C * H * W * 4
    offb = n * 2 * H * W * 4
    alg = plane + offb + plane  # per direction: image in, the elastic offsets, image out (maps are KB)
    res = line("images/sec and HBM GB/s (% peak), float32 elastic + grid chain forward + backward", n, ms_f + ms_b,
               args, "f32", {"workload": "elastic_grid_f32_16x3x4096x4096"},
               hbm_roof(2 * alg, ms_f + ms_b, "k_chain_f_* (forward + backward)"),
               {"forward_ms": ms_f, "forward_roofline": hbm_roof(alg, ms_f, "k_chain_f_elastic + k_chain_f_grid"),
                "backward_ms": ms_b,
                "backward_roofline": hbm_roof(alg, ms_b, "k_chain_f_grid_adj + k_chain_f_elastic_adj")})
    res["steps"] = steps
    return res


def bench_stats(args, torch, m):
    """Per-image statistics (sum, min, max, 256-bin histogram per channel) of 256
    smooth-noise RGB 512x512 u8 images, buffers cycled over >= 1 GiB."""
    import synth
    n, S = 256, 512
    img = synth.smooth_u8_hwc(1809068397, n, S, S, device="cuda")
    alg = img.numel()
    K = n_sets(alg)
    imgs = [img] + [img.clone() for _ in range(K - 1)]
    L = m.lib()
    sm = torch.empty((n, 3), dtype=torch.int64, device="cuda")
    mn = torch.empty((n, 3), dtype=torch.int32, device="cuda")
    mx = torch.empty((n, 3), dtype=torch.int32, device="cuda")
    h = torch.empty((n, 3, 256), dtype=torch.int32, device="cuda")

    def fn(st, k):
        m._check(L.miaug_image_stats_u8(m._p(imgs[k]), n, S * S, 3, m._p(sm), m._p(mn), m._p(mx), m._p(h),
                                         m._stream(st)))
    s = torch.cuda.Stream()
    ms = time_rotating(torch, fn, K, args.steps, args.warmup, s)
    return line("images/sec and HBM GB/s (% peak), per-image statistics", n, ms, args, "u8",
                {"workload": "image_stats_256x512x512x3",
                 "timing": "%d buffer copies (%.2f GB) cycled" % (K, K * alg / 1e9)}, hbm_roof(alg, ms, "k_stats"))


def bench_copy(args, torch, m):
    """Plain device-to-device copy of 1 GiB: the reference for scaling the HBM
    byte counters (FETCH_SIZE, WRITE_SIZE) of the other kernels."""
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.Stream()
    ms = time_on_stream(torch, lambda st: b.copy_(a), args.steps, args.warmup, s)
    gbs = 2 * n / (ms * 1e-3) / 1e9
    return {"metric": "copy GB/s (read + write)", "value": gbs, "unit": "GB/s", "bytes_read": n, "bytes_written": n,
            "ms_per_step": ms, "steps": args.steps, "config": {"workload": "copy_1GiB"}}


def bench_table1(args, torch, m):
    """Every row of the paper's Table I as a single op on 256 smooth-noise RGB 512x512 u8 images
    (PadToSize512 pads 448x448 images), one GPU launch per op and batch."""
    import synth
    n, S = 256, 512
    img = synth.smooth_u8_hwc(1809068397, n, S, S, device="cuda")
    small = synth.smooth_u8_hwc(1809068398, n, 448, 448, device="cuda")
    K = n_sets(2 * img.numel())  # every op reads and writes about one batch per step
    imgs = [img] + [img.clone() for _ in range(K - 1)]
    smalls = [small] + [small.clone() for _ in range(K - 1)]
    outs = [torch.empty_like(img) for _ in range(K)]
    s = torch.cuda.Stream()
    rng = np.random.default_rng(1809068397)
    zero_fl = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    fl_h = zero_fl.clone(); fl_h[:, 0] = 1
    fl_v = zero_fl.clone(); fl_v[:, 1] = 1
    ab = torch.from_numpy(np.stack([rng.uniform(0.8, 1.2, n), rng.uniform(-51, 51, n)], 1).astype(np.float32)).cuda()
    ident_ab = torch.tensor([[1.0, 0.0]] * n, dtype=torch.float32, device="cuda")
    sh = rng.uniform(-20, 20, (n, 3)).astype(np.float32)
    luts_rgb = torch.from_numpy(m.compile_color_luts(None, sh, n)).cuda()
    luts_id = torch.from_numpy(m.compile_color_luts(None, None, n)).cuda()
    gray = torch.ones(n, dtype=torch.int32, device="cuda")
    f_rot = np.stack([rng.uniform(-45, 45, n), np.ones(n), np.zeros(n), np.zeros(n)], 1).astype(np.float32)
    f_ssr = np.stack([rng.uniform(-45, 45, n), rng.uniform(0.9, 1.1, n), rng.uniform(-0.0625, 0.0625, n),
                      rng.uniform(-0.0625, 0.0625, n)], 1).astype(np.float32)
    aq_rot = torch.from_numpy(m.compile_ssr_q32(f_rot, S, S)).cuda()
    aq_ssr = torch.from_numpy(m.compile_ssr_q32(f_ssr, S, S)).cuda()

    def c2_rec(f5, k5, crop):
        return torch.from_numpy(m.compile_c2(np.asarray(f5, np.float32), np.asarray(k5, np.int32), S, S, crop)).cuda()
    ident_f = [[0.0, 1.0, 0.0, 0.0, 1.0]] * n
    dhsv = torch.tensor([[int(rng.integers(-20, 21)), int(rng.integers(-30, 31)), 0] for _ in range(n)],
                        dtype=torch.int32, device="cuda")
    luts_gam = torch.from_numpy(m.compile_gamma_luts(np.array([rng.uniform(0.8, 1.2) for _ in range(n)],
                                                              np.float32))).cuda()
    rec_crop = c2_rec(ident_f, [[int(rng.integers(0, S - 63)), int(rng.integers(0, S - 63)), 0, 0, 0]
                                for _ in range(n)], 64)
    out64 = torch.empty((n, 64, 64, 3), dtype=torch.uint8, device="cuda")
    px = n * S * S * 3
    # each op is fn(stream, k): buffer copy k of the K cycled ones
    ops = [
        ("RandomCrop64", lambda st, k: m.ssr_crop_resize_hsv_gamma_blur_u8(imgs[k], rec_crop, 64, 64, out64, st),
         2 * n * 64 * 64 * 3, "k_c2 (identity warp, 64x64 crop)"),
        ("PadToSize512", lambda st, k: m.pad_u8(smalls[k], S, S, 0, 0, outs[k], st), n * (448 * 448 * 3) + px,
         "k_pad<3>"),
        ("HorizontalFlip", lambda st, k: m.d4_bc_u8(imgs[k], fl_h, ident_ab, outs[k], st), 2 * px, "k_d4_bc<3>"),
        ("VerticalFlip", lambda st, k: m.d4_bc_u8(imgs[k], fl_v, ident_ab, outs[k], st), 2 * px, "k_d4_bc<3>"),
        ("Rotate", lambda st, k: m.warp_affine_u8(imgs[k], aq_rot, 0, 0, outs[k], st), 2 * px, "k_warp<3>"),
        ("ShiftScaleRotate", lambda st, k: m.warp_affine_u8(imgs[k], aq_ssr, 0, 0, outs[k], st), 2 * px,
         "k_warp<3>"),
        ("Brightness", lambda st, k: m.d4_bc_u8(imgs[k], zero_fl, ab, outs[k], st), 2 * px, "k_d4_bc<3>"),
        ("ShiftHSV", lambda st, k: m.hsv_shift_u8(imgs[k], dhsv, outs[k], st), 2 * px, "k_hsv_u8"),
        ("ShiftRGB", lambda st, k: m.d4_lut_u8(imgs[k], zero_fl, luts_rgb, None, outs[k], st), 2 * px,
         "k_d4_bc<3, LUTs>"),
        ("Gamma", lambda st, k: m.d4_lut_u8(imgs[k], zero_fl, luts_gam, None, outs[k], st), 2 * px,
         "k_d4_bc<3, LUTs>"),
        ("Grayscale", lambda st, k: m.d4_lut_u8(imgs[k], zero_fl, luts_id, gray, outs[k], st), 2 * px,
         "k_d4_bc<3, gray>"),
    ]
    extra = [  # not Table I rows: the blur of the u8 chain, alone, on the same batch
        ("Blur3x3", lambda st, k: m.blur_u8(imgs[k], 3, None, outs[k], st), 2 * px, "k_blur<3, 1>"),
        ("Blur5x5", lambda st, k: m.blur_u8(imgs[k], 5, None, outs[k], st), 2 * px, "k_blur<3, 2>"),
    ]
    extra_rows = {}
    for name, fn, alg, kernel in extra:
        ms = time_rotating(torch, fn, K, args.steps, args.warmup, s)
        extra_rows[name] = {"ms_per_batch": ms, "images_per_s": n / (ms * 1e-3), "gb_per_s": alg / (ms * 1e-3) / 1e9,
                            "kernel": kernel}
        print("# %-16s %8.3f ms  %10.0f img/s  %7.0f GB/s (not a Table I row)" % (name, ms, n / (ms * 1e-3),
              extra_rows[name]["gb_per_s"]), file=sys.stderr, flush=True)
    rows = {}
    for name, fn, alg, kernel in ops:
        ms = time_rotating(torch, fn, K, args.steps, args.warmup, s)
        rows[name] = {"ms_per_batch": ms, "images_per_s": n / (ms * 1e-3), "gb_per_s": alg / (ms * 1e-3) / 1e9,
                      "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "kernel": kernel}
        print("# %-16s %8.3f ms  %10.0f img/s  %7.0f GB/s" % (name, ms, n / (ms * 1e-3), rows[name]["gb_per_s"]),
              file=sys.stderr, flush=True)
    total = sum(r["ms_per_batch"] for r in rows.values())
    res = line("images/sec per Table I op (one launch per op), 256 x 512x512x3 u8", n * len(rows), total, args, "u8",
               {"workload": "table1_single_ops_256x512x512x3",
                "timing": "%d buffer copies (%.2f GB) cycled" % (K, K * 2 * px / 1e9)}, None,
               {"ops": rows, "other_ops": extra_rows})
    res["value"] = n / (total * 1e-3) * len(rows)
    res["unit"] = "op-images/s"
    return res


WORKLOADS = {"table1": bench_table1, "copy": bench_copy, "ragged": bench_ragged, "d4bc": bench_d4bc, "c2": bench_c2, "wc": bench_wc, "elastic": bench_elastic,
             "elastic_f32": bench_elastic_f32, "stats": bench_stats}


def main():
    args = parse()
    global MIN_WARMUP_S
    MIN_WARMUP_S = args.min_warmup_s
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
