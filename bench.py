#!/usr/bin/env python3
"""Benchmark of the non-separable 2-D lifting DWT on one MI355X.

Headline workload: CDF 9/7 forward transform, one level, of one 8192 x 8192
FP32 image (pixels uniform in [0, 1), seed 0), whole-point symmetric borders.
A step is one dwt2_fwd call on that image (timed after the other forms, so
the GPU runs at its steady clocks); inputs are resident in HBM before
the timed region, and three input/output pairs are rotated so that the 256 MB
Infinity Cache cannot serve a step from the previous step's data.  The steps
run back to back; one HIP event pair around the timed region gives the
kernel's average launch time (an event pair per step would add several
microseconds to every step), and a separate sample of 100 individually
bracketed launches gives their spread.

Printed: one JSON line with the contract fields, a `roofline` object for the
level kernel (algorithmic bytes: each pixel read once, each coefficient
written once = 2 * 4 B/px) and a `cpu_baseline` object (the CPU oracle timed
on a bounded crop of the same image).  `forms` lists the other forms of the
path, measured the same way with fewer steps: 5 levels, the P0/P1 split,
inverse, the separable comparison scheme (twice the steps and barriers),
the factored fused steps, real CDF 5/3, BF16 / FP16 storage, reversible
5/3, warm and gradient-input variants, 1024^2 (per call and under graph replay), 4096^2 (cold and warm)
and 16384^2 images, 3 x 8192^2 planes forward + inverse at each storage type
with coefficient error and reconstruction PSNR, the autograd training step
(64 x 3 x 1024^2, forward + adjoint backward), and the batched forward
(eager and graph replay).  `copy_reference` is a plain device copy on the
same buffers; roofline.of_copy is the headline against it.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "level_kernel_fwd_cdf97_f32_8192_traffic.txt")


def kernel_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1704_08657_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size),
    or None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel_source_sha256_16", "").strip() != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # about 0.2 s of warmup brings the GPU to its steady clocks (20 steps
    # read about 1% slower); 1000 timed steps take about 0.1 s
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--no-forms", action="store_true", help="skip the secondary forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tune", action="store_true",
                    help="time every kernel configuration on this GPU first and use the fastest, instead of the "
                         "committed autotuner cache (tuned_configs.json)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--only", default=None, metavar="REGEX",
                    help="run only the forms whose name matches REGEX (the headline always runs)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="accepted for older profiling commands; the plain copy always runs")
    return ap.parse_args()


def algorithmic_bytes(h, w, levels, elem):
    """Compulsory traffic: every level reads its input once and writes its
    h x w outputs once."""
    total = 0
    for _ in range(levels):
        total += 2 * h * w * elem
        h, w = (h + 1) // 2, (w + 1) // 2
    return total


def time_steps(torch, fn, steps, warmup, warm_ms=0.0):
    """Run warmup untimed steps (and more, until at least warm_ms of them
    have run), then time `steps` back-to-back steps.
    Returns (total ms between the synchronisations, the steps' average ms
    from one HIP event pair around the whole timed region on the stream the
    kernels run on).  No event sits between the steps: an event pair per
    step costs several microseconds per step on this GPU."""
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    i = warmup
    while (time.perf_counter() - t0) * 1e3 < warm_ms:
        for _ in range(8):
            fn(i)
            i += 1
        torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(steps):
        fn(i)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    return total_ms, start.elapsed_time(end) / steps


def per_launch_sample(torch, fn, n):
    """Durations (ms) of n launches, each bracketed by its own event pair
    (the pair itself adds a few microseconds to what it brackets)."""
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for i in range(n):
        starts[i].record(stream)
        fn(i)
        ends[i].record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in zip(starts, ends)]


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(x, seconds):
    """The CPU oracle (FP64 NumPy separable lifting, one core) on a 2048 x 2048
    crop of the benchmark image, repeated for about `seconds`."""
    from oracle import lifting
    crop = x[:2048, :2048]
    n = 0
    t0 = time.perf_counter()
    while True:
        lifting.fwd(crop, "cdf97", 1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    gpx = n * crop.size / el / 1e9
    return {"value": gpx, "unit": "Gpixel/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"{n} x CDF 9/7 fwd 1 level on the 2048x2048 top-left crop of the same "
                      f"image, FP64 NumPy, single thread, {el:.1f} s"}


def _pool_job(job):
    """One oracle transform in a worker process: (pixels, seconds)."""
    h, w, seed, levels = job
    from oracle import lifting
    import workloads
    x = workloads.uniform(h, w, seed=seed)
    t0 = time.perf_counter()
    lifting.fwd(x, "cdf97", levels)
    return h * w, time.perf_counter() - t0


def cpu_pool_baseline():
    """The CPU oracle over images of the batched and multi-plane workloads in a
    pool of worker processes (one image per task), on bounded samples: the
    first 24 images of the 256-image uneven batch (5 levels) and the 192
    planes of 1024^2 of the differentiation workload (3 levels).  Run before
    the GPU is initialised; workers = min(16, CPU count)."""
    import multiprocessing as mp
    import workloads
    workers = max(1, min(16, os.cpu_count() or 1))
    out = {}
    samples = {
        "batched: 24 of the 256 uneven images 64..4096, 5 levels":
            [(h, w, 100 + k, 5) for k, (h, w) in enumerate(workloads.uneven_shapes(256, 64, 4096, seed=1)[:24])],
        "planes: 192 x 1024^2 (64 x 3), 3 levels": [(1024, 1024, 200 + k, 3) for k in range(192)],
    }
    ctx = mp.get_context("fork")
    pool = ctx.Pool(workers)
    try:
        for name, jobs in samples.items():
            t0 = time.perf_counter()
            res = pool.map(_pool_job, jobs, chunksize=1)
            el = time.perf_counter() - t0
            px = sum(r[0] for r in res)
            out[name] = {"value": px / el / 1e9, "unit": "Gpixel/s", "seconds": round(el, 2),
                         "pixels": px, "busy_seconds": round(sum(r[1] for r in res), 2)}
    finally:
        # wait for every worker to exit before the GPU is touched, so that
        # no process outlives the benchmark
        pool.close()
        pool.join()
    for child in mp.active_children():
        child.join(5)
    return {"cores": workers, "kind": "oracle", "cpu_model": cpu_model(),
            "method": "multiprocessing pool, one image per task, "
            "FP64 NumPy; wall time includes generating each input in its worker", "samples": out}


def oracle_precision_errors(saved):
    """Coefficient errors of the precision forms against the FP64 oracle (the
    CPU leg of the benchmark, after the GPU timing): for every saved plane,
    the oracle's 5-level forward of the storage-rounded input on the nine
    probe crops (corners, edge midpoints, centre), compared over the crops'
    exactly evaluated part with the GPU's coefficients.  Returns per form the
    largest |gpu - oracle|, the largest |coefficient| and their ratio."""
    from oracle import lifting, window
    out = {}
    for name, (planes_in, planes_coef, lv) in saved.items():
        worst, scale, crops = 0.0, 0.0, 0
        for xp, cp in zip(planes_in, planes_coef):
            H, W = xp.shape
            scale = max(scale, float(np.abs(cp).max()))
            m = window.default_margin(lv)
            for r0, r1, c0, c1 in window.probe_crops(H, W, lv, size=256):
                sub = lifting.fwd(xp[r0:r1, c0:c1].astype(np.float64), "cdf97", lv)
                cut = window.crop_pyramid(cp, lv, r0, r1, c0, c1)
                mask = window.crop_valid_mask(H, W, lv, r0, r1, c0, c1, m)
                worst = max(worst, float(np.abs(cut[mask].astype(np.float64) - sub[mask]).max()))
                crops += 1
        out[name] = {"coeff_max_abs_vs_fp64_oracle": worst, "max_abs_coeff": scale,
                     "coeff_max_abs_rel": worst / scale if scale else None, "oracle_crops": crops}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    # the CPU pool runs before anything touches the GPU (its workers are forked)
    pool = None if args.no_cpu else cpu_pool_baseline()

    import torch
    import paper_1704_08657_amd as d
    import workloads

    dev = torch.device("cuda", 0)
    N = args.size
    px = N * N
    x_host = workloads.uniform(N, N, seed=0)
    pairs = 3
    xs = [torch.from_numpy(x_host).to(dev)]
    for k in range(1, pairs):
        xs.append(xs[0].roll(k, dims=1).contiguous())
    ys = [torch.empty_like(xs[0]) for _ in range(pairs)]
    torch.cuda.synchronize()

    from paper_1704_08657_amd import autotune

    # tile shape: the autotuner's committed cache (tuned_configs.json), or
    # with --tune every kernel configuration timed on this GPU first (untimed,
    # before the warmup) and the fastest used
    tuned = {}

    def tune(name, direction, wavelet, dtype, levels, run):
        if not args.tune:
            return
        best, times = autotune.tune_case(direction, wavelet, dtype, N, N, levels, run)
        tuned[name] = {"config": best, "ms": {str(c): round(t, 5) for c, t in times.items()}}

    tune("headline", "fwd", "cdf97", "f32", 1,
         lambda c, i: d.fwd(xs[i % pairs], "cdf97", 1, out=ys[i % pairs], config=c))

    forms = []
    precision_saved = {}

    def want(name):
        return args.only is None or re.search(args.only, name) is not None

    if not args.no_forms:
        def form(name, fn, levels, elem, steps=50, tune_key=None):
            if not want(name):
                return
            if tune_key is not None:
                tune(name, *tune_key, levels, lambda c, i: fn(i, c))
            # a form right after new buffers or an idle host phase reads up to
            # 15% slow after 30 steps alone (the GPU is still raising its
            # clocks): warm up for at least 25 ms as well
            _, ms = time_steps(torch, lambda i: fn(i, None), steps, 30, warm_ms=25.0)
            ab = algorithmic_bytes(N, N, levels, elem)
            forms.append({"form": name, "Gpixel/s": round(px / (ms * 1e-3) / 1e9, 2),
                          "ms": round(ms, 4), "GB/s": round(ab / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})

        ws5 = d.workspace(N, N, 5, d.DWT2_F32, dev)
        form("cdf97 fwd f32 5 levels", lambda i, c: d.fwd(xs[i % pairs], "cdf97", 5, out=ys[i % pairs], config=c),
             5, 4, tune_key=("fwd", "cdf97", "f32"))
        # the same 5 levels in one persistent launch (levels overlap; every
        # tile publishes its LL rows to the other XCDs, results bit-identical)
        form("cdf97 fwd f32 5 levels, one persistent launch",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 5, out=ys[i % pairs], config=c, persistent=True,
                                workspace=ws5), 5, 4)
        form("cdf97 fwd f32 1 level split P0/P1",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 1, split=True, out=ys[i % pairs], config=c), 1, 4,
             tune_key=None)
        form("cdf97 inv f32 1 level", lambda i, c: d.inv(ys[i % pairs], "cdf97", 1, out=xs[i % pairs], config=c),
             1, 4, tune_key=("inv", "cdf97", "f32"))
        # the hand-written adjoint W^T (transposed fused steps in reverse
        # order, transposed border weights): same bytes as the forward
        form("cdf97 adj f32 1 level", lambda i, c: d.adj(ys[i % pairs], 1, out=xs[i % pairs], config=c),
             1, 4, tune_key=("adj", "cdf97", "f32"))
        form("cdf97 adj f32 5 levels", lambda i, c: d.adj(ys[i % pairs], 5, out=xs[i % pairs], config=c),
             5, 4, tune_key=("adj", "cdf97", "f32"))
        # the separable comparison scheme (8 steps and barriers per level
        # instead of 4), same tile configuration as the fused forms
        form("cdf97 fwd f32 1 level separable (8 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 1, out=ys[i % pairs], config=c, separable=True), 1, 4)
        form("cdf97 inv f32 1 level separable (8 barriers)",
             lambda i, c: d.inv(ys[i % pairs], "cdf97", 1, out=xs[i % pairs], config=c, separable=True), 1, 4)
        form("cdf97 fwd f32 5 levels separable (8 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 5, out=ys[i % pairs], config=c, separable=True), 5, 4)
        # the real-valued CDF 5/3 (one fused predict + update, 2 barriers)
        form("cdf53 real fwd f32 1 level",
             lambda i, c: d.fwd(xs[i % pairs], "cdf53f", 1, out=ys[i % pairs], config=c), 1, 4)
        form("cdf53 real inv f32 1 level",
             lambda i, c: d.inv(ys[i % pairs], "cdf53f", 1, out=xs[i % pairs], config=c), 1, 4)
        # the fused steps evaluated as their two 1-D factors (4 barriers)
        form("cdf97 fwd f32 1 level factored (4 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 1, out=ys[i % pairs], config=c, factored=True), 1, 4)
        form("cdf97 inv f32 1 level factored (4 barriers)",
             lambda i, c: d.inv(ys[i % pairs], "cdf97", 1, out=xs[i % pairs], config=c, factored=True), 1, 4)
        form("cdf97 fwd f32 5 levels factored (4 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 5, out=ys[i % pairs], config=c, factored=True), 5, 4)
        # the LDS-plane kernel (the paper's on-chip-memory design: tile and
        # halo as the four polyphase planes in LDS, one barrier per step):
        # the three schemes of Section "Proposed Schemes" side by side --
        # polyconvolution (one step per lifting pair: 2 barriers), fused
        # lifting (4) and separable lifting (8) -- and DD 13/7 (Section
        # "Evaluation"), which only this kernel runs
        lds_cfg = next(c for c in range(d.DWT2_NUM_KERNEL_CONFIGS)
                       if d.dwt2_kernel_config(c)[1] == d.DWT2_ALGO_LDS)
        for sch, kw in (("polyconvolution (2 barriers)", {"polyconv": True}), ("fused (4 barriers)", {}),
                        ("separable (8 barriers)", {"separable": True})):
            form(f"cdf97 fwd f32 1 level, LDS-plane kernel, {sch}",
                 lambda i, c, kw=kw: d.fwd(xs[i % pairs], "cdf97", 1, out=ys[i % pairs], config=lds_cfg, **kw), 1, 4)
            form(f"cdf97 inv f32 1 level, LDS-plane kernel, {sch}",
                 lambda i, c, kw=kw: d.inv(ys[i % pairs], "cdf97", 1, out=xs[i % pairs], config=lds_cfg, **kw), 1, 4)
        form("cdf97 fwd f32 5 levels, LDS-plane kernel, polyconvolution (2 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "cdf97", 5, out=ys[i % pairs], config=lds_cfg, polyconv=True), 5, 4)
        for sch, kw in (("fused (2 barriers)", {}), ("separable (4 barriers)", {"separable": True})):
            form(f"dd137 fwd f32 1 level, LDS-plane kernel, {sch}",
                 lambda i, c, kw=kw: d.fwd(xs[i % pairs], "dd137", 1, out=ys[i % pairs], config=lds_cfg, **kw), 1, 4)
            form(f"dd137 inv f32 1 level, LDS-plane kernel, {sch}",
                 lambda i, c, kw=kw: d.inv(ys[i % pairs], "dd137", 1, out=xs[i % pairs], config=lds_cfg, **kw), 1, 4)
        form("dd137 fwd f32 5 levels, LDS-plane kernel, fused (2 barriers)",
             lambda i, c: d.fwd(xs[i % pairs], "dd137", 5, out=ys[i % pairs], config=lds_cfg), 5, 4)
        del ws5
        for tdt, nm in [(torch.bfloat16, "bf16"), (torch.float16, "f16")]:
            xb = [t.to(tdt) for t in xs]
            yb = [torch.empty_like(t) for t in xb]
            form(f"cdf97 fwd {nm} 1 level", lambda i, c: d.fwd(xb[i % pairs], "cdf97", 1, out=yb[i % pairs], config=c),
                 1, 2, tune_key=("fwd", "cdf97", nm))
            form(f"cdf97 fwd {nm} 5 levels",
                 lambda i, c: d.fwd(xb[i % pairs], "cdf97", 5, out=yb[i % pairs], config=c), 5, 2,
                 tune_key=("fwd", "cdf97", nm))
            # 16-bit storage runs the fused steps in factored form by default
            # (8 instead of 11 operations per block and step: with half the
            # bytes per pixel the arithmetic bounds the kernel); the direct
            # evaluation of T_P, S_U for comparison
            form(f"cdf97 fwd {nm} 1 level, fused steps evaluated directly",
                 lambda i, c: d.fwd(xb[i % pairs], "cdf97", 1, out=yb[i % pairs], config=c, fused=True), 1, 2)
            form(f"cdf97 inv {nm} 1 level",
                 lambda i, c: d.inv(yb[i % pairs], "cdf97", 1, out=xb[i % pairs], config=c), 1, 2,
                 tune_key=("inv", "cdf97", nm))
            del xb, yb
        xi = [(t * 255).to(torch.int32) for t in xs]
        yi = [torch.empty_like(t) for t in xi]
        form("cdf53 fwd i32 1 level", lambda i, c: d.fwd(xi[i % pairs], "cdf53", 1, out=yi[i % pairs], config=c),
             1, 4, tune_key=("fwd", "cdf53", "i32"))
        form("cdf53 inv i32 1 level", lambda i, c: d.inv(yi[i % pairs], "cdf53", 1, out=xi[i % pairs], config=c),
             1, 4, tune_key=("inv", "cdf53", "i32"))
        form("cdf53 fwd i32 1 level separable (4 barriers)",
             lambda i, c: d.fwd(xi[i % pairs], "cdf53", 1, out=yi[i % pairs], config=c, separable=True), 1, 4)
        del xi, yi
        form("cdf97 fwd f32 1 level, warm (one buffer pair, repeated)",
             lambda i, c: d.fwd(xs[0], "cdf97", 1, out=ys[0], config=c), 1, 4)
        xg = torch.from_numpy(workloads.gradient_noise(N, N, seed=0)).to(dev)
        form("cdf97 fwd f32 1 level, gradient + noise input",
             lambda i, c: d.fwd(xg if i % 2 == 0 else xs[1], "cdf97", 1, out=ys[i % pairs], config=c), 1, 4)
        del xg
        del xs[1:], ys[1:]
        torch.cuda.empty_cache()

        def sized_form(name, n, levels, npairs, steps=40, graph_calls=0):
            """Forward CDF 9/7 FP32 on n x n images rotating over npairs
            input/output pairs (cold when they total >= 1 GiB; warm with one
            pair).  graph_calls > 0: also time one captured graph replaying
            that many calls (per-call time = replay time / graph_calls)."""
            if not want(name):
                return
            g = torch.Generator(device=dev).manual_seed(7)
            xn = [torch.rand((n, n), device=dev, generator=g) for _ in range(npairs)]
            yn = [torch.empty_like(t) for t in xn]
            def run(i):
                d.fwd(xn[i % npairs], "cdf97", levels, out=yn[i % npairs])
            _, ms = time_steps(torch, run, steps, 5)
            ab = algorithmic_bytes(n, n, levels, 4)
            entry = {"form": name, "Gpixel/s": round(n * n / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 5),
                     "GB/s": round(ab / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "buffer_pairs": npairs, "pairs_GiB": round(2 * npairs * n * n * 4 / 2 ** 30, 3)}
            if graph_calls:
                s2 = torch.cuda.Stream()
                s2.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(s2):
                    for i in range(graph_calls):
                        run(i)
                torch.cuda.current_stream().wait_stream(s2)
                torch.cuda.synchronize()
                gr = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gr, stream=s2):
                    for i in range(graph_calls):
                        run(i)
                _, gms = time_steps(torch, lambda i: gr.replay(), 20, 3)
                gms /= graph_calls
                entry.update({"graph_calls": graph_calls, "graph_ms_per_call": round(gms, 5),
                              "graph_Gpixel/s": round(n * n / (gms * 1e-3) / 1e9, 2)})
                del gr
            forms.append(entry)
            del xn, yn
            torch.cuda.empty_cache()

        sized_form("cdf97 fwd f32 1 level, 4096^2 cold", 4096, 1, 8)
        sized_form("cdf97 fwd f32 1 level, 4096^2 warm", 4096, 1, 1)
        sized_form("cdf97 fwd f32 5 levels, 4096^2 cold", 4096, 5, 8)
        sized_form("cdf97 fwd f32 1 level, 1024^2 cold, per call and under graph replay", 1024, 1, 64,
                   graph_calls=64)
        sized_form("cdf97 fwd f32 1 level, 16384^2", 16384, 1, 2, steps=20)
        sized_form("cdf97 fwd f32 5 levels, 16384^2", 16384, 5, 2, steps=20)

        # precision: 3 x 8192^2 planes (seed 3), 5-level forward + inverse per
        # step, FP32 / BF16 / FP16 storage.  The reconstruction is compared
        # on the GPU with the storage-rounded input and with the FP32
        # original (PSNR with peak 1.0); the coefficients are compared with
        # the FP64 oracle of the storage-rounded input by the CPU leg below
        # (probe crops of every plane), so the inputs and coefficients are
        # kept on the host until then.
        x3 = (torch.from_numpy(workloads.planes(3, N, N, seed=3)).to(dev)
              if any(want(f"cdf97 fwd+inv {nm} 5 levels, 3 x {N}^2 planes") for nm in ("f32", "bf16", "f16"))
              else None)
        for tdt, nm in [(torch.float32, "f32"), (torch.bfloat16, "bf16"), (torch.float16, "f16")]:
            if not want(f"cdf97 fwd+inv {nm} 5 levels, 3 x {N}^2 planes"):
                continue
            xq = x3.to(tdt)
            cq = torch.empty_like(xq)
            rq = torch.empty_like(xq)

            def fwd_inv(i, xq=xq, cq=cq, rq=rq):
                d.fwd(xq, "cdf97", 5, out=cq)
                d.inv(cq, "cdf97", 5, out=rq)
            _, ms = time_steps(torch, fwd_inv, 10, 2)
            el = 4 if tdt == torch.float32 else 2
            ab = 2 * 3 * algorithmic_bytes(N, N, 5, el)
            entry = {"form": f"cdf97 fwd+inv {nm} 5 levels, 3 x {N}^2 planes",
                     "Gpixel/s": round(3 * N * N / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
                     "GB/s": round(ab / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            fwd_inv(0)
            torch.cuda.synchronize()
            for tag, base in (("rounded_input", xq.float()), ("fp32_original", x3)):
                mse = ((rq.double() - base.double()) ** 2).mean().item()
                entry[f"psnr_db_vs_{tag}"] = round(10 * np.log10(1.0 / mse), 2) if mse > 0 else None
            precision_saved[entry["form"]] = ([xq[p].double().cpu().numpy() for p in range(3)],
                                              [cq[p].float().cpu().numpy() for p in range(3)], 5)
            forms.append(entry)
            del xq, cq, rq
            torch.cuda.empty_cache()
        del x3
        torch.cuda.empty_cache()

        # differentiation: 64 x 3 x 1024^2 FP32 (seed 4), 3-level forward via
        # the autograd function, loss = sum |details| + MSE(LL_3, target (seed
        # 5)), backward through the hand-written adjoint
        ag_name = "autograd: 64 x 3 x 1024^2 FP32, 3-level forward + loss + adjoint backward"
        xa = tgt = None
        if want(ag_name):
            xa = torch.from_numpy(workloads.planes(64 * 3, 1024, 1024, seed=4).reshape(64, 3, 1024, 1024)).to(dev)
            xa.requires_grad_(True)
            tgt = torch.from_numpy(workloads.planes(64 * 3, 128, 128, seed=5).reshape(64, 3, 128, 128)).to(dev)

        def train_step(i):
            y = d.dwt2(xa, 3)
            ll = y[..., :128, :128]
            loss = y.abs().sum() - ll.abs().sum() + ((ll - tgt) ** 2).mean()
            loss.backward()
            xa.grad = None
        if want(ag_name):
            _, ms = time_steps(torch, train_step, 10, 2)
            # the two transforms of the step alone (forward of the stack,
            # adjoint of a cotangent of the same shape), timed the same way;
            # the rest of the step is PyTorch's loss and its gradient
            xd = xa.detach()
            ya = torch.empty_like(xd)
            ga = torch.empty_like(xd)
            _, fms = time_steps(torch, lambda i: d.fwd(xd, "cdf97", 3, out=ya), 10, 2)
            _, ams = time_steps(torch, lambda i: d.adj(ya, 3, out=ga), 10, 2)
            ab1 = 64 * 3 * algorithmic_bytes(1024, 1024, 3, 4)
            forms.append({"form": ag_name,
                          "Gpixel/s": round(64 * 3 * 1024 * 1024 / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
                          "forward_ms": round(fms, 4), "forward_hbm_frac": round(ab1 / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "adjoint_ms": round(ams, 4), "adjoint_hbm_frac": round(ab1 / (ams * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "loss_and_other_ms": round(ms - fms - ams, 4)})
            del xd, ya, ga
        del xa, tgt
        torch.cuda.empty_cache()

        # batched: a planner launch plus one launch per level covering every
        # image (or, persistent, one launch for every level of every image):
        # 256 images with H, W uniform in [64, 4096] (even), 5 levels; 1024
        # images of 256^2
        def batched_form(name, shapes, seed, steps=5, persistent=False):
            if not want(name):
                return
            g = torch.Generator(device=dev).manual_seed(seed)
            imgs = [torch.rand(s, device=dev, generator=g) for s in shapes]
            call = d.BatchedForward(imgs, 5, persistent=persistent)
            _, ms = time_steps(torch, lambda i: call.run(), steps, 2)
            # the same call captured once in a graph and replayed
            s2 = torch.cuda.Stream()
            s2.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s2):
                call.run()
            torch.cuda.current_stream().wait_stream(s2)
            torch.cuda.synchronize()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=s2):
                call.run()
            _, gms = time_steps(torch, lambda i: gr.replay(), steps, 2)
            if persistent and call.status() != d.DWT2_OK:
                raise RuntimeError(f"{name}: a dependency wait of the persistent launch ran out of time")
            npx = sum(h * w for h, w in shapes)
            ab = sum(algorithmic_bytes(h, w, 5, 4) for h, w in shapes)
            forms.append({"form": name, "Gpixel/s": round(npx / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
                          "GB/s": round(ab / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "graph_Gpixel/s": round(npx / (gms * 1e-3) / 1e9, 2), "graph_ms": round(gms, 4),
                          "images": len(shapes), "pixels": npx})
            del imgs, call, gr
            torch.cuda.empty_cache()

        batched_form("cdf97 fwd f32 5 levels, batched: 256 uneven images 64..4096",
                     workloads.uneven_shapes(256, 64, 4096, seed=1), seed=1)
        batched_form("cdf97 fwd f32 5 levels, batched: 1024 images 256x256", [(256, 256)] * 1024, seed=2, steps=10)
        batched_form("cdf97 fwd f32 5 levels, batched, one persistent launch: 256 uneven images 64..4096",
                     workloads.uneven_shapes(256, 64, 4096, seed=1), seed=1, steps=3, persistent=True)
        batched_form("cdf97 fwd f32 5 levels, batched, one persistent launch: 1024 images 256x256",
                     [(256, 256)] * 1024, seed=2, steps=5, persistent=True)

        # the same 1024 equal-size images as one plane batch (one launch per
        # level)
        pb_name = "cdf97 fwd f32 5 levels, plane batch: 1024 images 256x256"
        if want(pb_name):
            xp = torch.rand((1024, 256, 256), device=dev, generator=torch.Generator(device=dev).manual_seed(2))
            yp = torch.empty_like(xp)
            _, ms = time_steps(torch, lambda i: d.fwd(xp, "cdf97", 5, out=yp), 10, 2)
            ab = 1024 * algorithmic_bytes(256, 256, 5, 4)
            forms.append({"form": pb_name,
                          "Gpixel/s": round(1024 * 256 * 256 / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
                          "GB/s": round(ab / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
            del xp, yp

    # the headline runs after the other forms, on a GPU that has been busy
    # for a while (steady clocks), with its own three rotating pairs
    while len(xs) < pairs:
        xs.append(xs[0].roll(len(xs), dims=1).contiguous())
    while len(ys) < pairs:
        ys.append(torch.empty_like(xs[0]))
    torch.cuda.synchronize()

    def fwd_step(i):
        d.fwd(xs[i % pairs], "cdf97", 1, out=ys[i % pairs])

    head_cfg = d.tuned_config("fwd", "cdf97", d.DWT2_F32, N, N, 1)
    if head_cfg is None:
        head_cfg = "default"
    total_ms, kern_ms = time_steps(torch, fwd_step, args.steps, args.warmup)
    ms_step = total_ms / args.steps
    value = px / (ms_step * 1e-3) / 1e9
    per = per_launch_sample(torch, fwd_step, 100)
    abytes = algorithmic_bytes(N, N, 1, 4)
    achieved = abytes / (kern_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": f"level_kernel<fwd, cdf97, f32>, kernel configuration {head_cfg}",
                "algorithmic_bytes_per_launch": abytes,
                "avg_launch_ms": round(kern_ms, 5),
                "per_launch_sample": {"launches": len(per), "median_ms": round(float(np.median(per)), 5),
                                      "p10_ms": round(float(np.percentile(per, 10)), 5),
                                      "p90_ms": round(float(np.percentile(per, 90)), 5),
                                      "note": "after the timed region, an event pair around each launch"}}

    # a plain device copy of one input to one output buffer (N*N*4 bytes read
    # and written) on the same rotating buffers: the box's streaming bandwidth
    _, cms = time_steps(torch, lambda i: ys[i % pairs].copy_(xs[i % pairs]), 50, 5)
    copy_ref = {"bytes_per_launch": 2 * N * N * 4, "avg_ms": round(cms, 5),
                "GB/s": round(2 * N * N * 4 / (cms * 1e-3) / 1e9, 1), "kernel": "torch copy_"}
    roofline["of_copy"] = round(achieved / copy_ref["GB/s"], 4)

    cpu = None if args.no_cpu else cpu_baseline(x_host, args.cpu_seconds)
    if cpu is not None:
        cpu["pool"] = pool
        # the CPU leg also checks the precision forms against the FP64 oracle
        errs = oracle_precision_errors(precision_saved)
        for f in forms:
            if f["form"] in errs:
                f.update(errs[f["form"]])
    precision_saved.clear()

    line = {
        "metric": "Gpixel/s 2-D CDF 9/7 fwd 8192^2 FP32 (+ % HBM roofline)",
        "value": round(value, 2),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"CDF 9/7 forward, 1 level, one {N}x{N} FP32 image, uniform [0,1) seed 0, "
                               "whole-point symmetric borders, non-separable lifting (4 barriers)",
                   "height": N, "width": N, "levels": 1, "rotating_buffers": pairs,
                   "kernel_config": head_cfg},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    line["copy_reference"] = copy_ref
    if tuned:
        line["autotune"] = tuned
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
