"""Autotuner for the kernel configuration (tile shape / algorithm).

Times every kernel configuration that the library offers for a case
(direction, wavelet, storage type, image size class, level count) on the
current GPU and records the fastest in a JSON cache.  The binding consults
the cache when a call does not name a configuration; all configurations
compute bit-identical results, so the choice affects speed only.

    python -m paper_1704_08657_amd.autotune [--out FILE] [--quick]

The cache key is "arch|direction|wavelet|dtype|size-class|levels"; the size
class is the image side rounded up to a power of two (64 ... 16384).
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_PATH = os.path.join(HERE, "tuned_configs.json")


def size_class(h: int, w: int) -> int:
    s = 64
    while s < max(h, w) and s < 16384:
        s *= 2
    return s


def key(arch: str, direction: str, wavelet: str, dtype: str, h: int, w: int, levels: int) -> str:
    return f"{arch}|{direction}|{wavelet}|{dtype}|{size_class(h, w)}|{levels}"


_arch = None


def arch_name() -> str:
    """The GPU's architecture name (queried once per process)."""
    global _arch
    if _arch is None:
        import torch
        p = torch.cuda.get_device_properties(0)
        _arch = getattr(p, "gcnArchName", p.name).split(":")[0]
    return _arch


_cache = None


def load_cache(path: str = CACHE_PATH) -> dict:
    global _cache
    if _cache is None:
        try:
            with open(path) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def lookup(direction: str, wavelet: str, dtype: str, h: int, w: int, levels: int):
    """Tuned configuration index for a case, or None."""
    cache = load_cache()
    if not cache:
        return None
    try:
        arch = arch_name()
    except Exception:
        return None
    return cache.get(key(arch, direction, wavelet, dtype, h, w, levels))


def tune_case(direction: str, wavelet: str, dtype: str, h: int, w: int, levels: int, run, configs=None,
              steps: int = 8, warm: int = 3):
    """Time `run(config, i)` for every kernel configuration (or `configs`) on
    the current GPU and stream, record the fastest (median of `steps`
    launches) in the in-memory cache under this case's key, so calls that
    name no configuration use it, and return (best, {config: ms})."""
    import torch
    import paper_1704_08657_amd as d
    if configs is None:
        configs = [c for c in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.config_supports(c, direction, wavelet)]
    times = {c: _time(torch, lambda i, c=c: run(c, i), steps=steps, warm=warm) for c in configs}
    best = min(times, key=times.get)
    cache = load_cache()
    global _cache
    _cache = dict(cache)
    _cache[key(arch_name(), direction, wavelet, dtype, h, w, levels)] = best
    from . import _tuned               # the binding's memo of cache lookups
    _tuned.clear()
    return best, times


def _time(torch, fn, steps=20, warm=4):
    """Average ms per call of `steps` back-to-back calls, from one event pair
    around them (an event pair per call would add its own cost to each)."""
    stream = torch.cuda.current_stream()
    for i in range(warm):
        fn(i)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for i in range(steps):
        fn(i)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune(sizes=(256, 1024, 4096, 8192), levels=(1, 5), quick=False, out=CACHE_PATH, log=print,
         dtypes=("f32", "bf16", "f16", "i32")):
    import torch
    import paper_1704_08657_amd as d

    dev = torch.device("cuda", 0)
    arch = arch_name()
    result = dict(load_cache(out)) if os.path.exists(out) else {}
    dts = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16, "i32": torch.int32}
    cases = []
    for n in sizes:
        for lv in levels:
            for dt in (("f32", "bf16") if quick else ("f32", "bf16", "f16")):
                if dt not in dtypes:
                    continue
                cases += [("fwd", "cdf97", dt, n, lv), ("inv", "cdf97", dt, n, lv)]
                if dt == "f32":
                    cases.append(("adj", "cdf97", dt, n, lv))
            if "i32" in dtypes:
                cases += [("fwd", "cdf53", "i32", n, lv), ("inv", "cdf53", "i32", n, lv)]
    nconf = d.DWT2_NUM_KERNEL_CONFIGS
    for direction, wav, dt, n, lv in cases:
        g = torch.Generator(device=dev).manual_seed(0)
        # three buffer pairs, so large images are timed from HBM, not the
        # last-level cache, as in repeated use
        nb = 3
        if dt == "i32":
            xs = [torch.randint(0, 256, (n, n), device=dev, dtype=torch.int32, generator=g) for _ in range(nb)]
        else:
            xs = [torch.rand((n, n), device=dev, generator=g).to(dts[dt]) for _ in range(nb)]
        ys = [torch.empty_like(x) for x in xs]
        fn = {"fwd": lambda x, y, c: d.fwd(x, wav, lv, out=y, config=c),
              "inv": lambda x, y, c: d.inv(x, wav, lv, out=y, config=c),
              "adj": lambda x, y, c: d.adj(x, lv, out=y, config=c)}[direction]
        best, best_ms = None, float("inf")
        for c in range(nconf):
            # the LDS-plane configurations run what the register tile kernel
            # does not (and are never faster where both run)
            if not d.config_supports(c, direction, wav) or d.dwt2_kernel_config(c)[1] == d.DWT2_ALGO_LDS:
                continue
            ms = _time(torch, lambda i: fn(xs[i % nb], ys[i % nb], c), steps=8 if quick else 30)
            if ms < best_ms:
                best, best_ms = c, ms
        k = key(arch, direction, wav, dt, n, n, lv)
        result[k] = best
        log(f"{k}: config {best} ({best_ms * 1e3:.1f} us)")
    # batched: between the configurations the batched kernels support
    for dt in [t for t in ("f32", "bf16") if t in dtypes]:
        shapes = [(int(h), int(w)) for h, w in zip(*[iter(
            torch.randint(32, 2049, (64,), generator=torch.Generator().manual_seed(1)).mul(2).tolist())] * 2)]
        imgs = [torch.rand(s, device=dev).to(dts[dt]) for s in shapes]
        best, best_ms = None, float("inf")
        for c in [i for i in range(nconf) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_TILE]:
            call = d.BatchedForward(imgs, 5, config=c)
            ms = _time(torch, lambda i: call.run(), steps=5 if quick else 10, warm=2)
            if ms < best_ms:
                best, best_ms = c, ms
        k = f"{arch}|batched|cdf97|{dt}|any|5"
        result[k] = best
        log(f"{k}: config {best} ({best_ms * 1e3:.1f} us)")
    with open(out, "w") as f:
        json.dump(result, f, indent=1, sort_keys=True)
    global _cache
    _cache = result
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE_PATH)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--sizes", default="256,1024,4096,8192")
    ap.add_argument("--dtypes", default="f32,bf16,f16,i32", help="storage types to tune (the others keep their entries)")
    a = ap.parse_args()
    t0 = time.time()
    tune(sizes=tuple(int(s) for s in a.sizes.split(",")), quick=a.quick, out=a.out,
         log=lambda s: print(s, flush=True), dtypes=tuple(a.dtypes.split(",")))
    print(f"tuned in {time.time() - t0:.1f} s -> {a.out}", flush=True)


if __name__ == "__main__":
    main()
