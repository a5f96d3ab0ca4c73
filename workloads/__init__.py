"""Seeded synthetic inputs for the 2-D DWT workloads.

This module only draws numbers: it holds no wavelet arithmetic and is shared
by the tests, the benchmark and the oracle-side checks alike.  The paper
measures throughput against image resolution on synthetic images (Section
"Evaluation"); the shapes below stand in for those resolution sweeps.

All generators use numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np


def uniform(h: int, w: int, seed: int = 0, dtype=np.float32) -> np.ndarray:
    """Pixels uniform in [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((h, w), dtype=np.float32).astype(dtype, copy=False)


def gradient_noise(h: int, w: int, seed: int = 0, sigma: float = 0.05) -> np.ndarray:
    """Smooth ramp 0.5 (i/(h-1) + j/(w-1)) plus Gaussian noise, FP32, unclipped."""
    rng = np.random.default_rng(seed)
    i = np.arange(h, dtype=np.float32)[:, None] / max(h - 1, 1)
    j = np.arange(w, dtype=np.float32)[None, :] / max(w - 1, 1)
    noise = rng.standard_normal((h, w), dtype=np.float32) * np.float32(sigma)
    return (np.float32(0.5) * (i + j) + noise).astype(np.float32)


def pixels_u8(h: int, w: int, seed: int = 0) -> np.ndarray:
    """Integer pixels uniform in {0, ..., 255}, stored as int32."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, (h, w), dtype=np.int32)


def integers(h: int, w: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, (h, w), dtype=np.int32)


def uneven_shapes(count: int = 256, lo: int = 64, hi: int = 4096, seed: int = 1):
    """Heights and widths each uniform in [lo, hi], rounded to even."""
    rng = np.random.default_rng(seed)
    hs = 2 * rng.integers(lo // 2, hi // 2 + 1, count)
    ws = 2 * rng.integers(lo // 2, hi // 2 + 1, count)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


def uneven_batch(count: int = 256, lo: int = 64, hi: int = 4096, seed: int = 1):
    """A list of FP32 images of uneven even sizes, pixels uniform in [0, 1)."""
    rng = np.random.default_rng(seed)
    shapes = uneven_shapes(count, lo, hi, seed)
    return [rng.random(s, dtype=np.float32) for s in shapes]


def planes(n: int, h: int, w: int, seed: int = 0) -> np.ndarray:
    """n independent FP32 planes uniform in [0, 1) (channels / batch)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, h, w), dtype=np.float32)
