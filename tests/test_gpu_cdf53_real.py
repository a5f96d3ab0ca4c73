"""The real-valued CDF 5/3 ("cdf53f", DWT2_CDF53) against the oracle.

The paper evaluates CDF 5/3 beside CDF 9/7 (Section "Evaluation"); the
library computes it with the same kernels (one fused predict and one fused
update per scale, 2 barriers).  Bars as for CDF 9/7: FP32 storage within
1e-5 of the largest oracle coefficient per image, 16-bit storage within 8
unit roundoffs; every kernel configuration and scheme is checked.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import lifting, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

TOL = 1e-5
UNIT = {torch.bfloat16: 2.0 ** -9, torch.float16: 2.0 ** -12}
WAV = "cdf53f"
SCHEMES = [{}, {"split": True}, {"separable": True}, {"factored": True}]


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def host(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


SMALL = [(2, 2), (2, 3), (3, 2), (3, 3), (5, 7), (8, 8), (9, 4), (17, 33), (64, 66), (130, 250),
         (255, 257), (300, 1000), (512, 512)]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("kw", SCHEMES, ids=["fused", "split", "separable", "factored"])
def test_small_shapes(shape, kw):
    h, w = shape
    x = workloads.uniform(h, w, seed=h * 1000 + w + 9)
    m = lifting.max_levels(h, w)
    for lv in sorted({1, min(m, 5), m}):
        say(WAV, shape, "levels", lv, kw)
        ref = lifting.fwd(x, WAV, lv)
        y = d.fwd(gpu(x), WAV, lv, **kw)
        assert rel_err(host(y), ref) <= TOL
        c = ref.astype(np.float32)
        xr = d.inv(gpu(c), WAV, lv, **kw)
        assert rel_err(host(xr), lifting.inv(c, WAV, lv)) <= TOL


CFG_SHAPES = [(1100, 2104), (1034, 2062), (2, 3000), (3000, 6)]


@pytest.mark.parametrize("shape", CFG_SHAPES)
def test_every_config_and_scheme(shape):
    h, w = shape
    x = workloads.uniform(h, w, seed=51)
    lv = min(3, lifting.max_levels(h, w))
    ref = lifting.fwd(x, WAV, lv)
    xg = gpu(x)
    for cfg in range(d.DWT2_NUM_KERNEL_CONFIGS):
        for kw in SCHEMES:
            scheme = next((k for k in ("split", "separable", "factored") if kw.get(k)), "fused")
            if not d.config_supports(cfg, "fwd", WAV, scheme):
                continue
            say(WAV, "config", cfg, shape, lv, kw)
            y = d.fwd(xg, WAV, lv, config=cfg, **kw)
            assert rel_err(host(y), ref) <= TOL, (cfg, kw)
            assert rel_err(host(d.inv(y, WAV, lv, config=cfg, **kw)), x) <= TOL, (cfg, kw)


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
def test_storage_bound(tdt):
    h, w, lv = 1100, 2104, 3
    xs = torch.from_numpy(workloads.uniform(h, w, seed=52)).to(tdt)
    ref = lifting.fwd(xs.to(torch.float64).numpy(), WAV, lv)
    for cfg in range(d.DWT2_NUM_KERNEL_CONFIGS):
        say(WAV, "storage", tdt, cfg)
        y = d.fwd(xs.to(dev()), WAV, lv, config=cfg)
        assert rel_err(host(y), ref) <= 8 * UNIT[tdt], cfg


def test_plane_batch():
    n, h, w, lv = 3, 260, 2056, 2
    x = gpu(workloads.planes(n, h, w, seed=53))
    y = d.fwd(x, WAV, lv)
    for k in range(n):
        assert torch.equal(y[k], d.fwd(x[k], WAV, lv)), k
    assert rel_err(host(y[1]), lifting.fwd(host(x[1]), WAV, lv)) <= TOL


@pytest.mark.parametrize("lv", [1, 5])
def test_full_size_crops(lv):
    """8192^2 on crops the oracle evaluates exactly; the inverse restores it."""
    n = 8192
    x = workloads.uniform(n, n, seed=0)
    say(WAV, "full size", n, lv)
    y = d.fwd(gpu(x), WAV, lv)
    yh = host(y)
    scale = float(np.abs(yh).max())
    m = window.default_margin(lv)
    worst = 0.0
    for r0, r1, c0, c1 in window.probe_crops(n, n, lv, size=256):
        sub = lifting.fwd(x[r0:r1, c0:c1], WAV, lv)
        cut = window.crop_pyramid(yh, lv, r0, r1, c0, c1)
        mask = window.crop_valid_mask(n, n, lv, r0, r1, c0, c1, m)
        worst = max(worst, float(np.abs(cut[mask] - sub[mask]).max()))
    assert worst / scale <= TOL
    xr = host(d.inv(y, WAV, lv))
    assert np.abs(xr - x).max() <= 1e-4
