"""The separable and factored schemes against the oracle.

DWT2_FLAG_SEPARABLE replaces every fused step by its horizontal and its
vertical separable lifting step (Section "Proposed Schemes": the scheme the
fused steps are compared with), one barrier each.  DWT2_FLAG_FACTORED keeps
the fused steps and their single barrier but evaluates each as those two
factors in registers.  Both compute the same transform, so the bars are
those of the fused kernels: CDF 9/7 with FP32 storage within 1e-5 of the
largest oracle coefficient, 16-bit storage within 8 unit roundoffs,
reversible CDF 5/3 bit-exact (and bit-identical to the fused kernels, whose
integer steps are defined by the same separable order).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import lifting, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

TOL97 = 1e-5
UNIT = {torch.bfloat16: 2.0 ** -9, torch.float16: 2.0 ** -12}


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
    return t.detach().to("cpu").to(torch.float64 if t.is_floating_point() else torch.int64).numpy()


def tile_configs():
    return [i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_TILE]


SCHEMES = ["separable", "factored"]

SMALL = [(2, 2), (2, 3), (3, 3), (5, 7), (9, 4), (17, 33), (64, 66), (130, 250), (255, 257), (300, 1000)]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", SMALL)
def test_scheme_small_shapes(shape, scheme):
    kw = {scheme: True}
    h, w = shape
    x = workloads.uniform(h, w, seed=h * 1000 + w + 5)
    xi = workloads.integers(h, w, -3000, 3000, seed=h + 7 * w + 5)
    m = lifting.max_levels(h, w)
    for lv in sorted({1, min(m, 4), m}):
        say(scheme, shape, "levels", lv)
        ref = lifting.fwd(x, "cdf97", lv)
        y = d.fwd(gpu(x), "cdf97", lv, **kw)
        assert rel_err(host(y), ref) <= TOL97
        c = ref.astype(np.float32)
        xr = d.inv(gpu(c), "cdf97", lv, **kw)
        assert rel_err(host(xr), lifting.inv(c, "cdf97", lv)) <= TOL97
        ref_i = lifting.fwd(xi, "cdf53", lv)
        yi = d.fwd(gpu(xi), "cdf53", lv, **kw)
        assert np.array_equal(host(yi), ref_i)
        assert np.array_equal(host(d.inv(yi, "cdf53", lv, **kw)), xi)


# interior tiles for every tile width plus ragged last tiles (see the fused
# kernels' configuration tests for how these shapes were chosen)
CFG_SHAPES = [(1100, 2104), (1034, 2062), (2, 3000), (3000, 6)]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", CFG_SHAPES)
def test_scheme_tile_configs(shape, scheme):
    kw = {scheme: True}
    h, w = shape
    x = workloads.uniform(h, w, seed=41)
    xi = workloads.pixels_u8(h, w, seed=42)
    lv = min(3, lifting.max_levels(h, w))
    ref = lifting.fwd(x, "cdf97", lv)
    ref_i = lifting.fwd(xi, "cdf53", lv)
    xg, xig = gpu(x), gpu(xi)
    for cfg in tile_configs():
        say(scheme, "tile config", cfg, shape, lv)
        y = d.fwd(xg, "cdf97", lv, config=cfg, **kw)
        assert rel_err(host(y), ref) <= TOL97, cfg
        assert rel_err(host(d.inv(y, "cdf97", lv, config=cfg, **kw)), x) <= TOL97, cfg
        yi = d.fwd(xig, "cdf53", lv, config=cfg, **kw)
        assert np.array_equal(host(yi), ref_i), cfg
        # the integer transform is defined by the separable order: the fused
        # kernels give the same integers
        assert torch.equal(yi, d.fwd(xig, "cdf53", lv, config=cfg)), cfg
        assert torch.equal(d.inv(yi, "cdf53", lv, config=cfg, **kw), xig), cfg


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
def test_scheme_storage_bound(tdt, scheme):
    kw = {scheme: True}
    h, w, lv = 1100, 2104, 2
    xs = torch.from_numpy(workloads.uniform(h, w, seed=43)).to(tdt)
    ref = lifting.fwd(xs.to(torch.float64).numpy(), "cdf97", lv)
    for cfg in tile_configs():
        say(scheme, "storage", tdt, cfg)
        y = d.fwd(xs.to(dev()), "cdf97", lv, config=cfg, **kw)
        assert rel_err(host(y), ref) <= 8 * UNIT[tdt], cfg


@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_plane_batch(scheme):
    kw = {scheme: True}
    n, h, w, lv = 3, 260, 2056, 2
    x = gpu(workloads.planes(n, h, w, seed=44))
    y = d.fwd(x, "cdf97", lv, **kw)
    r = d.inv(y, "cdf97", lv, **kw)
    for k in range(n):
        assert torch.equal(y[k], d.fwd(x[k], "cdf97", lv, **kw)), k
        assert torch.equal(r[k], d.inv(y[k], "cdf97", lv, **kw)), k
    assert rel_err(host(y[0]), lifting.fwd(host(x[0]), "cdf97", lv)) <= TOL97


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("lv", [1, 5])
def test_scheme_full_size_crops(lv, scheme):
    """8192^2 (the benchmark image) on crops the oracle evaluates exactly."""
    kw = {scheme: True}
    n = 8192
    x = workloads.uniform(n, n, seed=0)
    say(scheme, "full size", n, lv)
    y = d.fwd(gpu(x), "cdf97", lv, **kw)
    yh = host(y)
    scale = float(np.abs(yh).max())
    m = window.default_margin(lv)
    worst = 0.0
    for r0, r1, c0, c1 in window.probe_crops(n, n, lv, size=256):
        sub = lifting.fwd(x[r0:r1, c0:c1], "cdf97", lv)
        cut = window.crop_pyramid(yh, lv, r0, r1, c0, c1)
        mask = window.crop_valid_mask(n, n, lv, r0, r1, c0, c1, m)
        worst = max(worst, float(np.abs(cut[mask] - sub[mask]).max()))
    assert worst / scale <= TOL97
    xr = host(d.inv(y, "cdf97", lv, **kw))
    assert np.abs(xr - x).max() <= 1e-4
