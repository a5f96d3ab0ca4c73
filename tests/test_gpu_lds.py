"""GPU parity of the LDS-plane kernel (kernel configurations of algorithm
DWT2_ALGO_LDS) through the C ABI.

* DD 13/7 (four-tap steps, Section "Evaluation"), fused and separable
  lifting, forward and inverse, against the oracle's DD 13/7 lifting;
* the non-separable polyconvolution N_{P,U} for CDF 9/7 (one step per
  lifting pair, Section "Proposed Schemes"), forward and inverse, against
  the oracle (the separable definition and the oracle's own polyconvolution);
* the fused and separable CDF schemes on the LDS-plane kernel, bit-identical
  to the register tile kernel (the same block formulas).

Shapes span several tiles of both LDS configurations with ragged last tiles,
odd sides and tiny images; bars as elsewhere: FP32 within 1e-5 of the
largest coefficient, 16-bit storage within 8 unit roundoffs against the
oracle of the storage-rounded input.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import lifting, nonsep, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

TOL = 1e-5
UNIT = {torch.bfloat16: 2.0 ** -9, torch.float16: 2.0 ** -12}
SHAPES = [(2, 2), (3, 5), (7, 9), (17, 33), (64, 66), (130, 250), (255, 257), (300, 1000), (517, 1283)]


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


def lds_configs():
    return [i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_LDS]


def levels_for(h, w):
    m = lifting.max_levels(h, w)
    return sorted({1, min(m, 3), m})


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("separable", [False, True])
def test_dd137_against_oracle(shape, separable):
    h, w = shape
    x = workloads.uniform(h, w, seed=h * 997 + w)
    for cfg in lds_configs():
        for lv in levels_for(h, w):
            say("dd137", shape, "config", cfg, "levels", lv, "separable", separable)
            ref = lifting.fwd(x, "dd137", lv)
            y = d.fwd(gpu(x), "dd137", lv, config=cfg, separable=separable)
            assert rel_err(host(y), ref) <= TOL, (cfg, lv)
            c = ref.astype(np.float32)
            xr = d.inv(gpu(c), "dd137", lv, config=cfg, separable=separable)
            assert rel_err(host(xr), lifting.inv(c, "dd137", lv)) <= TOL, (cfg, lv)


@pytest.mark.parametrize("shape", SHAPES)
def test_polyconv_against_oracle(shape):
    h, w = shape
    x = workloads.uniform(h, w, seed=h * 991 + w)
    for cfg in lds_configs():
        for lv in levels_for(h, w):
            say("polyconv cdf97", shape, "config", cfg, "levels", lv)
            ref = lifting.fwd(x, "cdf97", lv)
            y = host(d.fwd(gpu(x), "cdf97", lv, config=cfg, polyconv=True))
            assert rel_err(y, ref) <= TOL, (cfg, lv)
            assert rel_err(y, nonsep.polyconv_fwd(x, "cdf97", lv)) <= TOL, (cfg, lv)
            c = ref.astype(np.float32)
            xr = host(d.inv(gpu(c), "cdf97", lv, config=cfg, polyconv=True))
            assert rel_err(xr, lifting.inv(c, "cdf97", lv)) <= TOL, (cfg, lv)
            assert rel_err(xr, nonsep.polyconv_inv(c, "cdf97", lv)) <= TOL, (cfg, lv)


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("wav,kw", [("dd137", {}), ("cdf97", {"polyconv": True})])
def test_storage_bound(tdt, wav, kw):
    h, w, lv = 300, 1000, 3
    xs = torch.from_numpy(workloads.uniform(h, w, seed=13)).to(tdt)
    ref = lifting.fwd(xs.to(torch.float64).numpy(), wav, lv)
    for cfg in lds_configs():
        say("storage", tdt, wav, kw, cfg)
        y = host(d.fwd(xs.to(dev()), wav, lv, config=cfg, **kw))
        assert rel_err(y, ref) <= 8 * UNIT[tdt], cfg


@pytest.mark.parametrize("wav", ["cdf97", "cdf53f"])
@pytest.mark.parametrize("shape,lv", [((517, 1283), 3), ((600, 2056), 2), ((2, 3000), 1), ((3000, 6), 2),
                                      ((1034, 2062), 3)])
def test_cdf_schemes_bit_identical_to_register_kernel(wav, shape, lv):
    """The LDS-plane kernel evaluates the CDF fused and separable steps with
    the register tile kernel's block formulas: bit for bit the same
    coefficients and images, FP32 and BF16."""
    h, w = shape
    xf = gpu(workloads.uniform(h, w, seed=71))
    for x in (xf, xf.to(torch.bfloat16)):
        for sep in (False, True):
            # the register kernel's direct fused evaluation (16-bit storage
            # defaults to the factored one there)
            ref = d.fwd(x, wav, lv, config=0, separable=sep, fused=not sep)
            back = d.inv(ref, wav, lv, config=0, separable=sep, fused=not sep)
            for cfg in lds_configs():
                say("bit-identical", wav, shape, lv, x.dtype, "separable", sep, "config", cfg)
                assert torch.equal(d.fwd(x, wav, lv, config=cfg, separable=sep), ref), cfg
                assert torch.equal(d.inv(ref, wav, lv, config=cfg, separable=sep), back), cfg


def test_plane_batch_dd137_and_polyconv():
    n, h, w, lv = 3, 260, 2056, 3
    x = gpu(workloads.planes(n, h, w, seed=72))
    for cfg in lds_configs():
        for wav, kw in (("dd137", {}), ("cdf97", {"polyconv": True})):
            say("plane batch", wav, kw, cfg)
            y = d.fwd(x, wav, lv, config=cfg, **kw)
            r = d.inv(y, wav, lv, config=cfg, **kw)
            for k in range(n):
                assert torch.equal(y[k], d.fwd(x[k], wav, lv, config=cfg, **kw)), (wav, cfg, k)
                assert torch.equal(r[k], d.inv(y[k], wav, lv, config=cfg, **kw)), (wav, cfg, k)
            assert rel_err(host(y[2]), lifting.fwd(host(x[2]), wav, lv)) <= TOL


def test_default_configuration():
    """Without a named configuration DD 13/7 and the polyconvolution run on
    the LDS-plane kernel (the only one that has them)."""
    x = gpu(workloads.uniform(200, 301, seed=73))
    assert torch.equal(d.fwd(x, "dd137", 2), d.fwd(x, "dd137", 2, config=lds_configs()[0]))
    assert torch.equal(d.fwd(x, "cdf97", 2, polyconv=True), d.fwd(x, "cdf97", 2, config=lds_configs()[0],
                                                                     polyconv=True))


@pytest.mark.parametrize("wav,kw", [("dd137", {}), ("cdf97", {"polyconv": True})])
@pytest.mark.parametrize("lv", [1, 5])
def test_full_size_crops(wav, kw, lv):
    """8192^2 on probe crops the oracle evaluates exactly; the inverse
    restores the image."""
    n = 8192
    x = workloads.uniform(n, n, seed=0)
    say("full size", wav, kw, lv)
    xg = gpu(x)
    y = d.fwd(xg, wav, lv, **kw)
    yh = y.cpu().numpy()
    scale = float(np.abs(yh).max())
    # the crop margin (16 * 2^lv + 16 pixels) also covers DD 13/7, whose
    # footprint grows by 6 * 2^l pixels per scale (13-tap low-pass)
    m = window.default_margin(lv)
    worst = 0.0
    for r0, r1, c0, c1 in window.probe_crops(n, n, lv, size=256):
        sub = lifting.fwd(x[r0:r1, c0:c1], wav, lv)
        cut = window.crop_pyramid(yh, lv, r0, r1, c0, c1)
        mask = window.crop_valid_mask(n, n, lv, r0, r1, c0, c1, m)
        worst = max(worst, float(np.abs(cut[mask].astype(np.float64) - sub[mask]).max()))
    assert worst / scale <= TOL
    assert float((d.inv(y, wav, lv, **kw) - xg).abs().max()) <= 1e-4
