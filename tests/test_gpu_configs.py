"""GPU parity at the sizes of the benchmark workloads (through the C ABI).

Each test takes one workload at its full size and checks the HIP result
against the CPU oracle: exactly where the oracle can run on the whole input,
and otherwise on crops the oracle evaluates exactly (corners, edge midpoints
and the centre, see oracle/window.py), plus properties that hold at any size
(perfect reconstruction, bit-identity between call forms).  Bars as in
test_gpu_parity.py: reversible CDF 5/3 bit-exact; FP32 CDF 9/7 within 1e-5 of
the largest coefficient; 16-bit storage within 8 unit roundoffs of the
largest coefficient against the oracle run on the storage-rounded input.

Workloads: single images of 1024^2 ... 16384^2 (uniform [0, 1), the smooth
ramp plus Gaussian noise, integer pixels in [0, 255]); the 256-image batch of
uneven even sizes in [64, 4096]; three 8192^2 planes stored as BF16 / FP16.
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


def crop_errors(x, y, wavelet, lv):
    """Largest |gpu - oracle| over the valid part of every probe crop (FP64);
    for the integer wavelet, asserts bit-exactness instead and returns 0.
    x: the image (host), y: the GPU pyramid (host, any float or int dtype)."""
    H, W = x.shape
    m = window.default_margin(lv)
    worst = 0.0
    for r0, r1, c0, c1 in window.probe_crops(H, W, lv, size=256):
        sub = lifting.fwd(x[r0:r1, c0:c1], wavelet, lv)
        cut = window.crop_pyramid(y, lv, r0, r1, c0, c1)
        mask = window.crop_valid_mask(H, W, lv, r0, r1, c0, c1, m)
        assert mask.sum() > 0
        if wavelet == "cdf53":
            assert np.array_equal(cut[mask].astype(np.int64), sub[mask]), (r0, c0)
        else:
            worst = max(worst, float(np.abs(cut[mask].astype(np.float64) - sub[mask]).max()))
    return worst


# ---- 16384^2 (1 GiB per FP32 array) -----------------------------------------

@pytest.mark.parametrize("lv", [1, 5])
def test_cdf97_16384_crops_and_reconstruction(lv):
    n = 16384
    x = workloads.uniform(n, n, seed=0)
    say("cdf97 16384^2 levels", lv)
    xg = torch.from_numpy(x).to(dev())
    y = d.fwd(xg, "cdf97", lv)
    yh = y.cpu().numpy()
    scale = float(np.abs(yh).max())
    worst = crop_errors(x, yh, "cdf97", lv)
    say("  crop max-abs", worst, "largest coefficient", scale)
    assert worst / scale <= TOL97
    del yh
    # the whole-image inverse restores the image (a property at any size)
    xr = d.inv(y, "cdf97", lv)
    err = float((xr - xg).abs().max())
    say("  reconstruction max-abs", err)
    assert err <= 1e-4


@pytest.mark.parametrize("lv", [1, 5])
def test_cdf53_16384_crops_bit_exact(lv):
    n = 16384
    x = workloads.pixels_u8(n, n, seed=0)
    say("cdf53 16384^2 levels", lv)
    xg = torch.from_numpy(x).to(dev())
    y = d.fwd(xg, "cdf53", lv)
    crop_errors(x, y.cpu().numpy(), "cdf53", lv)
    assert torch.equal(d.inv(y, "cdf53", lv), xg)


@pytest.mark.parametrize("n", [1024, 4096])
@pytest.mark.parametrize("lv", [1, 5])
def test_cdf53_whole_image_bit_exact(n, lv):
    """Reversible 5/3 of the whole image against the whole-image oracle."""
    x = workloads.pixels_u8(n, n, seed=0)
    say("cdf53 whole", n, "levels", lv)
    y = d.fwd(torch.from_numpy(x).to(dev()), "cdf53", lv)
    ref = lifting.fwd(x, "cdf53", lv)
    assert np.array_equal(y.cpu().numpy().astype(np.int64), ref)
    xr = d.inv(torch.from_numpy(ref.astype(np.int32)).to(dev()), "cdf53", lv)
    assert np.array_equal(xr.cpu().numpy(), x)


# ---- the smooth ramp + Gaussian noise input ---------------------------------

@pytest.mark.parametrize("lv", [1, 5])
def test_gradient_noise_4096_whole_image(lv):
    n = 4096
    x = workloads.gradient_noise(n, n, seed=0)
    say("gradient+noise whole", n, "levels", lv)
    y = d.fwd(torch.from_numpy(x).to(dev()), "cdf97", lv).cpu().numpy().astype(np.float64)
    ref = lifting.fwd(x, "cdf97", lv)
    err = float(np.abs(y - ref).max() / np.abs(ref).max())
    say("  relative max-abs", err)
    assert err <= TOL97


@pytest.mark.parametrize("lv", [1, 5])
def test_gradient_noise_8192_crops(lv):
    n = 8192
    x = workloads.gradient_noise(n, n, seed=0)
    say("gradient+noise crops", n, "levels", lv)
    xg = torch.from_numpy(x).to(dev())
    y = d.fwd(xg, "cdf97", lv)
    yh = y.cpu().numpy()
    scale = float(np.abs(yh).max())
    worst = crop_errors(x, yh, "cdf97", lv)
    say("  crop max-abs", worst, "largest coefficient", scale)
    assert worst / scale <= TOL97
    assert float((d.inv(y, "cdf97", lv) - xg).abs().max()) <= 1e-4


# ---- the 256-image batch of uneven sizes ------------------------------------

def test_batched_uneven_256_images():
    """The whole 256-image batch (heights and widths uniform in [64, 4096],
    even; 1.17 Gpixel), 5 levels in one batched call: every image equals the
    single-image transform bit for bit, and 8 images -- the smallest, the
    largest and six spread over the list -- equal the oracle (whole image up
    to 1024^2 pixels, probe crops beyond)."""
    shapes = workloads.uneven_shapes(256, 64, 4096, seed=1)
    g = torch.Generator(device=dev()).manual_seed(1)
    xs = [torch.rand(s, device=dev(), generator=g) for s in shapes]
    say("batched 256 uneven images", sum(h * w for h, w in shapes), "pixels")
    outs = d.fwd_batched(xs, levels=5)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(xs, outs)):
        assert torch.equal(y, d.fwd(x, "cdf97", 5)), (k, shapes[k])
    area = np.array([h * w for h, w in shapes])
    order = np.argsort(area)
    picks = sorted({int(order[0]), int(order[-1])} | {int(k) for k in np.linspace(1, 254, 6).astype(int)})
    assert len(picks) == 8
    for k in picks:
        x = xs[k].cpu().numpy()
        y = outs[k].cpu().numpy()
        say("  oracle on image", k, shapes[k])
        if x.size <= 1024 * 1024:
            ref = lifting.fwd(x, "cdf97", 5)
            assert np.abs(y - ref).max() / np.abs(ref).max() <= TOL97, (k, shapes[k])
        else:
            assert crop_errors(x, y, "cdf97", 5) / float(np.abs(y).max()) <= TOL97, (k, shapes[k])


# ---- 3 x 8192^2 planes stored as BF16 / FP16 --------------------------------

@pytest.mark.parametrize("tdt,min_psnr", [(torch.bfloat16, 48.0), (torch.float16, 64.0)])
def test_precision_3x8192_planes(tdt, min_psnr):
    """5-level forward + inverse of three 8192^2 planes stored as BF16 / FP16
    (FP32 arithmetic): coefficient max-abs against the FP64 oracle of the
    storage-rounded input on probe crops of every plane, and reconstruction
    PSNR (peak 1.0) against that input over the whole stack."""
    n, lv = 8192, 5
    x3 = workloads.planes(3, n, n, seed=3)
    xq = torch.from_numpy(x3).to(dev()).to(tdt)          # storage-rounded input
    say("precision 3 x 8192^2", tdt)
    c = d.fwd(xq, "cdf97", lv)
    r = d.inv(c, "cdf97", lv)
    mse = float(((r.double() - xq.double()) ** 2).mean())
    psnr = 10 * np.log10(1.0 / mse)
    worst, scale = 0.0, 0.0
    for p in range(3):
        xp = xq[p].double().cpu().numpy()
        cp = c[p].float().cpu().numpy()
        scale = max(scale, float(np.abs(cp).max()))
        worst = max(worst, crop_errors(xp, cp, "cdf97", lv))
    say("  coefficient max-abs", worst, "largest coefficient", scale, "PSNR dB", psnr)
    assert worst <= 8 * UNIT[tdt] * scale
    assert psnr >= min_psnr
