"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle.

Bars: reversible CDF 5/3 bit-exact; CDF 9/7 with FP32 storage within
max|gpu - oracle| / max|oracle| <= 1e-5 per image (all levels); BF16 / FP16
storage within the rounding bound derived in test_storage_bound below.
Inputs are seeded synthetic images (workloads).  Large images are checked on
crops (corners, edge midpoints, centre) that the oracle evaluates exactly.
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads
from oracle import adjoint, lifting, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

TOL97 = 1e-5


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


def gpu(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x)).to(dev())
    return t if dtype is None else t.to(dtype)


def host(t):
    return t.detach().to("cpu").to(torch.float64 if t.is_floating_point() else torch.int64).numpy()


SMALL = [(2, 2), (2, 3), (3, 2), (3, 3), (5, 7), (8, 8), (9, 4), (17, 33), (64, 66),
         (130, 250), (255, 257), (300, 1000), (512, 512)]


def levels_for(h, w):
    m = lifting.max_levels(h, w)
    return sorted({1, min(m, 5), m})


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("split", [False, True])
def test_fwd_inv_cdf97_f32(shape, split):
    h, w = shape
    x = workloads.uniform(h, w, seed=h * 1000 + w)
    for lv in levels_for(h, w):
        say("cdf97 f32", shape, "levels", lv, "split", split)
        ref = lifting.fwd(x, "cdf97", lv)
        y = d.fwd(gpu(x), "cdf97", lv, split=split)
        torch.cuda.synchronize()
        assert rel_err(host(y), ref) <= TOL97
        # inverse of the oracle's coefficients (as FP32)
        c = ref.astype(np.float32)
        xr = d.inv(gpu(c), "cdf97", lv, split=split)
        torch.cuda.synchronize()
        assert rel_err(host(xr), lifting.inv(c, "cdf97", lv)) <= TOL97


@pytest.mark.parametrize("shape", SMALL + [(31, 2), (2, 77), (1023, 1025)])
def test_cdf53_bit_exact(shape):
    h, w = shape
    for lo, hi in [(0, 256), (-3000, 3000)]:
        x = workloads.integers(h, w, lo, hi, seed=h + 7 * w)
        for lv in levels_for(h, w):
            say("cdf53", shape, "levels", lv, "range", lo, hi)
            ref = lifting.fwd(x, "cdf53", lv)
            y = host(d.fwd(gpu(x), "cdf53", lv))
            assert np.array_equal(y, ref)
            xr = host(d.inv(gpu(ref.astype(np.int32)), "cdf53", lv))
            assert np.array_equal(xr, x)


@pytest.mark.parametrize("shape", SMALL)
def test_adjoint_cdf97_f32(shape):
    h, w = shape
    g = workloads.uniform(h, w, seed=3 * h + w) - np.float32(0.5)
    for lv in levels_for(h, w):
        say("adj", shape, "levels", lv)
        ref = adjoint.adj(g, "cdf97", lv)
        got = host(d.adj(gpu(g), lv))
        assert rel_err(got, ref) <= TOL97


def test_adjoint_dot_product_on_gpu():
    h, w, lv = 96, 130, 3
    x = workloads.uniform(h, w, seed=1) - np.float32(0.5)
    y = workloads.uniform(h, w, seed=2) - np.float32(0.5)
    wx = host(d.fwd(gpu(x), "cdf97", lv))
    wty = host(d.adj(gpu(y), lv))
    lhs = float(np.vdot(wx, y))
    rhs = float(np.vdot(x, wty))
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1.0)


# BF16 keeps 8 significant bits (unit roundoff 2^-9), FP16 11 (2^-12).  Every
# stored coefficient carries one rounding relative to its own magnitude, and
# the LL of each level is rounded before the next level reads it; the next
# level's filters (DC gain 2 per level in 2-D, l1 norm of the 2-D low-pass
# ~ 2.6) amplify that input error.  A bound of 8 unit roundoffs of the largest
# coefficient covers one level plus the propagated LL rounding of up to five
# levels with margin; it is a factor ~30 below a dropped term's error.
UNIT = {torch.bfloat16: 2.0 ** -9, torch.float16: 2.0 ** -12}


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("shape,lv", [((512, 512), 1), ((512, 512), 5), ((300, 1000), 3), ((17, 33), 2)])
def test_storage_bound(tdt, shape, lv):
    h, w = shape
    x32 = workloads.uniform(h, w, seed=11)
    xs = torch.from_numpy(x32).to(tdt)                  # storage-rounded input
    xs64 = xs.to(torch.float64).numpy()
    say("storage", tdt, shape, lv)
    ref = lifting.fwd(xs64, "cdf97", lv)
    y = host(d.fwd(xs.to(dev()), "cdf97", lv))
    assert rel_err(y, ref) <= 8 * UNIT[tdt]
    # inverse of the oracle's (storage-rounded) coefficients
    cs = torch.from_numpy(ref).to(tdt)
    xr = host(d.inv(cs.to(dev()), "cdf97", lv))
    assert rel_err(xr, lifting.inv(cs.to(torch.float64).numpy(), "cdf97", lv)) <= 8 * UNIT[tdt]


def test_pitched_buffers():
    """src / dst rows padded (pitch > width) through the raw C ABI."""
    h, w, lv = 200, 301, 3
    x = workloads.uniform(h, w, seed=5)
    src = torch.zeros(h, 320, device=dev())
    src[:, :w] = gpu(x)
    dst = torch.full((h, 333), float("nan"), device=dev())
    ws = d.workspace(h, w, lv, d.DWT2_F32, dev())
    st = d.dwt2_fwd(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), h, w, 320, 333,
                    d.DWT2_F32, d.DWT2_CDF97, lv, 0, 0, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    got = host(dst)
    assert rel_err(got[:, :w], lifting.fwd(x, "cdf97", lv)) <= TOL97
    assert np.isnan(got[:, w:]).all()                   # padding untouched


def test_nan_poisoned_outputs_are_all_written():
    h, w = 257, 391
    x = workloads.uniform(h, w, seed=6)
    out = torch.full((h, w), float("nan"), device=dev())
    d.fwd(gpu(x), "cdf97", 4, out=out)
    assert not torch.isnan(out).any().item()
    back = torch.full((h, w), float("nan"), device=dev())
    d.inv(out, "cdf97", 4, out=back)
    assert not torch.isnan(back).any().item()


# ---- full-size images: sampled parity on crops -----------------------------

def crop_check(x, y_gpu, wavelet, lv, tol):
    H, W = x.shape
    m = window.default_margin(lv)
    worst = 0.0
    for r0, r1, c0, c1 in window.probe_crops(H, W, lv, size=256):
        sub = lifting.fwd(x[r0:r1, c0:c1], wavelet, lv)
        cut = window.crop_pyramid(y_gpu, lv, r0, r1, c0, c1)
        mask = window.crop_valid_mask(H, W, lv, r0, r1, c0, c1, m)
        if wavelet == "cdf53":
            assert np.array_equal(cut[mask], sub[mask]), (r0, c0)
        else:
            worst = max(worst, float(np.abs(cut[mask] - sub[mask]).max()))
    return worst


@pytest.mark.parametrize("n", [4096, 8192])
@pytest.mark.parametrize("lv", [1, 5])
def test_full_size_cdf97_crops(n, lv):
    x = workloads.uniform(n, n, seed=0)
    say("full-size cdf97", n, lv)
    y = d.fwd(gpu(x), "cdf97", lv)
    yh = host(y)
    # relative to the largest coefficient of the whole pyramid (LL grows 2x per level)
    scale = float(np.abs(yh).max())
    worst = crop_check(x, yh, "cdf97", lv, TOL97)
    assert worst / scale <= TOL97
    # the inverse brings the image back (property at any size)
    xr = host(d.inv(y, "cdf97", lv))
    assert np.abs(xr - x).max() <= 1e-4


@pytest.mark.parametrize("lv", [1, 5])
def test_full_size_cdf53_crops(lv):
    n = 8192
    x = workloads.pixels_u8(n, n, seed=0)
    say("full-size cdf53", n, lv)
    y = d.fwd(gpu(x), "cdf53", lv)
    crop_check(x, host(y), "cdf53", lv, 0)
    xr = d.inv(y, "cdf53", lv)
    assert torch.equal(xr.cpu(), torch.from_numpy(x))


# ---- every kernel configuration computes the same values --------------------

def test_kernel_configs_bit_identical():
    """Each coefficient's arithmetic does not depend on the tiling, so every
    kernel configuration (tile shapes, streaming strips and segments) must
    give bit-identical results (a halo, pipeline or race bug breaks it)."""
    # (600, 2056) and (520, 2056): subband widths a multiple of 4, so the
    # vector paths of every tile width run, with interior tiles in between
    cases = [("cdf97", torch.float32, (517, 1283), 3, False), ("cdf97", torch.float32, (1000, 700), 1, True),
             ("cdf97", torch.bfloat16, (300, 260), 2, False), ("cdf53", torch.int32, (613, 901), 4, False),
             ("cdf97", torch.float32, (600, 2056), 2, False), ("cdf97", torch.float32, (600, 2056), 1, True),
             ("cdf97", torch.bfloat16, (260, 2056), 1, False), ("cdf53", torch.int32, (520, 2056), 2, False),
             ("cdf53f", torch.float32, (517, 1283), 3, False), ("cdf53f", torch.float32, (600, 2056), 2, False)]
    for wav, tdt, (h, w), lv, split in cases:
        if wav == "cdf53":
            x = gpu(workloads.pixels_u8(h, w, seed=4))
        else:
            x = gpu(workloads.uniform(h, w, seed=4)).to(tdt)
        # 16-bit storage runs the factored evaluation by default on the tile
        # configurations only; across every configuration the direct fused
        # evaluation is compared (and the default across the tile ones below)
        half = tdt in (torch.bfloat16, torch.float16)
        ref_f = d.fwd(x, wav, lv, split=split, config=0, fused=half)
        ref_i = d.inv(ref_f, wav, lv, split=split, config=0, fused=half)
        if half:
            dflt_f = d.fwd(x, wav, lv, config=0)
            dflt_i = d.inv(dflt_f, wav, lv, config=0)
            for sh in tile_configs()[1:]:
                say("kernel config (16-bit default)", sh, wav, tdt, (h, w), lv)
                f = d.fwd(x, wav, lv, config=sh)
                assert torch.equal(f, dflt_f), sh
                assert torch.equal(d.inv(f, wav, lv, config=sh), dflt_i), sh
        for sh in range(1, d.DWT2_NUM_KERNEL_CONFIGS):
            if not d.config_supports(sh, "fwd", wav, "split" if split else "fused"):
                continue                  # the LDS-plane kernel runs neither the split nor the integer 5/3
            say("kernel config", sh, wav, tdt, (h, w), lv, split)
            f = d.fwd(x, wav, lv, split=split, config=sh, fused=half)
            if split:
                # The split (P = P0 + P1, U = U0 + U1) runs in interior tiles
                # only, and which tiles are interior depends on the tile
                # shape; split and fused arithmetic differ by rounding, so
                # the two results agree to the bar both meet against the
                # oracle (1e-5 relative max-abs), not bit for bit.
                assert rel_err(host(f), host(ref_f)) <= 1e-5
            else:
                assert torch.equal(f, ref_f)
                assert torch.equal(d.inv(f, wav, lv, config=sh, fused=half), ref_i)
        if wav == "cdf97" and tdt == torch.float32 and not split:
            g = ref_f
            a0 = d.adj(g, lv, config=0)
            for sh in range(1, d.DWT2_NUM_KERNEL_CONFIGS):
                if d.config_supports(sh, "adj", wav):
                    assert torch.equal(d.adj(g, lv, config=sh), a0)


# ---- every tile configuration against the oracle ---------------------------
# Shapes with interior tiles for every tile width (subband widths above
# 2 * (64 * BPL) + 4 blocks) and ragged last tiles: heights leave a partial
# last wave, widths end one or a few blocks past a tile; (1034, 2062) has odd
# subband widths (no vector access), (1100, 2104) has subband widths that are
# multiples of 4 (vector access for both tile widths).
CFG_SHAPES = [(1100, 2104), (1034, 2062), (2, 3000), (3000, 6)]


def tile_configs():
    return [i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_TILE]


@pytest.mark.parametrize("shape", CFG_SHAPES)
def test_tile_configs_against_oracle(shape):
    h, w = shape
    x = workloads.uniform(h, w, seed=21)
    xi = workloads.pixels_u8(h, w, seed=22)
    lv = min(3, lifting.max_levels(h, w))
    ref = lifting.fwd(x, "cdf97", lv)
    ref_i = lifting.fwd(xi, "cdf53", lv)
    xg, xig = gpu(x), gpu(xi)
    for cfg in tile_configs():
        say("tile config vs oracle", cfg, shape, lv)
        y = d.fwd(xg, "cdf97", lv, config=cfg)
        assert rel_err(host(y), ref) <= TOL97, cfg
        assert rel_err(host(d.inv(y, "cdf97", lv, config=cfg)), x) <= TOL97, cfg
        ys = d.fwd(xg, "cdf97", lv, split=True, config=cfg)
        assert rel_err(host(ys), ref) <= TOL97, cfg
        yi = d.fwd(xig, "cdf53", lv, config=cfg)
        assert np.array_equal(host(yi), ref_i), cfg
        assert torch.equal(d.inv(yi, "cdf53", lv, config=cfg), xig), cfg


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
def test_storage_bound_interior_tiles(tdt):
    """16-bit storage on an image with interior tiles for every tile width."""
    h, w, lv = 1100, 2104, 2
    xs = torch.from_numpy(workloads.uniform(h, w, seed=23)).to(tdt)
    ref = lifting.fwd(xs.to(torch.float64).numpy(), "cdf97", lv)
    for cfg in tile_configs():
        say("storage interior", tdt, cfg)
        y = d.fwd(xs.to(dev()), "cdf97", lv, config=cfg)
        assert rel_err(host(y), ref) <= 8 * UNIT[tdt], cfg


@pytest.mark.parametrize("tdt,min_psnr", [(torch.bfloat16, 48.0), (torch.float16, 64.0)])
def test_precision_report_1024_5_levels(tdt, min_psnr):
    """16-bit storage, 1024^2, 5 levels forward + inverse: coefficient max-abs
    against the FP64 oracle of the storage-rounded input, and reconstruction
    PSNR (peak 1.0) against that input.  The floors sit ~4 dB below the
    values the arithmetic gives (about 52 dB BF16, 70 dB FP16)."""
    n, lv = 1024, 5
    xq = torch.from_numpy(workloads.uniform(n, n, seed=3)).to(tdt)
    x64 = xq.to(torch.float64).numpy()
    c = d.fwd(xq.to(dev()), "cdf97", lv)
    ref = lifting.fwd(x64, "cdf97", lv)
    err = float(np.abs(host(c) - ref).max())
    r = host(d.inv(c, "cdf97", lv))
    psnr = 10 * np.log10(1.0 / float(((r - x64) ** 2).mean()))
    say("precision", tdt, "coeff max-abs", err, "max |coeff|", float(np.abs(ref).max()), "PSNR dB", psnr)
    assert err <= 8 * UNIT[tdt] * float(np.abs(ref).max())
    assert psnr >= min_psnr


@pytest.mark.parametrize("shape,lv", [((3, 37, 53), 3), ((5, 260, 2056), 2), ((2, 2, 3000), 1),
                                      ((3, 300, 1030), 2)])
def test_plane_batch_equals_single_planes(shape, lv):
    """A plane batch (one launch per level for all planes) equals the
    single-image transform of every plane, bit for bit, in every direction
    and kernel configuration; plane 0 is also checked against the oracle."""
    n, h, w = shape
    x = gpu(workloads.planes(n, h, w, seed=31))
    xi = gpu(np.stack([workloads.pixels_u8(h, w, seed=32 + k) for k in range(n)]))
    for cfg in range(d.DWT2_NUM_KERNEL_CONFIGS):
        say("plane batch", shape, lv, cfg)
        full = d.config_supports(cfg, "adj", "cdf97")       # adjoint and integer 5/3 too
        y = d.fwd(x, "cdf97", lv, config=cfg)
        r = d.inv(y, "cdf97", lv, config=cfg)
        a = d.adj(y, lv, config=cfg) if full else None
        yi = d.fwd(xi, "cdf53", lv, config=cfg) if full else None
        for k in range(n):
            assert torch.equal(y[k], d.fwd(x[k], "cdf97", lv, config=cfg)), (cfg, k)
            assert torch.equal(r[k], d.inv(y[k], "cdf97", lv, config=cfg)), (cfg, k)
            if full:
                assert torch.equal(a[k], d.adj(y[k], lv, config=cfg)), (cfg, k)
                assert torch.equal(yi[k], d.fwd(xi[k], "cdf53", lv, config=cfg)), (cfg, k)
    assert rel_err(host(y[0]), lifting.fwd(host(x[0]), "cdf97", lv)) <= TOL97


# ---- the semi-vector interior path (rows only 8-byte aligned) ---------------
def fwd_pitched(x, wavelet, lv, dst_pitch, config, flags=0):
    """Forward through the raw C ABI into a destination of row pitch
    `dst_pitch` (elements), with `flags` besides the configuration; returns
    the h x w pyramid."""
    h, w = x.shape
    dt = d.dtype_code(x)
    dst = torch.zeros((h, dst_pitch), dtype=x.dtype, device=dev())
    ws = d.workspace(h, w, lv, dt, dev())
    wsp = ctypes.c_void_p(ws.data_ptr() if ws is not None else 0)
    st = d.dwt2_fwd(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(dst.data_ptr()), h, w, w, dst_pitch,
                    dt, d.WAVELETS[wavelet], lv, 0, d.DWT2_FLAG_KERNEL(config) | flags, wsp,
                    ws.numel() if ws is not None else 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return dst[:, :w]


@pytest.mark.parametrize("shape", [(1034, 2062), (600, 1030), (520, 2054), (1100, 2052)])
def test_semi_vector_path_bit_identical(shape):
    """Widths of 2 mod 4 (odd low-pass width) and subband widths of 2 mod 4
    (for 4-block tiles): with an even destination pitch the interior tiles
    take the semi-vector path, with an odd one the border path everywhere.
    Both compute the same arithmetic, so they agree bit for bit; the result
    is also checked against the oracle."""
    h, w = shape
    xf = gpu(workloads.uniform(h, w, seed=61))
    xi = gpu(workloads.pixels_u8(h, w, seed=62))
    ref = lifting.fwd(host(xf), "cdf97", 3)
    for cfg in tile_configs():
        # BF16 twice: with the direct fused evaluation (which has the
        # semi-vector path) and with the default factored one
        for x, wav, fl in ((xf, "cdf97", 0), (xf.to(torch.bfloat16), "cdf97", d.DWT2_FLAG_FUSED),
                           (xf.to(torch.bfloat16), "cdf97", 0), (xf, "cdf53f", 0), (xi, "cdf53", 0)):
            for lv in (1, 3):
                say("semi-vector path", shape, cfg, wav, x.dtype, fl, lv)
                even = fwd_pitched(x, wav, lv, w + 2 if w % 4 == 0 else w, cfg, fl)
                odd = fwd_pitched(x, wav, lv, w + 1, cfg, fl)
                assert torch.equal(even, odd), (cfg, wav, x.dtype, lv)
                assert torch.equal(even, d.fwd(x, wav, lv, config=cfg, fused=fl != 0)), (cfg, wav, x.dtype, lv)
        y = fwd_pitched(xf, "cdf97", 3, w, cfg)
        assert rel_err(host(y), ref) <= TOL97, cfg


def back_pitched(fn, c, wavelet, lv, src_pitch, config, flags=0):
    """Inverse or adjoint through the raw C ABI from a source of row pitch
    `src_pitch` (elements) holding the pyramid c; returns the h x w image."""
    h, w = c.shape
    dt = d.dtype_code(c)
    src = torch.zeros((h, src_pitch), dtype=c.dtype, device=dev())
    src[:, :w] = c
    dst = torch.empty_like(c)
    ws = d.workspace(h, w, lv, dt, dev())
    wsp = ctypes.c_void_p(ws.data_ptr() if ws is not None else 0)
    st = fn(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), h, w, src_pitch, w,
            dt, d.WAVELETS[wavelet], lv, 0, d.DWT2_FLAG_KERNEL(config) | flags, wsp,
            ws.numel() if ws is not None else 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return dst


@pytest.mark.parametrize("shape", [(1034, 2062), (600, 1030), (1100, 2052)])
def test_semi_vector_path_inverse_adjoint_bit_identical(shape):
    """The inverse and adjoint of the same shapes: an even source pitch takes
    the semi-vector path in the interior tiles, an odd one the border path
    everywhere (destination contiguous, even width); bit for bit equal, and
    the inverse restores the oracle's coefficients' image."""
    h, w = shape
    x = workloads.uniform(h, w, seed=63)
    c = lifting.fwd(x, "cdf97", 3).astype(np.float32)
    cg = gpu(c)
    ci = gpu(lifting.fwd(workloads.pixels_u8(h, w, seed=64), "cdf53", 3).astype(np.int32))
    for cfg in tile_configs():
        for cc, wav, fl in ((cg, "cdf97", 0), (cg.to(torch.bfloat16), "cdf97", d.DWT2_FLAG_FUSED),
                            (cg.to(torch.bfloat16), "cdf97", 0), (cg, "cdf53f", 0), (ci, "cdf53", 0)):
            for lv in (1, 3):
                say("semi-vector inverse", shape, cfg, wav, cc.dtype, fl, lv)
                even = back_pitched(d.dwt2_inv, cc, wav, lv, w + 2 if w % 4 == 0 else w, cfg, fl)
                odd = back_pitched(d.dwt2_inv, cc, wav, lv, w + 1, cfg, fl)
                assert torch.equal(even, odd), (cfg, wav, cc.dtype, lv)
                assert torch.equal(even, d.inv(cc, wav, lv, config=cfg, fused=fl != 0)), (cfg, wav, cc.dtype, lv)
        say("semi-vector adjoint", shape, cfg)
        even = back_pitched(d.dwt2_adj, cg, "cdf97", 3, w + 2 if w % 4 == 0 else w, cfg)
        odd = back_pitched(d.dwt2_adj, cg, "cdf97", 3, w + 1, cfg)
        assert torch.equal(even, odd), cfg
        r = back_pitched(d.dwt2_inv, cg, "cdf97", 3, w + 2 if w % 4 == 0 else w, cfg)
        assert rel_err(host(r), lifting.inv(c, "cdf97", 3)) <= TOL97, cfg


@pytest.mark.parametrize("tdt", [torch.float32, torch.bfloat16])
def test_two_levels_equal_two_single_level_calls(tdt):
    # 8192^2: level 1's LL band (64 MiB FP32, 32 MiB BF16) and, for the
    # inverse, level 2's image take the variant that stores them with
    # ordinary stores for the next level; every single-level call stores
    # nontemporally.  Same values either way: a two-level call equals two
    # one-level calls bit for bit, forward and inverse.
    n, h = 8192, 4096
    say("two levels vs two single-level calls", tdt)
    x = gpu(workloads.uniform(n, n, seed=4), tdt)
    two = d.fwd(x, "cdf97", 2, config=3)
    one = d.fwd(x, "cdf97", 1, config=3)
    one[:h, :h] = d.fwd(one[:h, :h].contiguous(), "cdf97", 1, config=3)
    assert torch.equal(two, one)
    back = d.inv(two, "cdf97", 2, config=3)
    c1 = two.clone()
    c1[:h, :h] = d.inv(two[:h, :h].contiguous(), "cdf97", 1, config=3)
    assert torch.equal(back, d.inv(c1, "cdf97", 1, config=3))


def test_multilevel_graph_replay():
    """A 5-level forward + inverse of a plane stack (one launch per level,
    workspace from the graph's pool) captured in a graph and replayed with
    eager work and synchronisations in between; every replay must equal
    the eager result."""
    x = gpu(workloads.planes(2, 700, 1030, seed=71))
    y = torch.empty_like(x)
    r = torch.empty_like(x)

    def step():
        d.fwd(x, "cdf97", 5, out=y)
        d.inv(y, "cdf97", 5, out=r)
    step()
    torch.cuda.synchronize()
    ey, er = y.clone(), r.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    for rep in range(3):
        y.fill_(float("nan"))
        r.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ey) and torch.equal(r, er), rep
    assert rel_err(host(y[1]), lifting.fwd(host(x[1]), "cdf97", 5)) <= TOL97
