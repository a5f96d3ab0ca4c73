"""Host-side checks of the C ABI: the library loads, exports every function
include/dwt2.h declares, and rejects every invalid call before touching HIP
(no compute call runs here: each call below fails its argument checks)."""
import ctypes
import os
import re

import pytest

import paper_1704_08657_amd as d
from oracle import lifting

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwt2.h")

pytestmark = pytest.mark.skipif(not os.path.exists(d.LIB_PATH), reason="libdwt2.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(dwt2_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert {"dwt2_fwd", "dwt2_inv", "dwt2_adj", "dwt2_max_levels", "dwt2_workspace_bytes"} <= set(names)
    L = d.lib()
    for n in names:
        assert hasattr(L, n), n
    # the binding wraps every declared function with a signature
    assert set(names) <= set(d.SIGNATURES)


@pytest.mark.parametrize("h,w", [(1, 5), (2, 2), (3, 2), (5, 7), (64, 66), (8192, 8192), (2, 1 << 20), (1000, 3)])
def test_max_levels_matches_oracle(h, w):
    expect = lifting.max_levels(h, w) if h >= 2 and w >= 2 else 0
    assert d.dwt2_max_levels(h, w) == expect


def test_workspace_bytes():
    st, n = d.dwt2_workspace_bytes(512, 512, 1, d.DWT2_F32)
    assert st == 0 and n == 0
    # one level never needs a workspace, for any plane count (the binding
    # relies on it and skips the query)
    for h, w, planes in [(2, 2, 1), (37, 53, 3), (4096, 4094, 1000)]:
        m = ctypes.c_size_t(1)
        assert d.lib().dwt2_workspace_bytes_planes(h, w, 1, d.DWT2_F32, planes, ctypes.byref(m)) == 0
        assert m.value == 0
    # a float multi-level forward runs persistently: the LL band of every
    # level but the last (4096^2, 2048^2, 1024^2, 512^2, pitches multiple of
    # 64) plus the work tables, which for one image fit in a few KiB
    bands = 4096 * 4096 + 2048 * 2048 + 1024 * 1024 + 512 * 512
    st, n = d.dwt2_workspace_bytes(8192, 8192, 5, d.DWT2_F32)
    assert st == 0 and bands * 4 <= n <= bands * 4 + 16384
    st, n = d.dwt2_workspace_bytes(8192, 8192, 5, d.DWT2_BF16)
    assert st == 0 and bands * 2 <= n <= bands * 2 + 16384
    # int32 (reversible 5/3) keeps the two ping-pong buffers of the level
    # launches: LL of level 1 (4096^2) and level 2 (2048^2)
    st, n = d.dwt2_workspace_bytes(8192, 8192, 5, d.DWT2_I32)
    assert st == 0 and n == 4096 * 4096 * 4 + 2048 * 2048 * 4
    st, _ = d.dwt2_workspace_bytes(8192, 8192, 14, d.DWT2_F32)
    assert st == -3
    st, _ = d.dwt2_workspace_bytes(1, 8, 1, d.DWT2_F32)
    assert st == -2
    st, _ = d.dwt2_workspace_bytes(8, 8, 1, 9)
    assert st == -4


FAKE_SRC = 0x10000000
FAKE_DST = 0x20000000
FAKE_WS = 0x30000000


def call(fn=d.dwt2_fwd, src=FAKE_SRC, dst=FAKE_DST, h=64, w=64, sp=64, dp=64, dtype=d.DWT2_F32,
         wav=d.DWT2_CDF97, levels=1, boundary=0, flags=0, ws=0, ws_n=0):
    return fn(ctypes.c_void_p(src), ctypes.c_void_p(dst), h, w, sp, dp, dtype, wav, levels, boundary,
              flags, ctypes.c_void_p(ws), ws_n, None)


@pytest.mark.parametrize("fn", [d.dwt2_fwd, d.dwt2_inv, d.dwt2_adj])
def test_argument_errors(fn):
    assert call(fn, src=0) == -1
    assert call(fn, dst=0) == -1
    assert call(fn, h=1) == -2
    assert call(fn, w=0) == -2
    assert call(fn, sp=63) == -7
    assert call(fn, dp=10) == -7
    assert call(fn, levels=0) == -3
    assert call(fn, levels=7) == -3          # 64 x 64 allows 6
    assert call(fn, boundary=1) == -6
    assert call(fn, dtype=7) == -4
    assert call(fn, flags=1 << 7) == -11
    assert call(fn, flags=d.DWT2_FLAG_FUSED | d.DWT2_FLAG_FACTORED) == -11   # one scheme at most
    # workspace required for 2 levels
    assert call(fn, levels=2) == -8
    assert call(fn, levels=2, ws=FAKE_WS, ws_n=10) == -8
    # overlapping src / dst
    assert call(fn, dst=FAKE_SRC + 64 * 4) == -9
    # workspace overlapping dst
    st, n = d.dwt2_workspace_bytes(64, 64, 2, d.DWT2_F32)
    assert call(fn, levels=2, ws=FAKE_DST + 16, ws_n=n) == -9


def test_wavelet_dtype_pairs():
    assert call(dtype=d.DWT2_I32, wav=d.DWT2_CDF97) == -4
    assert call(dtype=d.DWT2_F32, wav=d.DWT2_CDF53_REV) == -4
    assert call(dtype=d.DWT2_BF16, wav=d.DWT2_CDF53_REV) == -4
    assert call(wav=5) == -5
    # the real-valued CDF 5/3 takes float storage, has no adjoint, allows the split
    assert call(dtype=d.DWT2_I32, wav=d.DWT2_CDF53) == -4
    assert call(d.dwt2_adj, wav=d.DWT2_CDF53) == -5
    for dt in (d.DWT2_F32, d.DWT2_BF16, d.DWT2_F16):
        assert call(wav=d.DWT2_CDF53, dtype=dt, flags=d.DWT2_FLAG_SPLIT, dst=FAKE_SRC + 4) == -9
    # the adjoint is defined for the linear CDF 9/7 only
    assert call(d.dwt2_adj, dtype=d.DWT2_I32, wav=d.DWT2_CDF53_REV) == -5
    # the split is a CDF 9/7 forward / inverse option
    assert call(dtype=d.DWT2_I32, wav=d.DWT2_CDF53_REV, flags=d.DWT2_FLAG_SPLIT) == -11
    assert call(d.dwt2_adj, flags=d.DWT2_FLAG_SPLIT) == -11


def test_separable_flag_combinations():
    # the separable comparison scheme: forward / inverse, both wavelets, tile
    # configurations only, not together with the split, no adjoint
    stream_cfg = next(i for i in range(d.DWT2_NUM_KERNEL_CONFIGS)
                      if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_STREAM)
    for sep in (d.DWT2_FLAG_SEPARABLE, d.DWT2_FLAG_FACTORED):
        for fn in (d.dwt2_fwd, d.dwt2_inv):
            assert call(fn, flags=sep | d.DWT2_FLAG_SPLIT) == -11
            assert call(fn, flags=sep | d.DWT2_FLAG_KERNEL(stream_cfg)) == -11
            # valid combinations get past the flag checks (to the fake-pointer alias check)
            assert call(fn, flags=sep, dst=FAKE_SRC + 4) == -9
            assert call(fn, flags=sep | d.DWT2_FLAG_KERNEL(3), dst=FAKE_SRC + 4) == -9
            assert call(fn, flags=sep, dtype=d.DWT2_I32, wav=d.DWT2_CDF53_REV, dst=FAKE_SRC + 4) == -9
        assert call(d.dwt2_adj, flags=sep) == -11
    assert call(flags=d.DWT2_FLAG_SEPARABLE | d.DWT2_FLAG_FACTORED) == -11


def test_status_strings():
    for s in range(0, -13, -1):
        assert d.status_string(s) != "unknown status"
    assert d.status_string(-99) == "unknown status"


def test_tensor_api_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(RuntimeError, match="GPU only"):
        d.fwd(torch.zeros(8, 8))


def test_batched_argument_errors():
    imgs = (d.dwt2_image * 2)()
    imgs[0] = d.dwt2_image(FAKE_SRC, FAKE_DST, 64, 64, 64, 64)
    imgs[1] = d.dwt2_image(FAKE_SRC + (1 << 24), FAKE_DST + (1 << 24), 100, 70, 70, 70)
    L = d.lib()
    hp = ctypes.cast(imgs, ctypes.c_void_p)
    n = ctypes.c_size_t(0)
    assert L.dwt2_workspace_bytes_batched(hp, 2, d.DWT2_F32, 3, ctypes.byref(n)) == 0 and n.value > 0
    need = n.value
    assert L.dwt2_workspace_bytes_batched(hp, 0, d.DWT2_F32, 3, ctypes.byref(n)) == -12
    assert L.dwt2_workspace_bytes_batched(hp, 2, d.DWT2_F32, 9, ctypes.byref(n)) == -3

    # every call below must fail its argument checks (the pointers are fake)
    def fb(host=hp, dev_=0x50000000, count=2, dtype=d.DWT2_F32, wav=d.DWT2_CDF97, levels=3, boundary=0,
           flags=0, ws=FAKE_WS, ws_n=need):
        return L.dwt2_fwd_batched(host, ctypes.c_void_p(dev_), count, dtype, wav, levels, boundary, flags,
                                  ctypes.c_void_p(ws), ws_n, None)
    assert fb(host=None) == -1
    assert fb(dev_=0) == -1
    assert fb(ws=0) == -1
    assert fb(count=0) == -12
    assert fb(dtype=d.DWT2_I32) == -4
    assert fb(wav=d.DWT2_CDF53_REV) == -5
    assert fb(boundary=2) == -6
    assert fb(levels=0) == -3
    assert fb(ws_n=need - 1) == -8
    stream_cfg = next(i for i in range(d.DWT2_NUM_KERNEL_CONFIGS)
                      if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_STREAM)
    assert fb(flags=d.DWT2_FLAG_KERNEL(stream_cfg)) == -11   # not a batched configuration
    assert fb(ws=FAKE_DST + 8) == -9
    bad = (d.dwt2_image * 1)()
    bad[0] = d.dwt2_image(FAKE_SRC, FAKE_SRC + 4, 64, 64, 64, 64)
    assert fb(host=ctypes.cast(bad, ctypes.c_void_p), count=1) == -9
    bad[0] = d.dwt2_image(FAKE_SRC, FAKE_DST, 1, 64, 64, 64)
    assert fb(host=ctypes.cast(bad, ctypes.c_void_p), count=1) == -2


def test_batched_rejects_overlap_across_images():
    """All images' tiles run in the same launches: one image's dst must not
    overlap another image's dst or src (sources may share memory)."""
    L = d.lib()
    img = 64 * 64 * 4                                   # bytes of one 64 x 64 FP32 image

    def batch(*specs):
        a = (d.dwt2_image * len(specs))()
        for k, (s, t) in enumerate(specs):
            a[k] = d.dwt2_image(s, t, 64, 64, 64, 64)
        return a

    def fb(arr):
        hp = ctypes.cast(arr, ctypes.c_void_p)
        n = ctypes.c_size_t(0)
        assert L.dwt2_workspace_bytes_batched(hp, len(arr), d.DWT2_F32, 2, ctypes.byref(n)) == 0
        return L.dwt2_fwd_batched(hp, ctypes.c_void_p(0x50000000), len(arr), d.DWT2_F32, d.DWT2_CDF97, 2, 0, 0,
                                  ctypes.c_void_p(FAKE_WS), n.value, None)
    S, T = FAKE_SRC, FAKE_DST
    # two images writing overlapping destinations (last element of one, first of the next)
    assert fb(batch((S, T), (S + img, T + img - 4))) == -9
    # the same destination twice
    assert fb(batch((S, T), (S + img, T))) == -9
    # one image's destination inside another image's source, either order
    assert fb(batch((S, T), (S + img, S + 8))) == -9
    assert fb(batch((S + img, S + 8), (S, T))) == -9
    # destinations far apart, an unordered list, and three overlapping
    # destinations among five images
    far = [(S + k * img, T + (4 - k) * 2 * img) for k in range(5)]
    far[3] = (far[3][0], far[1][1] + img - 4)
    assert fb(batch(*far)) == -9

    # batches that pass the overlap check: they then fail the workspace size
    # check that follows it (these fake pointers must never reach a launch)
    def fb_small_ws(arr):
        hp = ctypes.cast(arr, ctypes.c_void_p)
        n = ctypes.c_size_t(0)
        assert L.dwt2_workspace_bytes_batched(hp, len(arr), d.DWT2_F32, 2, ctypes.byref(n)) == 0
        return L.dwt2_fwd_batched(hp, ctypes.c_void_p(0x50000000), len(arr), d.DWT2_F32, d.DWT2_CDF97, 2, 0, 0,
                                  ctypes.c_void_p(FAKE_WS), n.value - 1, None)
    far = [(S + k * img, T + (4 - k) * 2 * img) for k in range(5)]
    assert fb_small_ws(batch(*far)) == -8
    # sources may overlap one another: they are only read
    assert fb_small_ws(batch((S, T), (S, T + img))) == -8
    # adjacent destinations, touching but not overlapping
    assert fb_small_ws(batch((S, T), (S + img, T + img))) == -8


def test_kernel_configs_listed():
    for i in range(d.DWT2_NUM_KERNEL_CONFIGS):
        st, algo, waves, rows, cc, cr = d.dwt2_kernel_config(i)
        assert st == 0 and algo in (d.DWT2_ALGO_TILE, d.DWT2_ALGO_STREAM, d.DWT2_ALGO_LDS) and waves >= 1 and cr >= 1
    assert d.dwt2_kernel_config(d.DWT2_NUM_KERNEL_CONFIGS)[0] == -11


def test_plane_batch_argument_errors():
    L = d.lib()
    n = ctypes.c_size_t(0)
    assert L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_F32, 3, ctypes.byref(n)) == 0
    one = ctypes.c_size_t(0)
    assert L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_F32, 1, ctypes.byref(one)) == 0
    # every plane keeps its own LL bands (plus the persistent forward's
    # work tables, which grow with the plane count)
    assert n.value >= 3 * (32 * 64 * 4) and n.value > one.value > 0
    ni, onei = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_I32, 3, ctypes.byref(ni)) == 0
    assert L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_I32, 1, ctypes.byref(onei)) == 0
    assert ni.value == 3 * onei.value > 0             # int32: one LL buffer pair per plane
    assert L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_F32, 0, ctypes.byref(n)) == -12
    need = L.dwt2_workspace_bytes_planes(64, 64, 2, d.DWT2_F32, 3, ctypes.byref(n)) or n.value

    def fp(fn=L.dwt2_fwd_planes, src=FAKE_SRC, dst=FAKE_DST, planes=3, sps=64 * 64, dps=64 * 64, levels=2,
           ws=FAKE_WS, ws_n=need):
        return fn(ctypes.c_void_p(src), ctypes.c_void_p(dst), planes, sps, dps, 64, 64, 64, 64, d.DWT2_F32,
                  d.DWT2_CDF97, levels, 0, 0, ctypes.c_void_p(ws), ws_n, None)
    for fn in (L.dwt2_fwd_planes, L.dwt2_inv_planes, L.dwt2_adj_planes):
        assert fp(fn, planes=0) == -12
        assert fp(fn, sps=64 * 64 - 1) == -7          # planes of src would overlap
        assert fp(fn, dps=100) == -7
        assert fp(fn, ws_n=need - 1) == -8
        assert fp(fn, dst=FAKE_SRC + 2 * 64 * 64 * 4) == -9   # dst inside src's third plane
        assert fp(fn, ws=FAKE_DST + 3 * 64 * 64 * 4 - 8) == -9
    # one plane: the stride is not used
    st, n1 = d.dwt2_workspace_bytes(64, 64, 2, d.DWT2_F32)
    assert fp(planes=1, sps=0, dps=0, ws_n=n1 - 1) == -8


def test_lds_kernel_argument_rules():
    """DD 13/7 and the polyconvolution run on the LDS-plane configurations
    only (the default for them); those configurations run the float
    wavelets' forward and inverse with the fused, separable and
    polyconvolution schemes.  Every call below fails its checks on the host
    (fake pointers)."""
    L = d.lib()
    lds = [i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_LDS]
    tile = [i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_TILE]
    assert lds and tile

    def c(fn, wav=d.DWT2_CDF97, dtype=d.DWT2_F32, flags=0, dst=FAKE_DST):
        return fn(ctypes.c_void_p(FAKE_SRC), ctypes.c_void_p(dst), 64, 64, 64, 64, dtype, wav, 1, 0, flags,
                  None, 0, None)
    for fn in (L.dwt2_fwd, L.dwt2_inv):
        assert c(fn, wav=d.DWT2_DD137, flags=d.DWT2_FLAG_KERNEL(tile[0])) == -11
        assert c(fn, flags=d.DWT2_FLAG_POLYCONV | d.DWT2_FLAG_KERNEL(tile[0])) == -11
        assert c(fn, wav=d.DWT2_CDF53, flags=d.DWT2_FLAG_POLYCONV) == -11      # one pair: no polyconvolution
        assert c(fn, wav=d.DWT2_DD137, flags=d.DWT2_FLAG_POLYCONV) == -11
        assert c(fn, flags=d.DWT2_FLAG_POLYCONV | d.DWT2_FLAG_SEPARABLE) == -11
        assert c(fn, wav=d.DWT2_CDF53_REV, dtype=d.DWT2_I32, flags=d.DWT2_FLAG_KERNEL(lds[0])) == -11
        assert c(fn, flags=d.DWT2_FLAG_SPLIT | d.DWT2_FLAG_KERNEL(lds[0])) == -11
        assert c(fn, flags=d.DWT2_FLAG_FACTORED | d.DWT2_FLAG_KERNEL(lds[0])) == -11
        assert c(fn, wav=d.DWT2_DD137, dtype=d.DWT2_I32) == -4
        # valid otherwise: only the overlap check (dst inside src) stops these
        assert c(fn, wav=d.DWT2_DD137, dst=FAKE_SRC + 8) == -9
        assert c(fn, flags=d.DWT2_FLAG_POLYCONV, dst=FAKE_SRC + 8) == -9
        assert c(fn, flags=d.DWT2_FLAG_SEPARABLE | d.DWT2_FLAG_KERNEL(lds[1]), dst=FAKE_SRC + 8) == -9
    assert c(L.dwt2_adj, wav=d.DWT2_DD137) == -5
    assert c(L.dwt2_adj, flags=d.DWT2_FLAG_KERNEL(lds[0])) == -11
    for i in lds:
        st, algo, waves, rows, cc, cr = d.dwt2_kernel_config(i)
        assert (st, algo, waves) == (0, d.DWT2_ALGO_LDS, 4) and cc >= 32 and cr >= 16
    # the binding's table of supported cases agrees
    assert d.config_supports(lds[0], "fwd", "dd137") and not d.config_supports(tile[0], "fwd", "dd137")
    assert d.config_supports(lds[0], "inv", "cdf97", "polyconv") and not d.config_supports(lds[0], "adj", "cdf97")


def test_noalloc_rejects_before_hip():
    """dwt2_fwd_noalloc checks its arguments, and the fixed scratch size,
    on the host before any HIP call (fake pointers: nothing may run)."""
    def na(h=64, w=64, levels=2, dtype=d.DWT2_F32, wav=d.DWT2_CDF97, src=FAKE_SRC, dst=FAKE_DST, flags=0):
        return d.dwt2_fwd_noalloc(ctypes.c_void_p(src), ctypes.c_void_p(dst), h, w, w, w, dtype, wav, levels, 0,
                                  flags, None)
    assert na(src=0) == -1
    assert na(h=1) == -2
    assert na(levels=9) == -3
    assert na(dtype=d.DWT2_I32) == -4
    assert na(flags=1 << 7) == -11
    assert na(dst=FAKE_SRC + 64) == -9
    # 16384^2 FP32 at 2 levels keeps an 8192^2 LL band (256 MiB): beyond the array
    st, n = d.dwt2_workspace_bytes(16384, 16384, 2, d.DWT2_F32)
    assert st == 0 and n > d.DWT2_SCRATCH_BYTES
    assert na(h=16384, w=16384, levels=2, dst=FAKE_DST + (1 << 31)) == d.DWT2_E_SCRATCH
    assert "scratch" in d.status_string(d.DWT2_E_SCRATCH)
    # the largest case the array is sized for fits: 8192^2 FP32 at every level count
    for lv in range(1, 14):
        st, n = d.dwt2_workspace_bytes(8192, 8192, lv, d.DWT2_F32)
        assert st == 0 and n <= d.DWT2_SCRATCH_BYTES


def test_persistent_flag_rules():
    """DWT2_FLAG_PERSISTENT: forward CDF 9/7, fused, split or factored steps,
    tile configurations; every other use is rejected on the host (fake
    pointers)."""
    P = d.DWT2_FLAG_PERSISTENT
    st, n = d.dwt2_workspace_bytes(64, 64, 3, d.DWT2_F32)
    assert st == 0 and n > 0
    for fn in (d.dwt2_inv, d.dwt2_adj):
        assert call(fn, flags=P, levels=3, ws=FAKE_WS, ws_n=n) == -11
    assert call(flags=P, levels=3, dtype=d.DWT2_I32, wav=d.DWT2_CDF53_REV, ws=FAKE_WS, ws_n=n) == -11
    assert call(flags=P | d.DWT2_FLAG_SEPARABLE, levels=3, ws=FAKE_WS, ws_n=n) == -11
    assert call(flags=P | d.DWT2_FLAG_POLYCONV, levels=3, ws=FAKE_WS, ws_n=n) == -11
    assert call(flags=P | d.DWT2_FLAG_FUSED | d.DWT2_FLAG_SPLIT, levels=3, ws=FAKE_WS, ws_n=n) == -11
    stream_cfg = next(i for i in range(d.DWT2_NUM_KERNEL_CONFIGS) if d.dwt2_kernel_config(i)[1] == d.DWT2_ALGO_STREAM)
    assert call(flags=P | d.DWT2_FLAG_KERNEL(stream_cfg), levels=3, ws=FAKE_WS, ws_n=n) == -11
    assert call(flags=P, levels=3, ws=FAKE_WS, ws_n=n - 1) == -8     # the persistent tables need the full workspace
