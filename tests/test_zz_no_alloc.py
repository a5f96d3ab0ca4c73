"""dwt2_fwd_noalloc: the forward transform with its workspace in the
library's fixed device array (for callers that cannot allocate), called
through the C ABI and compared bit for bit with dwt2_fwd given a caller
workspace (same kernels, same default configuration).  Each case makes two
calls in a row, the second on a smaller image, so the second call runs on
the array the first one left behind."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def c_args(x, y, levels, wavelet):
    h, w = x.shape
    return (ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), h, w, x.stride(0), y.stride(0),
            d.dtype_code(x), d.WAVELETS[wavelet], levels, d.DWT2_SYMMETRIC_WHOLE, 0)


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def noalloc(x, levels, wavelet):
    y = torch.full_like(x, -7)
    print(f"dwt2_fwd_noalloc {tuple(x.shape)} {x.dtype} {wavelet} levels={levels}", flush=True)
    st = d.dwt2_fwd_noalloc(*c_args(x, y, levels, wavelet), stream())
    assert st == d.DWT2_OK, d.status_string(st)
    return y


def with_workspace(x, levels, wavelet):
    y = torch.full_like(x, -7)
    h, w = x.shape
    st, n = d.dwt2_workspace_bytes(h, w, levels, d.dtype_code(x))
    assert st == d.DWT2_OK
    assert n <= d.DWT2_SCRATCH_BYTES
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=x.device)
    st = d.dwt2_fwd(*c_args(x, y, levels, wavelet), ctypes.c_void_p(ws.data_ptr() if n else 0), n, stream())
    assert st == d.DWT2_OK, d.status_string(st)
    return y


def image(h, w, dtype, seed):
    if dtype == torch.int32:
        return torch.from_numpy(workloads.pixels_u8(h, w, seed)).to(dev())
    return torch.from_numpy(workloads.uniform(h, w, seed)).to(dev()).to(dtype)


# (first call, second call): (h, w, levels), the second image smaller
CASES = [
    ("cdf97", torch.float32, (8192, 8192, 5), (1030, 998, 3)),
    ("cdf97", torch.bfloat16, (4096, 4094, 6), (515, 333, 4)),
    ("cdf53", torch.int32, (4096, 4096, 4), (777, 513, 2)),
    ("cdf97", torch.float32, (2050, 1026, 1), (64, 66, 5)),
]


@pytest.mark.parametrize("wavelet,dtype,first,second", CASES)
def test_noalloc_equals_workspace_call(wavelet, dtype, first, second):
    xs = [image(h, w, dtype, seed) for seed, (h, w, _) in enumerate((first, second))]
    lv = [first[2], second[2]]
    # two calls in a row on the shared array, then the references
    ys = [noalloc(x, l, wavelet) for x, l in zip(xs, lv)]
    torch.cuda.synchronize()
    refs = [with_workspace(x, l, wavelet) for x, l in zip(xs, lv)]
    torch.cuda.synchronize()
    for y, r in zip(ys, refs):
        assert torch.equal(y, r)
    # the larger call again after the smaller one: the array's old contents do not matter
    y = noalloc(xs[0], lv[0], wavelet)
    torch.cuda.synchronize()
    assert torch.equal(y, refs[0])
