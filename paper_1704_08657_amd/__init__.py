"""Python binding of libdwt2: the non-separable 2-D lifting DWT on MI355X.

The library (C ABI in include/dwt2.h) computes the transform of Barina et
al., "Accelerating Discrete Wavelet Transforms on Parallel Architectures":
each pair of separable lifting steps fused into one spatial predict T_P and
one spatial update S_U per barrier, CDF 9/7 (FP32 arithmetic; FP32, BF16 or
FP16 storage) and reversible CDF 5/3 (int32), forward, inverse and adjoint,
multi-level Mallat layout, whole-point symmetric borders.

This module only marshals arguments: PyTorch supplies device memory and the
current stream; every step of the transform runs in the HIP kernels.  There
is no CPU fallback: if the library is not built or the tensor is not on a
GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwt2.so")

# enums of include/dwt2.h
DWT2_OK = 0
DWT2_E_HIP = -10
DWT2_E_SCRATCH = -13
DWT2_E_TIMEOUT = -14
DWT2_WORKSPACE_STATUS_BYTES = 4
DWT2_SCRATCH_BYTES = 96 << 20
DWT2_CDF97, DWT2_CDF53_REV, DWT2_CDF53, DWT2_DD137 = 0, 1, 2, 3
DWT2_F32, DWT2_BF16, DWT2_F16, DWT2_I32 = 0, 1, 2, 3
DWT2_SYMMETRIC_WHOLE = 0
DWT2_FLAG_SPLIT = 1
DWT2_FLAG_SEPARABLE = 2
DWT2_FLAG_FACTORED = 4
DWT2_FLAG_POLYCONV = 8
DWT2_FLAG_PERSISTENT = 16
DWT2_FLAG_FUSED = 32
DWT2_FLAG_KERNEL_SHIFT = 8
DWT2_NUM_KERNEL_CONFIGS = 10
DWT2_ALGO_TILE, DWT2_ALGO_STREAM, DWT2_ALGO_LDS = 0, 1, 2


def DWT2_FLAG_KERNEL(i: int) -> int:
    return (i + 1) << DWT2_FLAG_KERNEL_SHIFT


# "cdf53": the reversible integer CDF 5/3; "cdf53f": the real-valued one;
# "dd137": Deslauriers-Dubuc 13/7
WAVELETS = {"cdf97": DWT2_CDF97, "cdf53": DWT2_CDF53_REV, "cdf53f": DWT2_CDF53, "dd137": DWT2_DD137}

# every function the header declares, with its ctypes signature
_c_int, _c_i32, _c_i64, _c_u, _c_sz, _c_p = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.c_uint, ctypes.c_size_t, ctypes.c_void_p)
_TRANSFORM_ARGS = [_c_p, _c_p, _c_i32, _c_i32, _c_i64, _c_i64, _c_int, _c_int, _c_int, _c_int,
                   _c_u, _c_p, _c_sz, _c_p]
_PLANES_ARGS = [_c_p, _c_p, _c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _c_i64, _c_i64, _c_int, _c_int, _c_int,
                _c_int, _c_u, _c_p, _c_sz, _c_p]
SIGNATURES = {
    "dwt2_max_levels": (_c_int, [_c_i32, _c_i32]),
    "dwt2_workspace_bytes": (_c_int, [_c_i32, _c_i32, _c_int, _c_int, ctypes.POINTER(_c_sz)]),
    "dwt2_fwd": (_c_int, _TRANSFORM_ARGS),
    "dwt2_inv": (_c_int, _TRANSFORM_ARGS),
    "dwt2_adj": (_c_int, _TRANSFORM_ARGS),
    "dwt2_workspace_bytes_planes": (_c_int, [_c_i32, _c_i32, _c_int, _c_int, _c_i32, ctypes.POINTER(_c_sz)]),
    "dwt2_fwd_planes": (_c_int, _PLANES_ARGS),
    "dwt2_inv_planes": (_c_int, _PLANES_ARGS),
    "dwt2_adj_planes": (_c_int, _PLANES_ARGS),
    "dwt2_kernel_config": (_c_int, [_c_int] + [ctypes.POINTER(_c_int)] * 5),
    "dwt2_workspace_bytes_batched": (_c_int, [_c_p, _c_int, _c_int, _c_int, ctypes.POINTER(_c_sz)]),
    "dwt2_fwd_batched": (_c_int, [_c_p, _c_p, _c_int, _c_int, _c_int, _c_int, _c_int, _c_u, _c_p, _c_sz, _c_p]),
    "dwt2_fwd_noalloc": (_c_int, [_c_p, _c_p, _c_i32, _c_i32, _c_i64, _c_i64, _c_int, _c_int, _c_int, _c_int,
                                  _c_u, _c_p]),
    "dwt2_workspace_status": (_c_int, [_c_p]),
    "dwt2_status_string": (ctypes.c_char_p, [_c_int]),
    "dwt2_last_hip_error": (ctypes.c_char_p, []),
}

_lib = None


class DWT2Error(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = f"{what}: {status_string(status)} ({status})"
        if status == DWT2_E_HIP:
            msg += ": " + lib().dwt2_last_hip_error().decode()
        super().__init__(msg)
        self.status = status


def lib():
    """The loaded libdwt2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1704_08657_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ---- thin wrappers with the C names -------------------------------------

def dwt2_max_levels(height: int, width: int) -> int:
    return lib().dwt2_max_levels(height, width)


def dwt2_workspace_bytes(height: int, width: int, levels: int, dtype: int):
    """(status, bytes)."""
    n = ctypes.c_size_t(0)
    st = lib().dwt2_workspace_bytes(height, width, levels, dtype, ctypes.byref(n))
    return st, n.value


def dwt2_fwd(*args) -> int:
    return lib().dwt2_fwd(*args)


def dwt2_inv(*args) -> int:
    return lib().dwt2_inv(*args)


def dwt2_adj(*args) -> int:
    return lib().dwt2_adj(*args)


def dwt2_fwd_noalloc(*args) -> int:
    return lib().dwt2_fwd_noalloc(*args)


def dwt2_kernel_config(index: int):
    """(status, algorithm, waves, rows, core_cols, core_rows) of a kernel configuration."""
    v = [ctypes.c_int(0) for _ in range(5)]
    st = lib().dwt2_kernel_config(index, *[ctypes.byref(x) for x in v])
    return (st, *[x.value for x in v])


def status_string(status: int) -> str:
    return lib().dwt2_status_string(status).decode()


# ---- tensor-level API -----------------------------------------------------

def _torch():
    import torch
    return torch


_dtype_codes = None


def dtype_code(t) -> int:
    global _dtype_codes
    if _dtype_codes is None:
        torch = _torch()
        _dtype_codes = {torch.float32: DWT2_F32, torch.bfloat16: DWT2_BF16,
                        torch.float16: DWT2_F16, torch.int32: DWT2_I32}
    code = _dtype_codes.get(t.dtype)
    if code is None:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return code


def _check(x):
    if not x.is_cuda:
        raise RuntimeError("dwt2 runs on the GPU only: move the tensor to a HIP device")
    if x.dim() < 2:
        raise ValueError("expected a tensor [..., H, W]")
    if x.stride(-1) != 1:
        raise ValueError("the last dimension must be contiguous")


def _stream_ptr(x):
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)   # the current stream's handle, without a Stream object
    if raw is not None:
        return ctypes.c_void_p(raw(x.device.index))
    return ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)


def workspace(h: int, w: int, levels: int, dtype, device, planes: int = 1):
    """A workspace tensor for one call on `planes` h x w images (None if not needed)."""
    if levels == 1:
        return None                       # one level keeps no intermediate LL band
    torch = _torch()
    n = ctypes.c_size_t(0)
    st = lib().dwt2_workspace_bytes_planes(h, w, levels, dtype, planes, ctypes.byref(n))
    n = n.value
    if st != DWT2_OK:
        raise DWT2Error(st, "dwt2_workspace_bytes_planes")
    if n == 0:
        return None
    return torch.empty(n, dtype=torch.uint8, device=device)


_DTYPE_NAMES = {DWT2_F32: "f32", DWT2_BF16: "bf16", DWT2_F16: "f16", DWT2_I32: "i32"}
_DIRECTIONS = {"dwt2_fwd": "fwd", "dwt2_inv": "inv", "dwt2_adj": "adj"}


_tuned = {}


def tuned_config(direction: str, wavelet: str, dtype: int, h: int, w: int, levels: int):
    """Kernel configuration the autotuner recorded for this case, or None
    (looked up once per case and size class: small transforms are bound by
    the per-call host time)."""
    k0 = (direction, wavelet, dtype, h, w, levels)
    if k0 in _tuned:                      # this exact case seen before
        return _tuned[k0]
    from . import autotune
    k = (direction, wavelet, dtype, autotune.size_class(h, w), levels)
    if k not in _tuned:
        _tuned[k] = autotune.lookup(direction, wavelet, _DTYPE_NAMES[dtype], h, w, levels)
    _tuned[k0] = _tuned[k]
    return _tuned[k]


_supports = {}


def _config_ok(index: int, direction: str, wavelet: str, scheme: str) -> bool:
    k = (index, direction, wavelet, scheme)
    r = _supports.get(k)
    if r is None:
        r = _supports[k] = config_supports(index, direction, wavelet, scheme)
    return r


def config_supports(index: int, direction: str, wavelet: str, scheme: str = "fused") -> bool:
    """Whether kernel configuration `index` runs this case (the library
    rejects the others with DWT2_E_FLAGS): the LDS-plane configurations run
    the float wavelets forward and inverse with the fused, separable and
    polyconvolution schemes, and are the only ones that run DD 13/7 and the
    polyconvolution; the streaming ones run the fused and split schemes."""
    algo = dwt2_kernel_config(index)[1]
    if algo == DWT2_ALGO_LDS:
        return direction in ("fwd", "inv") and wavelet != "cdf53" and scheme in ("fused", "separable", "polyconv")
    if wavelet == "dd137" or scheme == "polyconv":
        return False
    if algo == DWT2_ALGO_STREAM:
        return scheme in ("fused", "split")
    return True


def workspace_status(ws) -> int:
    """dwt2_workspace_status of a workspace tensor after the call that used
    it has run: DWT2_OK, or DWT2_E_TIMEOUT if a dependency wait of the
    persistent forward ran out of time (its outputs are then invalid).
    Synchronises with the device (copies the status word to the host)."""
    head = bytes(ws[:DWT2_WORKSPACE_STATUS_BYTES].cpu().numpy().tobytes())
    return lib().dwt2_workspace_status(ctypes.c_char_p(head))


def _transform(fn, name, x, wavelet, levels, split, out, config=None, separable=False, factored=False,
               polyconv=False, persistent=False, ws=None, fused=False):
    torch = _torch()
    _check(x)
    if not x.is_contiguous():
        x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    else:
        _check(out)
        if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
            raise ValueError("out must match the input's shape, dtype and device")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
    result = out
    H, W = x.shape[-2], x.shape[-1]
    if x.dim() == 2:                      # one plane: no reshaped views (per-call host time)
        x2, planes = x, 1
    else:
        x2, out = x.reshape(-1, H, W), out.reshape(-1, H, W)
        planes = x2.shape[0]
    dt = dtype_code(x2)
    stream = _stream_ptr(x2)
    flags = ((DWT2_FLAG_SPLIT if split else 0) | (DWT2_FLAG_SEPARABLE if separable else 0)
             | (DWT2_FLAG_FACTORED if factored else 0) | (DWT2_FLAG_POLYCONV if polyconv else 0)
             | (DWT2_FLAG_PERSISTENT if persistent else 0) | (DWT2_FLAG_FUSED if fused else 0))
    if config is None:
        config = tuned_config(_DIRECTIONS[name], wavelet, dt, H, W, levels)
        scheme = ("split" if split else "separable" if separable else "factored" if factored
                  else "polyconv" if polyconv else "fused")
        if config is not None and not _config_ok(config, _DIRECTIONS[name], wavelet, scheme):
            config = None                 # the library's default for this case
    if config is not None:
        flags |= DWT2_FLAG_KERNEL(config)
    # one call for all planes (at most 2^31 - 1 per call)
    step = (1 << 31) - 1
    x_ptr, out_ptr, es = x2.data_ptr(), out.data_ptr(), x2.element_size()
    xp, op = x2.stride(-2), out.stride(-2)                 # pitches
    xs, os_ = (H * xp, H * op) if planes == 1 else (x2.stride(0), out.stride(0))
    for p0 in range(0, planes, step):
        n = min(step, planes - p0)
        w = ws if ws is not None else workspace(H, W, levels, dt, x2.device, n)
        ws_ptr = ctypes.c_void_p(w.data_ptr() if w is not None else 0)
        ws_n = w.numel() if w is not None else 0
        st = fn(ctypes.c_void_p(x_ptr + p0 * xs * es), ctypes.c_void_p(out_ptr + p0 * os_ * es), n, xs, os_,
                H, W, xp, op, dt, WAVELETS[wavelet], levels, DWT2_SYMMETRIC_WHOLE, flags, ws_ptr, ws_n, stream)
        if st != DWT2_OK:
            raise DWT2Error(st, name)
    return result


def fwd(x, wavelet: str = "cdf97", levels: int = 1, split: bool = False, out=None, config=None,
        separable: bool = False, factored: bool = False, polyconv: bool = False, persistent: bool = False,
        workspace=None, fused: bool = False):
    """Forward transform of every [H, W] plane of x into a Mallat pyramid
    (all planes in one call: one launch per level, or with `persistent` one
    persistent launch for every level).  `workspace`: a uint8 device tensor of at least
    dwt2_workspace_bytes_planes bytes to use instead of a fresh one (its
    status can be read with workspace_status afterwards).  `config` selects a
    kernel configuration index (None: tuned or library default).  At most
    one of `split` (the P0/P1 operation-count reduction), `separable` (the
    separable comparison scheme, twice the barriers), `factored` (each
    fused step evaluated as its two 1-D factors, one barrier per step) and
    `polyconv` (one polyconvolution step N_{P,U} per lifting pair, CDF 9/7,
    LDS-plane kernel); all compute the same values up to FP32 rounding.
    Wavelets: "cdf97", "cdf53" (reversible integer), "cdf53f" (real CDF
    5/3), "dd137" (Deslauriers-Dubuc 13/7, LDS-plane kernel)."""
    return _transform(lib().dwt2_fwd_planes, "dwt2_fwd", x, wavelet, levels, split, out, config, separable,
                      factored, polyconv, persistent, workspace, fused)


def inv(c, wavelet: str = "cdf97", levels: int = 1, split: bool = False, out=None, config=None,
        separable: bool = False, factored: bool = False, polyconv: bool = False, fused: bool = False):
    """Inverse transform of every [H, W] Mallat pyramid of c."""
    return _transform(lib().dwt2_inv_planes, "dwt2_inv", c, wavelet, levels, split, out, config, separable,
                      factored, polyconv, fused=fused)


def adj(g, levels: int = 1, out=None, config=None):
    """Adjoint W^T g of the CDF 9/7 forward transform (cotangent in Mallat layout)."""
    return _transform(lib().dwt2_adj_planes, "dwt2_adj", g, "cdf97", levels, False, out, config)


class dwt2_image(ctypes.Structure):
    """The C struct dwt2_image."""
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("src_pitch", ctypes.c_int64), ("dst_pitch", ctypes.c_int64)]


class BatchedForward:
    """One batched forward CDF 9/7 call over a list of [H, W] images.

    Holds the host and device descriptor arrays and the workspace, so that
    `run()` can be called repeatedly (or captured in a graph); `outs` are the
    Mallat pyramids, one per image."""

    def __init__(self, images, levels: int, split: bool = False, config=None, outs=None, persistent: bool = False):
        torch = _torch()
        if not images:
            raise ValueError("empty batch")
        for x in images:
            _check(x)
            if x.dim() != 2 or not x.is_contiguous():
                raise ValueError("every image must be a contiguous [H, W] tensor")
            if x.dtype != images[0].dtype or x.device != images[0].device:
                raise ValueError("images must share dtype and device")
        self.images = list(images)
        if outs is None:
            self.outs = [torch.empty_like(x) for x in images]
        else:
            # every pyramid is written through its data pointer and row pitch:
            # it must have its image's shape, dtype and device, and be contiguous
            self.outs = list(outs)
            if len(self.outs) != len(self.images):
                raise ValueError(f"{len(self.outs)} outputs for {len(self.images)} images")
            for k, (x, y) in enumerate(zip(self.images, self.outs)):
                _check(y)
                if y.shape != x.shape or y.dtype != x.dtype or y.device != x.device:
                    raise ValueError(f"outs[{k}] must match image {k} in shape, dtype and device")
                if not y.is_contiguous():
                    raise ValueError(f"outs[{k}] must be contiguous")
        self.levels = levels
        self.dtype = dtype_code(images[0])
        if config is None:
            from . import autotune
            config = autotune.load_cache().get(
                f"{autotune.arch_name()}|batched|cdf97|{_DTYPE_NAMES[self.dtype]}|any|5") \
                if autotune.load_cache() else None
        self.flags = ((DWT2_FLAG_SPLIT if split else 0) | (DWT2_FLAG_PERSISTENT if persistent else 0)
                      | (DWT2_FLAG_KERNEL(config) if config is not None else 0))
        n = len(images)
        self.host = (dwt2_image * n)()
        for i, (x, y) in enumerate(zip(self.images, self.outs)):
            self.host[i] = dwt2_image(x.data_ptr(), y.data_ptr(), x.shape[0], x.shape[1], x.stride(0), y.stride(0))
        raw = bytes(self.host)
        self.device = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(images[0].device)
        nbytes = ctypes.c_size_t(0)
        st = lib().dwt2_workspace_bytes_batched(ctypes.cast(self.host, ctypes.c_void_p), n, self.dtype, levels,
                                                ctypes.byref(nbytes))
        if st != DWT2_OK:
            raise DWT2Error(st, "dwt2_workspace_bytes_batched")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=images[0].device)

    def status(self) -> int:
        """dwt2_workspace_status of the last run (synchronises)."""
        return workspace_status(self.workspace)

    def run(self):
        st = lib().dwt2_fwd_batched(ctypes.cast(self.host, ctypes.c_void_p), ctypes.c_void_p(self.device.data_ptr()),
                                    len(self.images), self.dtype, DWT2_CDF97, self.levels, DWT2_SYMMETRIC_WHOLE,
                                    self.flags, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                    _stream_ptr(self.images[0]))
        if st != DWT2_OK:
            raise DWT2Error(st, "dwt2_fwd_batched")
        return self.outs


def fwd_batched(images, levels: int = 1, split: bool = False, config=None, outs=None, persistent: bool = False):
    """Forward CDF 9/7 of a list of [H, W] images of any sizes (a planner
    launch plus one launch per level, or with `persistent` one persistent
    launch for every level); returns the list of Mallat pyramids."""
    return BatchedForward(images, levels, split, config, outs, persistent).run()


def _make_function():
    torch = _torch()

    class DWT2Function(torch.autograd.Function):
        """Forward CDF 9/7 transform whose backward is the hand-written adjoint."""

        @staticmethod
        def forward(ctx, x, levels: int = 1):
            ctx.levels = levels
            return fwd(x.contiguous(), "cdf97", levels)

        @staticmethod
        def backward(ctx, g):
            return adj(g.contiguous(), ctx.levels), None

    return DWT2Function


_fn_cls = None


def DWT2Function():
    """The torch.autograd.Function class (created on first use)."""
    global _fn_cls
    if _fn_cls is None:
        _fn_cls = _make_function()
    return _fn_cls


def dwt2(x, levels: int = 1):
    """Differentiable forward CDF 9/7 transform of x [..., H, W] (FP32)."""
    return DWT2Function().apply(x, levels)
