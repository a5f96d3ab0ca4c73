"""The persistent forward (DWT2_FLAG_PERSISTENT: every level in one launch
after a planner launch; tiles of level l >= 1 wait for the tiles of level
l - 1 they read): on one image and a plane stack it must equal the
one-launch-per-level path bit for bit (the same tile arithmetic on the same
values), report no timed-out wait, survive reuse of its workspace and graph
replay, and, with the wait limit forced to zero from the host, end normally
and report the failure.  (Batches: tests/test_gpu_batched.py.)"""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads
from oracle import lifting, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def ws_for(x, levels):
    h, w = x.shape[-2:]
    planes = int(np.prod(x.shape[:-2])) if x.dim() > 2 else 1
    return d.workspace(h, w, levels, d.dtype_code(x), x.device, planes)


def persistent(x, levels, **kw):
    """Forward on the persistent path with its own workspace; asserts the
    call reported no timed-out wait."""
    ws = ws_for(x, levels)                    # None for one level: no workspace, one launch
    print(f"persistent fwd {tuple(x.shape)} {x.dtype} levels={levels} {kw}", flush=True)
    y = d.fwd(x, "cdf97", levels, workspace=ws, persistent=True, **kw)
    torch.cuda.synchronize()
    if ws is not None:
        assert d.workspace_status(ws) == d.DWT2_OK
    return y


SHAPES = [(64, 64, 5), (66, 130, 5), (257, 131, 4), (700, 1500, 5), (1030, 998, 6), (2050, 1026, 3),
          (4096, 4094, 5), (8192, 8192, 5), (3, 4000, 1), (5, 9, 2)]


@pytest.mark.parametrize("h,w,levels", SHAPES)
@pytest.mark.parametrize("config", [0, 3])
def test_one_image_equals_level_launches(h, w, levels, config):
    x = torch.from_numpy(workloads.uniform(h, w, seed=h + w)).to(dev())
    levels = min(levels, lifting.max_levels(h, w))
    y = persistent(x, levels, config=config)
    r = d.fwd(x, "cdf97", levels, config=config)
    assert torch.equal(y, r)


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("split", [False, True])
def test_storage_types_and_split(tdt, split):
    x = torch.from_numpy(workloads.uniform(1500, 2000, seed=9)).to(dev()).to(tdt)
    y = persistent(x, 5, split=split)
    assert torch.equal(y, d.fwd(x, "cdf97", 5, split=split))


def test_plane_stack_equals_level_launches():
    x = torch.from_numpy(workloads.planes(12, 515, 333, seed=3)).to(dev()).reshape(3, 4, 515, 333)
    y = persistent(x, 4)
    assert torch.equal(y, d.fwd(x, "cdf97", 4))


def test_one_image_against_oracle_on_crops():
    """8192^2, 5 levels (the benchmark's multi-level form) on the persistent
    path against the FP64 oracle on probe crops (corners, edge midpoints,
    centre), over every coefficient whose footprint stays inside the crop."""
    x = workloads.uniform(8192, 8192, seed=0)
    y = persistent(torch.from_numpy(x).to(dev()), 5).double().cpu().numpy()
    m = window.default_margin(5)
    for r0, r1, c0, c1 in window.probe_crops(8192, 8192, 5, size=256):
        ref = lifting.fwd(x[r0:r1, c0:c1], "cdf97", 5)
        cut = window.crop_pyramid(y, 5, r0, r1, c0, c1)
        mask = window.crop_valid_mask(8192, 8192, 5, r0, r1, c0, c1, m)
        assert mask.sum() > 0
        assert np.abs(cut[mask] - ref[mask]).max() <= 1e-5 * np.abs(ref[mask]).max(), (r0, c0)


def test_workspace_reuse_and_graph_replay():
    x = torch.from_numpy(workloads.uniform(2048, 1536, seed=4)).to(dev())
    ws = ws_for(x, 5)
    out = torch.empty_like(x)
    ref = d.fwd(x, "cdf97", 5)
    for rep in range(3):                      # the planner clears the counters of the last call
        out.fill_(float("nan"))
        d.fwd(x, "cdf97", 5, out=out, workspace=ws, persistent=True)
        torch.cuda.synchronize()
        assert d.workspace_status(ws) == d.DWT2_OK
        assert torch.equal(out, ref), rep
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        d.fwd(x, "cdf97", 5, out=out, workspace=ws, persistent=True)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        d.fwd(x, "cdf97", 5, out=out, workspace=ws, persistent=True)
    for rep in range(4):
        out.fill_(float("nan"))               # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert d.workspace_status(ws) == d.DWT2_OK
        assert torch.equal(out, ref), rep


def test_failed_wait_is_reported_and_the_call_ends():
    """With the wait limit forced to 0 from the host, the first wait that
    finds its dependency unfinished gives up: the launch still ends, and the
    workspace reports DWT2_E_TIMEOUT.  Run in a child process, so that the
    environment variable stays out of this one; the next call there, with
    the default limit, is correct again."""
    code = r"""
import os, sys, torch
sys.path.insert(0, %r)
import paper_1704_08657_amd as d, workloads
x = torch.from_numpy(workloads.uniform(8192, 8192, seed=0)).cuda()
ws = d.workspace(8192, 8192, 5, d.DWT2_F32, x.device)
ref = d.fwd(x, "cdf97", 5)
os.environ["DWT2_WAIT_LIMIT_US"] = "0"
d.fwd(x, "cdf97", 5, workspace=ws, persistent=True)
torch.cuda.synchronize()
print("forced", d.workspace_status(ws), flush=True)
del os.environ["DWT2_WAIT_LIMIT_US"]
y = d.fwd(x, "cdf97", 5, workspace=ws, persistent=True)
torch.cuda.synchronize()
print("default", d.workspace_status(ws), bool(torch.equal(y, ref)), flush=True)
""" % ROOT
    print("child: forced wait limit 0 on 8192^2, 5 levels", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert f"forced {d.DWT2_E_TIMEOUT}" in r.stdout
    assert f"default {d.DWT2_OK} True" in r.stdout
