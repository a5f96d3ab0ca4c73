"""Batched forward transform over many uneven images, with one launch per
level (default) and with one persistent launch for every level.

Every image of the batch must equal the single-image dwt2_fwd on that image
bit for bit (same kernel configuration: the same tile arithmetic), every
persistent call must report no timed-out dependency wait, and a sample of
images is also checked against the CPU oracle.  The call is then
captured in a graph and replayed several times, with eager work and
synchronisations in between, each replay checked against the eager result.
"""
import numpy as np
import pytest

import workloads
from oracle import lifting

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def uneven(count, lo, hi, seed, odd=False):
    shapes = workloads.uneven_shapes(count, lo, hi, seed)
    if odd:  # make some sizes odd as well
        shapes = [(h - (i % 2), w - ((i // 2) % 2)) for i, (h, w) in enumerate(shapes)]
    rng = np.random.default_rng(seed)
    return shapes, [rng.random(s, dtype=np.float32) for s in shapes]


def checked(call):
    """Run a batched call; a persistent one must report no timed-out wait."""
    print(f"batched call: {len(call.images)} images, levels {call.levels}, flags {call.flags:#x}", flush=True)
    outs = call.run()
    if call.flags & d.DWT2_FLAG_PERSISTENT:
        assert call.status() == d.DWT2_OK
    return outs


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("tdt", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("config", [0, 1, 2])
def test_batched_equals_single(tdt, config, persistent):
    shapes, imgs = uneven(24, 64, 700, seed=1, odd=True)
    xs = [torch.from_numpy(x).to(dev()).to(tdt) for x in imgs]
    lv = min(5, min(lifting.max_levels(*s) for s in shapes))
    outs = checked(d.BatchedForward(xs, lv, config=config, persistent=persistent))
    for x, y in zip(xs, outs):
        ref = d.fwd(x, "cdf97", lv, config=config)
        assert torch.equal(y, ref)


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_split_and_oracle(persistent):
    shapes, imgs = uneven(10, 64, 1500, seed=3)
    xs = [torch.from_numpy(x).to(dev()) for x in imgs]
    outs = checked(d.BatchedForward(xs, 5, split=True, persistent=persistent))
    for k in (0, 3, 7):
        ref = lifting.fwd(imgs[k], "cdf97", 5)
        got = outs[k].double().cpu().numpy()
        assert np.abs(got - ref).max() / np.abs(ref).max() <= 1e-5


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_many_small_images(persistent):
    xs = [torch.from_numpy(x).to(dev()) for x in workloads.planes(1024, 256, 256, seed=2)]
    outs = checked(d.BatchedForward(xs, 5, persistent=persistent))
    for k in (0, 511, 1023):
        assert torch.equal(outs[k], d.fwd(xs[k], "cdf97", 5))


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_thousands_of_tiny_images(persistent):
    # 5000 images of 8..40 pixels: finding a tile's image takes three passes
    # of the 64-entry search (more than 4096 images), and every image is a
    # single border tile
    shapes, imgs = uneven(5000, 8, 40, seed=11, odd=True)
    xs = [torch.from_numpy(x).to(dev()) for x in imgs]
    lv = min(2, min(lifting.max_levels(*s) for s in shapes))
    outs = checked(d.BatchedForward(xs, lv, persistent=persistent))
    for x, y in zip(xs, outs):
        assert torch.equal(y, d.fwd(x, "cdf97", lv))


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_graph_replay(persistent):
    shapes, imgs = uneven(16, 64, 900, seed=5)
    xs = [torch.from_numpy(x).to(dev()) for x in imgs]
    call = d.BatchedForward(xs, 4, persistent=persistent)
    call.run()
    torch.cuda.synchronize()
    eager = [y.clone() for y in call.outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        call.run()                        # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        call.run()
    for rep in range(4):
        for y in call.outs:
            y.fill_(float("nan"))         # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if persistent:
            assert call.status() == d.DWT2_OK
        for y, e in zip(call.outs, eager):
            assert torch.equal(y, e), rep
    