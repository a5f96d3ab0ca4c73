"""Differentiation through the hand-written adjoint (torch.autograd.Function).

Workload: batch x 3 x H x W FP32 images, 3-level CDF 9/7 forward, loss
    L = sum over levels of sum |HL| + |LH| + |HH|  +  mean((LL_3 - target)^2)
(sign(0) = 0), target seeded uniform [0, 1) of LL_3's shape.

Checks: (1) x.grad equals the oracle's transpose W^T applied to the same
upstream gradient (computed from the GPU coefficients), image 0, all
channels, within 1e-5 relative max-abs; (2) central finite differences with
eps = 1e-3 on a 64 x 64 crop (top-left of image 0, channel 0, transformed as
its own image) at 256 sampled pixels (corners, edges, interior).  The
difference quotient is accumulated per coefficient in FP64,
sum_j [l_j(c_j + eps d_j) - l_j(c_j - eps d_j)] / (2 eps) with d = W e_k
from the GPU forward transform of the unit impulse, so no FP32 cancellation
enters; pixels whose perturbation moves a detail coefficient across 0 (the
kink of |.|) are skipped.  Tolerance 1e-3 relative + 1e-4 absolute.
"""
import numpy as np
import pytest

import workloads
from oracle import adjoint, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1704_08657_amd as d  # noqa: E402

LEVELS = 3


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def detail_mask(h, w, levels):
    m = np.ones((h, w), dtype=bool)
    for lv, b, r0, r1, c0, c1 in window.band_boxes(h, w, levels):
        if b == "LL":
            m[r0:r1, c0:c1] = False
    return m


def ll_box(h, w, levels):
    for lv, b, r0, r1, c0, c1 in window.band_boxes(h, w, levels):
        if b == "LL":
            return r0, r1, c0, c1


def loss_torch(c, target, mask):
    r0, r1, c0, c1 = ll_box(c.shape[-2], c.shape[-1], LEVELS)
    det = (c.abs() * mask).sum()
    ll = c[..., r0:r1, c0:c1]
    return det + ((ll - target) ** 2).mean()


@pytest.mark.parametrize("shape", [(2, 3, 256, 256), (64, 3, 1024, 1024)])
def test_grad_equals_oracle_transpose(shape):
    B, C, H, W = shape
    x = torch.from_numpy(workloads.planes(B * C, H, W, seed=4).reshape(shape)).to(dev())
    x.requires_grad_(True)
    r0, r1, c0, c1 = ll_box(H, W, LEVELS)
    target = torch.from_numpy(np.random.default_rng(5).random((r1 - r0, c1 - c0), dtype=np.float32)).to(dev())
    mask = torch.from_numpy(detail_mask(H, W, LEVELS)).to(dev())
    c = d.dwt2(x, LEVELS)
    L = loss_torch(c, target, mask)
    L.backward()
    # upstream gradient dL/dc from the GPU coefficients, image 0
    cn = c.detach()[0].double().cpu().numpy()
    g = np.sign(cn) * mask.cpu().numpy()
    n = B * C * (r1 - r0) * (c1 - c0)
    g[:, r0:r1, c0:c1] = 2.0 * (cn[:, r0:r1, c0:c1] - target.double().cpu().numpy()) / n
    got = x.grad[0].double().cpu().numpy()
    for ch in range(C):
        ref = adjoint.adj(g[ch], "cdf97", LEVELS)
        err = np.abs(got[ch] - ref).max() / np.abs(ref).max()
        assert err <= 1e-5, (ch, err)


def test_grad_matches_central_differences():
    H = W = 64
    # image 0, channel 0 of the batch drawn by workloads.planes(.., seed=4):
    # its first plane is the first 1024 x 1024 draws of that generator
    x0 = workloads.uniform(1024, 1024, seed=4)[:H, :W].copy()
    r0, r1, c0, c1 = ll_box(H, W, LEVELS)
    target = np.random.default_rng(5).random((r1 - r0, c1 - c0))
    mask = detail_mask(H, W, LEVELS)
    n_ll = (r1 - r0) * (c1 - c0)

    xt = torch.from_numpy(x0).to(dev()).requires_grad_(True)
    c = d.dwt2(xt, LEVELS)
    L = loss_torch(c, torch.from_numpy(target.astype(np.float32)).to(dev()), torch.from_numpy(mask).to(dev()))
    L.backward()
    grad = xt.grad.double().cpu().numpy()
    cn = c.detach().double().cpu().numpy()

    def per_coeff_loss(cc):
        out = np.abs(cc) * mask
        ll = cc[r0:r1, c0:c1]
        out[r0:r1, c0:c1] = (ll - target) ** 2 / n_ll
        return out

    rng = np.random.default_rng(7)
    pts = {(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (0, W // 2), (H // 2, 0), (H - 1, 17), (23, W - 1)}
    while len(pts) < 256:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, W))))
    eps = 1e-3
    checked = 0
    for (i, j) in sorted(pts):
        e = torch.zeros(H, W, device=dev())
        e[i, j] = 1.0
        dk = d.fwd(e, "cdf97", LEVELS).double().cpu().numpy()
        plus, minus = cn + eps * dk, cn - eps * dk
        kink = mask & (np.sign(plus) != np.sign(minus)) & (dk != 0)
        if kink.any():
            continue
        fd = float((per_coeff_loss(plus) - per_coeff_loss(minus)).sum() / (2 * eps))
        assert abs(fd - grad[i, j]) <= 1e-3 * abs(fd) + 1e-4, ((i, j), fd, grad[i, j])
        checked += 1
    assert checked >= 128
