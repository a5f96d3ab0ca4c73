"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the closed
form of the CDF filters, brute-force convolution, exact polynomial algebra,
the paper's Table 1 and appendix example, invariants (perfect reconstruction,
constant and polynomial images, shift covariance) and the transpose identity.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import fsolve

from oracle import adjoint, filterbank, lifting, nonsep, polymat, window

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_err(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------- P1 ------
@pytest.mark.parametrize("h", list(range(2, 25)) + [31, 40])
def test_perfect_reconstruction(h):
    rng = np.random.default_rng(h)
    for w in list(range(2, 25)) + [33, 40]:
        lv = lifting.max_levels(h, w)
        X = rng.random((h, w))
        for levels in sorted({1, lv}):
            for wav in ("cdf97", "cdf53f"):
                Y = lifting.fwd(X, wav, levels)
                assert np.abs(lifting.inv(Y, wav, levels) - X).max() < 1e-13
        Xi = rng.integers(-1000, 1000, (h, w))
        for levels in sorted({1, lv}):
            Yi = lifting.fwd(Xi, "cdf53", levels)
            assert np.array_equal(lifting.inv(Yi, "cdf53", levels), Xi)


# ---------------------------------------------------------------- P2 ------
@pytest.mark.parametrize("wav", ["cdf97", "cdf53f"])
def test_lifting_equals_closed_form_filter_bank_1d_sizes(wav):
    """One scale equals separable convolution with the closed-form filters on
    the symmetrically extended image, for every row/column length 2..39."""
    rng = np.random.default_rng(7)
    for n in range(2, 40):
        X = rng.random((2, n))
        assert rel_err(lifting.fwd(X, wav), filterbank.separable_bank(X, wav)) < 1e-13
        X = rng.random((n, 3))
        assert rel_err(lifting.fwd(X, wav), filterbank.separable_bank(X, wav)) < 1e-13


@pytest.mark.parametrize("shape", [(2, 2), (3, 2), (5, 9), (8, 8), (9, 13), (16, 18), (23, 17)])
def test_lifting_equals_nonseparable_convolution(shape):
    """Non-separable convolution N = N^V N^H with 9x9 / 9x7 / 7x9 / 7x7 2-D
    kernels (Section "Proposed Schemes") gives the same values; for CDF 5/3
    the kernels are 5x5 / 5x3 / 3x5 / 3x3."""
    X = np.random.default_rng(1).random(shape)
    Yn, shapes = filterbank.nonseparable_bank(X, "cdf97")
    assert shapes == {"LL": (9, 9), "HL": (9, 7), "LH": (7, 9), "HH": (7, 7)}
    assert rel_err(lifting.fwd(X, "cdf97"), Yn) < 1e-13
    Yn, shapes = filterbank.nonseparable_bank(X, "cdf53f")
    assert shapes == {"LL": (5, 5), "HL": (5, 3), "LH": (3, 5), "HH": (3, 3)}
    assert rel_err(lifting.fwd(X, "cdf53f"), Yn) < 1e-13


# ---------------------------------------------------------------- P3 ------
def _lifting_lowpass(a, b, c, d, z):
    """Low-pass impulse response (centred, 9 taps) of the lifting factorisation,
    computed on an impulse in a long zero signal (no borders involved)."""
    n = 64
    x = np.zeros(n)
    x[32] = 1.0                    # even sample at index 32 -> s[16]
    s, dd = x[0::2].copy(), x[1::2].copy()
    for p, u in ((a, b), (c, d)):
        dd += p * (s + np.roll(s, -1))
        s += u * (np.roll(dd, 1) + dd)
    s *= z
    # s[k] = response at even position 2k to the impulse at 32: h[32 - 2k]
    # low-pass taps h[j] for even j come from s; for odd j from a shifted impulse.
    return s, dd / z


def test_cdf97_constants_from_closed_form():
    """The lifting constants follow from the closed-form CDF 9/7 filters
    (roots of the Daubechies polynomial 20y^3 + 10y^2 + 4y + 1, which the
    paper does not print): solving the factorisation reproduces them."""
    h, g = filterbank.cdf_filters("cdf97")
    assert len(h) == 9 and len(g) == 7           # 9-tap / 7-tap (Section "Background")

    def taps(v):
        a, b, c, d, z = v
        # full 9-tap low-pass: run lifting on impulses at an even and an odd index
        out = np.zeros(9)
        for off in range(-4, 5):
            n = 64
            x = np.zeros(n)
            x[32 + off] = 1.0
            s, dd = x[0::2].copy(), x[1::2].copy()
            for p, u in ((a, b), (c, d)):
                dd += p * (s + np.roll(s, -1))
                s += u * (np.roll(dd, 1) + dd)
            out[off + 4] = z * s[16]
        return out

    def resid(v):
        return (taps(v) - h)[4:]               # symmetric: 5 independent taps

    sol = fsolve(resid, [-1.5, -0.06, 0.9, 0.45, 1.1], xtol=1e-14)
    lit = [lifting.ALPHA, lifting.BETA, lifting.GAMMA, lifting.DELTA, lifting.ZETA]
    assert np.abs(taps(sol) - h).max() < 1e-13
    assert np.abs(np.array(sol) - np.array(lit)).max() < 1e-11


def test_closed_form_filters_properties():
    h, g = filterbank.cdf_filters("cdf97")
    k = np.arange(-3, 4)
    for q in range(4):                            # 4 vanishing moments
        assert abs((g * k ** q).sum()) < 1e-13
    assert abs(h.sum() - math.sqrt(2)) < 1e-14
    assert abs((h * (-1.0) ** np.arange(-4, 5)).sum()) < 1e-14   # zero at Nyquist
    h53, g53 = filterbank.cdf_filters("cdf53")
    assert np.allclose(h53, [-1 / 8, 1 / 4, 3 / 4, 1 / 4, -1 / 8])
    assert np.allclose(g53, [-1 / 2, 1, -1 / 2])


# ---------------------------------------------------------------- P4/P5 ---
def test_constant_images():
    for shape in [(2, 2), (7, 5), (64, 66), (33, 17)]:
        c = 0.37
        X = np.full(shape, c)
        lv = lifting.max_levels(*shape)
        Y = lifting.fwd(X, "cdf97", lv)
        boxes = window.band_boxes(*shape, lv)
        for l, b, r0, r1, c0, c1 in boxes:
            blk = Y[r0:r1, c0:c1]
            if b == "LL":
                assert np.abs(blk - c * 2 ** lv).max() < 1e-12
            else:
                assert np.abs(blk).max() < 1e-12
        Yf = lifting.fwd(X, "cdf53f", lv)
        for l, b, r0, r1, c0, c1 in boxes:
            blk = Yf[r0:r1, c0:c1]
            assert np.abs(blk - (c * 2 ** lv if b == "LL" else 0.0)).max() < 1e-12
        Xi = np.full(shape, 77)
        Yi = lifting.fwd(Xi, "cdf53", lv)
        for l, b, r0, r1, c0, c1 in boxes:
            blk = Yi[r0:r1, c0:c1]
            assert np.all(blk == (77 if b == "LL" else 0))


def test_polynomial_images_cdf97():
    """Images of degree <= 3 in each axis have zero details away from borders."""
    H, W = 64, 72
    i = np.arange(H)[:, None] / H
    j = np.arange(W)[None, :] / W
    X = 1 + 2 * i - 3 * i ** 2 + 0.5 * i ** 3 + j ** 3 - 0.7 * j + i * j ** 2 + (i ** 3) * (j ** 3)
    Y = lifting.fwd(X, "cdf97", 1)
    he, we = H // 2, W // 2
    m = 3   # interior: more than 4 pixels from each border
    for blk in (Y[m:he - m, we + m:W - m], Y[he + m:H - m, m:we - m], Y[he + m:H - m, we + m:W - m]):
        assert np.abs(blk).max() < 1e-12
    # a degree-4 term is not annihilated (the pin is sharp)
    Y4 = lifting.fwd(X + i ** 4, "cdf97", 1)
    assert np.abs(Y4[he + m:H - m, m:we - m]).max() > 1e-9


def test_linear_images_cdf53f():
    """Real CDF 5/3 (2 vanishing moments): images of degree <= 1 in each axis
    have zero details away from borders; a quadratic term is not annihilated."""
    H, W = 40, 46
    i = np.arange(H)[:, None] / H
    j = np.arange(W)[None, :] / W
    X = 0.3 + 1.7 * i - 0.9 * j + 2.5 * i * j
    Y = lifting.fwd(X, "cdf53f", 1)
    he, we = H // 2, W // 2
    m = 2
    for blk in (Y[m:he - m, we + m:W - m], Y[he + m:H - m, m:we - m], Y[he + m:H - m, we + m:W - m]):
        assert np.abs(blk).max() < 1e-13
    # LL away from the border: the image at even samples, times zeta^2 = 2,
    # plus the update's zero contribution
    assert np.abs(Y[m:he - m, m:we - m] - 2 * X[0::2, 0::2][m:he - m, m:we - m]).max() < 1e-13
    Y2 = lifting.fwd(X + i ** 2, "cdf53f", 1)
    assert np.abs(Y2[he + m:H - m, m:we - m]).max() > 1e-6


def test_real_53_constants_and_filters():
    """p = -1/2, u = 1/4, zeta = sqrt(2): the closed-form 5/3 pair with the
    CDF 9/7 normalisation (both low-pass filters of DC gain sqrt(2))."""
    h, g = filterbank.cdf_filters("cdf53f")
    r2 = math.sqrt(2.0)
    assert np.abs(h - r2 * np.array([-1, 2, 6, 2, -1]) / 8).max() < 1e-15
    assert np.abs(g - np.array([-1, 2, -1]) / (2 * r2)).max() < 1e-15
    assert lifting.lifting_pairs("cdf53f") == [(-0.5, 0.25)]
    assert abs(lifting.zeta("cdf53f") - r2) < 1e-15


def test_bilinear_integer_images_cdf53():
    H, W = 40, 46
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    X = 5 + 3 * i - 2 * j + i * j
    Y = lifting.fwd(X, "cdf53", 1)
    he, we = H // 2, W // 2
    m = 2
    assert np.all(Y[m:he - m, we + m:W - m] == 0)
    assert np.all(Y[he + m:H - m, m:we - m] == 0)
    assert np.all(Y[he + m:H - m, we + m:W - m] == 0)
    assert np.array_equal(Y[m:he - m, m:we - m], X[0::2, 0::2][m:he - m, m:we - m])


# ---------------------------------------------------------------- 5/3 ----
def test_integer_53_within_rounding_bound_of_real_53():
    """The reversible 5/3 equals the real-valued CDF 5/3 filter bank up to its
    floors.  Propagating the floor errors through the step order T^H, T^V,
    S^H, S^V bounds (int - real) per subband of one scale by
    LL [-3/4, 2], HL [-1/2, 3/2], LH [-1/2, 3/2], HH [-1/2, 1]."""
    rng = np.random.default_rng(11)
    bounds = {"LL": (-0.75, 2.0), "HL": (-0.5, 1.5), "LH": (-0.5, 1.5), "HH": (-0.5, 1.0)}
    seen = {k: [np.inf, -np.inf] for k in bounds}
    for shape in [(2, 2), (3, 5), (16, 18), (33, 31), (64, 64)]:
        for _ in range(4):
            X = rng.integers(-2000, 2000, shape)
            D = lifting.fwd(X, "cdf53", 1) - filterbank.separable_bank(X, "cdf53")
            for _, b, r0, r1, c0, c1 in window.band_boxes(*shape, 1):
                blk = D[r0:r1, c0:c1]
                lo, hi = bounds[b]
                assert blk.min() >= lo - 1e-9 and blk.max() <= hi + 1e-9, b
                seen[b][0] = min(seen[b][0], blk.min())
                seen[b][1] = max(seen[b][1], blk.max())
    # the bound is not vacuous: the rounding errors do reach well into it
    assert seen["LL"][1] > 1.0 and seen["HH"][0] < -0.2


def test_appendix_predict_example():
    with open(os.path.join(GOLDEN, "appendix_predict.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    even = np.array([[int(v) for v in rows[0]]] * 2)
    expect = np.array([int(v) for v in rows[1]])
    odd = np.zeros_like(even)
    lifting._predict(even, odd, None, lifting.H_AXIS, integer=True)
    assert np.array_equal(odd[0], expect)
    # the same weights in the real-valued closed form: g = (-1/2, 1, -1/2)
    _, g = filterbank.cdf_filters("cdf53")
    assert g[0] == g[2] == -0.5


# ---------------------------------------------------------------- P6 ------
@pytest.mark.parametrize("shape", [(2, 2), (2, 3), (3, 2), (6, 8), (7, 9), (33, 66), (128, 130)])
def test_separable_equals_nonseparable(shape):
    """Section "Proposed Schemes": the fused non-separable steps (plain and
    with the P0/P1 split of Section "Optimization Approach") reach exactly the
    coefficients of the separable lifting scheme; pinned here to FP64
    rounding for the real wavelets and bit for bit for the integer 5/3."""
    rng = np.random.default_rng(3)
    X = rng.random(shape)
    ref = lifting.fwd(X, "cdf97", 1)
    assert rel_err(nonsep.nonsep_fwd_level(X, "cdf97"), ref) < 1e-14
    assert rel_err(nonsep.nonsep_fwd_level(X, "cdf97", split_consts=True), ref) < 1e-14
    Xi = rng.integers(-300, 300, shape)
    assert np.array_equal(nonsep.nonsep_fwd_level(Xi, "cdf53"), lifting.fwd(Xi, "cdf53", 1))
    ref = lifting.fwd(X, "cdf53f", 1)
    assert rel_err(nonsep.nonsep_fwd_level(X, "cdf53f"), ref) < 1e-14
    assert rel_err(nonsep.nonsep_fwd_level(X, "cdf53f", split_consts=True), ref) < 1e-14


def test_separable_equals_nonseparable_int_all_small_shapes():
    rng = np.random.default_rng(5)
    for h in range(2, 15):
        for w in range(2, 15):
            Xi = rng.integers(-300, 300, (h, w))
            assert np.array_equal(nonsep.nonsep_fwd_level(Xi, "cdf53"), lifting.fwd(Xi, "cdf53", 1))


# ---------------------------------------------------------------- P7 ------
def _rand_poly(rng, nterms):
    from fractions import Fraction
    return polymat.horizontal([(int(rng.integers(-3, 4)), Fraction(int(rng.integers(-9, 10)), int(rng.integers(1, 9))))
                               for _ in range(nterms)])


def test_symbolic_identities():
    rng = np.random.default_rng(0)
    for _ in range(5):
        P, U = _rand_poly(rng, 3), _rand_poly(rng, 3)
        assert polymat.equal(polymat.T_fused(P), polymat.matmul(polymat.T_V(P), polymat.T_H(P)))
        assert polymat.equal(polymat.S_fused(U), polymat.matmul(polymat.S_V(U), polymat.S_H(U)))
        assert polymat.equal(polymat.N_polyconv(P, U),
                             polymat.matmul(polymat.S_fused(U), polymat.T_fused(P)))
        # the split P = P0 + P1: T_P = T_{P1} T_{P0}^V T_{P0}^H
        P0, P1 = polymat.split_constant(P)
        lhs = polymat.T_fused(P)
        rhs = polymat.matmul(polymat.T_fused(P1), polymat.matmul(polymat.T_V(P0), polymat.T_H(P0)))
        assert polymat.equal(lhs, rhs)
    # a transposed operand breaks the identity (the check is sharp)
    P = _rand_poly(rng, 3)
    bad = polymat.T_fused(polymat.star(P))
    assert not polymat.equal(bad, polymat.matmul(polymat.T_V(P), polymat.T_H(P)))


# ---------------------------------------------------------------- P8 ------
def test_table1_counts():
    with open(os.path.join(GOLDEN, "table1_lifting.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for wav, scheme, steps, ops in rows:
        if scheme == "nonseparable-lifting":
            scheme = "nonseparable-lifting-optimized"
        assert polymat.count(scheme, wav) == (int(steps), int(ops)), (wav, scheme)
    # without the optimisation the fused scheme needs more operations
    assert polymat.count("nonseparable-lifting", "cdf97") == (4, 48)
    # every scheme is the same transform
    for wav in ("cdf53", "cdf97", "dd137"):
        ref = polymat.product(polymat.scheme_steps("separable-lifting", wav))
        for s in ("nonseparable-lifting", "nonseparable-lifting-optimized"):
            assert polymat.equal(polymat.product(polymat.scheme_steps(s, wav)), ref)


# ---------------------------------------------------------------- P10 -----
def _dense_forward(h, w, levels):
    n = h * w
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = lifting.fwd(e.reshape(h, w), "cdf97", levels).ravel()
    return M


@pytest.mark.parametrize("shape,levels", [((8, 8), 1), ((9, 7), 2), ((16, 18), 3), ((5, 12), 2)])
def test_adjoint_is_dense_transpose(shape, levels):
    h, w = shape
    M = _dense_forward(h, w, levels)
    n = h * w
    MT = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        MT[:, k] = adjoint.adj(e.reshape(h, w), "cdf97", levels).ravel()
    assert np.abs(MT - M.T).max() < 1e-12
    # and W^T is not W^-1 (biorthogonal): the borders matter
    assert np.abs(np.linalg.inv(M) - M.T).max() > 0.1


def test_adjoint_dot_product():
    rng = np.random.default_rng(2)
    for shape, lv in [((64, 66), 3), ((33, 17), 2), ((128, 128), 5)]:
        x = rng.standard_normal(shape)
        y = rng.standard_normal(shape)
        lhs = np.vdot(lifting.fwd(x, "cdf97", lv), y)
        rhs = np.vdot(x, adjoint.adj(y, "cdf97", lv))
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_matrix_form_equals_definition():
    X = np.random.default_rng(4).random((13, 10))
    assert rel_err(adjoint._fwd_level_matrix_form(X, "cdf97"), lifting.fwd(X, "cdf97", 1)) < 1e-14


# ---------------------------------------------------------------- P11 -----
def test_shift_covariance():
    """Shifting the image by 2 pixels shifts every subband by 1 coefficient
    (away from the borders)."""
    rng = np.random.default_rng(9)
    X = rng.random((64, 80))
    A = lifting.fwd(X, "cdf97", 1)
    B = lifting.fwd(X[2:, 2:], "cdf97", 1)
    m = 4
    for (_, b, ar0, ar1, ac0, ac1), (_, b2, br0, br1, bc0, bc1) in zip(
            window.band_boxes(64, 80, 1), window.band_boxes(62, 78, 1)):
        a = A[ar0:ar1, ac0:ac1][1:, 1:]
        bb = B[br0:br1, bc0:bc1]
        n, k = min(a.shape[0], bb.shape[0]), min(a.shape[1], bb.shape[1])
        assert np.abs(a[m:n - m, m:k - m] - bb[m:n - m, m:k - m]).max() < 1e-12, b


# ---------------------------------------------------------------- S13 -----
def test_multilevel_is_recursive_on_ll():
    rng = np.random.default_rng(6)
    X = rng.random((66, 130))
    Y3 = lifting.fwd(X, "cdf97", 3)
    Y1 = lifting.fwd(X, "cdf97", 1)
    LL1 = Y1[:33, :65]
    Y2sub = lifting.fwd(LL1, "cdf97", 2)
    assert np.array_equal(Y3[:33, :65], Y2sub)
    assert np.array_equal(Y3[33:, :], Y1[33:, :]) and np.array_equal(Y3[:33, 65:], Y1[:33, 65:])


# ---------------------------------------------------------------- window --
@pytest.mark.parametrize("wav,levels", [("cdf97", 3), ("cdf53", 2), ("cdf97", 1), ("cdf53f", 3)])
def test_crop_window_matches_full_oracle(wav, levels):
    H, W = 352, 416
    rng = np.random.default_rng(8)
    X = rng.integers(0, 256, (H, W)) if wav == "cdf53" else rng.random((H, W))
    Y = lifting.fwd(X, wav, levels)
    for r0, r1, c0, c1 in window.probe_crops(H, W, levels, size=64):
        sub = lifting.fwd(X[r0:r1, c0:c1], wav, levels)
        cut = window.crop_pyramid(Y, levels, r0, r1, c0, c1)
        mask = window.crop_valid_mask(H, W, levels, r0, r1, c0, c1, window.default_margin(levels))
        assert mask.sum() > 0
        assert np.abs(sub[mask] - cut[mask]).max() < 1e-12
        Xb = lifting.inv(cut, wav, levels)
        # inverse windows: the image interior of the crop is reproduced
        assert np.abs(Xb[mask_interior(H, W, r0, r1, c0, c1, window.default_margin(levels))]
                      - X[r0:r1, c0:c1][mask_interior(H, W, r0, r1, c0, c1, window.default_margin(levels))]).max() < 1e-10


def mask_interior(H, W, r0, r1, c0, c1, m):
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    okr = np.ones(len(rows), bool)
    okc = np.ones(len(cols), bool)
    if r0 > 0:
        okr &= rows - r0 >= m
    if r1 < H:
        okr &= r1 - rows >= m
    if c0 > 0:
        okc &= cols - c0 >= m
    if c1 < W:
        okc &= c1 - cols >= m
    return np.outer(okr, okc)


# ------------------------------------------------- DD 13/7 (Section "Evaluation")
@pytest.mark.parametrize("h", [2, 3, 4, 5, 7, 9, 12, 17, 24, 31, 40])
def test_dd137_perfect_reconstruction(h):
    rng = np.random.default_rng(100 + h)
    for w in [2, 3, 4, 6, 7, 11, 16, 25, 33, 40]:
        X = rng.random((h, w))
        for levels in sorted({1, lifting.max_levels(h, w)}):
            Y = lifting.fwd(X, "dd137", levels)
            assert np.abs(lifting.inv(Y, "dd137", levels) - X).max() < 1e-13


def test_dd137_closed_form_filters():
    """The analysis pair derived without lifting (synthesis low-pass = the
    4-point Deslauriers-Dubuc interpolator c^2 (1 + 2y); analysis low-pass =
    the symmetric 13-tap solution of the biorthogonality conditions) is the
    published 13/7 pair: h = (-1, 0, 18, -16, -63, 144, 348, ...) / 512 and
    g = (1, 0, -9, 16, -9, 0, 1) / 16, each scaled by the DC-gain rule."""
    h, g = filterbank.cdf_filters("dd137")
    z = lifting.ZETA137
    assert z == pytest.approx(math.sqrt(2.0), abs=1e-15)
    hh = np.array([-1, 0, 18, -16, -63, 144, 348, 144, -63, -16, 18, 0, -1]) / 512.0
    gg = np.array([1, 0, -9, 16, -9, 0, 1]) / 16.0
    assert np.abs(h - z * hh).max() < 1e-14
    assert np.abs(g - gg / z).max() < 1e-14
    # the product of the analysis and synthesis low-pass filters is half-band
    f0 = np.abs(gg) * np.array([-1, 1, 1, 1, 1, 1, -1])
    prod = np.convolve(hh, f0)
    c = (len(prod) - 1) // 2
    even = [prod[c + k] for k in range(-c, c + 1) if k % 2 == 0 and k != 0]
    assert np.abs(even).max() < 1e-15 and prod[c] == pytest.approx(1.0)


def test_dd137_lifting_equals_closed_form_filter_bank():
    """One DD 13/7 scale equals separable convolution with the closed-form
    13/7 filters on the symmetrically extended image, for every length 2..39
    (the 4-tap steps read two samples across a border: the extension is a
    reflection of the pixel position, not a clamp of the component index)."""
    rng = np.random.default_rng(8)
    for n in range(2, 40):
        X = rng.random((2, n))
        assert rel_err(lifting.fwd(X, "dd137"), filterbank.separable_bank(X, "dd137")) < 1e-13
        X = rng.random((n, 3))
        assert rel_err(lifting.fwd(X, "dd137"), filterbank.separable_bank(X, "dd137")) < 1e-13


def test_dd137_constant_and_polynomial_images():
    """Constant images: LL = 2c per level, no detail anywhere.  Images of
    degree <= 3 in each axis (the 4-point interpolating predict is exact for
    cubics): zero details more than 6 pixels from the borders; a degree-4
    term is not annihilated (the pin is sharp)."""
    X = np.full((40, 46), 0.75)
    Y = lifting.fwd(X, "dd137", 3)
    for lv, b, r0, r1, c0, c1 in window.band_boxes(40, 46, 3):
        blk = Y[r0:r1, c0:c1]
        assert np.abs(blk - (0.75 * 8 if b == "LL" else 0.0)).max() < 1e-13
    H, W = 72, 80
    i = np.arange(H)[:, None] / H
    j = np.arange(W)[None, :] / W
    X = 1 + 2 * i - 3 * i ** 2 + 0.5 * i ** 3 + j ** 3 - 0.7 * j + i * j ** 2 + (i ** 3) * (j ** 3)
    Y = lifting.fwd(X, "dd137", 1)
    he, we = H // 2, W // 2
    m = 4
    for blk in (Y[m:he - m, we + m:W - m], Y[he + m:H - m, m:we - m], Y[he + m:H - m, we + m:W - m]):
        assert np.abs(blk).max() < 1e-12
    Y4 = lifting.fwd(X + j ** 4, "dd137", 1)
    assert np.abs(Y4[m:he - m, we + m:W - m]).max() > 1e-9


# ------------------------------------ non-separable polyconvolution N_{P,U}
@pytest.mark.parametrize("wav", ["cdf97", "cdf53f", "dd137"])
def test_matrix_schemes_equal_separable(wav):
    """Section "Proposed Schemes": one polyconvolution step N_{P,U} per
    lifting pair, and the fused steps T_P, S_U (for DD 13/7 with 4-tap
    filters), evaluated on the symmetrically extended image, reach the
    separable lifting's coefficients (FP64 rounding), on shapes with odd and
    even sides down to 2 x 2; the inverse polyconvolution restores the image."""
    rng = np.random.default_rng(9)
    for h in (2, 3, 4, 5, 8, 13, 21, 34):
        for w in (2, 3, 6, 7, 16, 19, 30):
            X = rng.random((h, w))
            ref = lifting.fwd_level(X, wav)
            assert rel_err(nonsep.matrix_scheme_fwd_level(X, wav, "polyconv"), ref) < 1e-14
            assert rel_err(nonsep.matrix_scheme_fwd_level(X, wav, "fused"), ref) < 1e-14
            assert np.abs(nonsep.matrix_scheme_inv_level(ref, wav) - X).max() < 1e-13
    X = rng.random((67, 130))
    lv = 5
    ref = lifting.fwd(X, wav, lv)
    assert rel_err(nonsep.polyconv_fwd(X, wav, lv), ref) < 1e-14
    assert np.abs(nonsep.polyconv_inv(ref, wav, lv) - X).max() < 1e-12


def test_polyconv_matrix_equals_symbolic_product():
    """The numeric N_{P,U} used by the oracle equals the exact symbolic
    product S_U T_P (polymat, with V = P U + 1) for both CDF 9/7 pairs and
    the CDF 5/3 pair: every entry, as a 2-D kernel."""
    from fractions import Fraction
    for wav in ("cdf97", "cdf53f"):
        for (P, U), (p, u) in zip(lifting.lifting_taps(wav), lifting.lifting_pairs(wav)):
            Ps = polymat.horizontal([(0, Fraction(p)), (1, Fraction(p))])
            Us = polymat.horizontal([(0, Fraction(u)), (-1, Fraction(u))])
            exact = polymat.matmul(polymat.S_fused(Us), polymat.T_fused(Ps))
            assert polymat.equal(exact, polymat.N_polyconv(Ps, Us))
            M = nonsep.polyconv_matrix(P, U)
            for r in range(4):
                for c in range(4):
                    vt, ht = M[r][c]
                    num = {}
                    for i, a in vt.items():
                        for j, b in ht.items():
                            num[(j, i)] = num.get((j, i), 0.0) + a * b
                    num = {k: v for k, v in num.items() if v != 0.0}
                    sym = {k: float(v) for k, v in exact[r][c].items()}
                    assert set(num) == set(sym), (wav, r, c)
                    assert max(abs(num[k] - sym[k]) for k in sym) < 1e-15


def test_polyconv_pixel_footprints():
    """For the CDF wavelets one polyconvolution step reads, per output
    component, a pixel footprint of 5 x 5 (LL), 5 x 3 (HL), 3 x 5 (LH) and
    3 x 3 (HH) samples (rows x columns), the filter sizes Section "Proposed
    Schemes" gives for N_{P,U}."""
    (P, U), _ = lifting.lifting_taps("cdf97")
    M = nonsep.polyconv_matrix(P, U)
    for c, want in zip(range(4), [(5, 5), (5, 3), (3, 5), (3, 3)]):
        rows, cols = set(), set()
        for k in range(4):
            vt, ht = M[c][k]
            # input component k = (row parity, column parity) at block offset
            # (i, j) sits at pixel offset (2 i + pk - pc) from the output pixel
            for i in vt:
                rows.add(2 * i + (k >> 1) - (c >> 1))
            for j in ht:
                cols.add(2 * j + (k & 1) - (c & 1))
        assert (max(rows) - min(rows) + 1, max(cols) - min(cols) + 1) == want
        assert rows == set(range(min(rows), max(rows) + 1)) and cols == set(range(min(cols), max(cols) + 1))
