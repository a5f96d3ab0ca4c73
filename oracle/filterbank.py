"""Closed-form CDF filters and brute-force convolution filter banks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Background" describes the single-scale DWT as a pair of filters
G0, G1 followed by subsampling by two (Mallat), and the 2-D transform as the
tensor product of two 1-D transforms: the separable convolution scheme
N^V | N^H |, or in one step the non-separable convolution N = N^V N^H with 2-D
filters of 9x9, 7x9, 9x7 and 7x7 taps for CDF 9/7 (Section "Proposed
Schemes").  The lifting constants are not printed in the paper; this module
derives the filters independently of any lifting code, from the closed form
of the Cohen-Daubechies-Feauveau family:

    with  y = sin^2(w/2),  c = cos^2(w/2) = (2 + z + z^-1) / 4,
    the half-band condition (1-y)^N Q(y) + y^N Q(1-y) = 1 is solved by
        Q_N(y) = sum_{k<N} binom(N-1+k, k) y^k.
    CDF 9/7 (N = 4): analysis low-pass  ~ c^2 (y - y1)(y - conj(y1)),
                     synthesis low-pass ~ c^2 (y - y0),
    with y0 the real and y1, conj(y1) the complex roots of Q_4.
    CDF 5/3 (N = 2): analysis low-pass  ~ c Q_2(y) = c (1 + 2y),
                     synthesis low-pass ~ c.
    The analysis high-pass is the modulated synthesis low-pass,
        g[k] = (-1)^k f0[k].

Filters are returned as centred tap arrays (index k = -L..L).  The brute-force
banks evaluate every output sample as an explicit dot product with the
whole-point symmetric extension of the input, with no lifting involved.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as npoly


# --------------------------------------------------------------------------
# Laurent polynomials in z as centred coefficient arrays
# --------------------------------------------------------------------------

def _lp_mul(a, b):
    return np.convolve(a, b)


def _c_term():
    """cos^2(w/2) = (z^-1 + 2 + z) / 4 as centred taps."""
    return np.array([0.25, 0.5, 0.25])


def _y_minus(root):
    """y - root with y = sin^2(w/2) = (-z^-1 + 2 - z) / 4."""
    return np.array([-0.25, 0.5 - root, -0.25], dtype=complex)


def half_band_Q(N: int) -> np.ndarray:
    """Coefficients (ascending powers of y) of Q_N(y)."""
    return np.array([math.comb(N - 1 + k, k) for k in range(N)], dtype=float)


def cdf_filters(name: str):
    """(h, g): analysis low-pass h (centred on an even sample) and high-pass g
    (centred on an odd sample), normalised as the oracle's lifting form
    ("dd137": see dd137_filters):
    CDF 9/7 with DC gain sqrt(2) for both low-pass filters, "cdf53" (the real
    counterpart of the reversible integer transform, unscaled) with h DC gain
    1 and g = (-1/2, 1, -1/2), and "cdf53f" (the real-valued CDF 5/3 with the
    CDF 9/7 normalisation) with DC gain sqrt(2) for both low-pass filters."""
    if name == "cdf97":
        roots = npoly.polyroots(half_band_Q(4))
        real = [r for r in roots if abs(r.imag) < 1e-12]
        cplx = [r for r in roots if abs(r.imag) >= 1e-12]
        assert len(real) == 1 and len(cplx) == 2
        h = _lp_mul(_lp_mul(_c_term(), _c_term()), _lp_mul(_y_minus(cplx[0]), _y_minus(cplx[1])))
        f0 = _lp_mul(_lp_mul(_c_term(), _c_term()), _y_minus(real[0].real))
        h, f0 = h.real, f0.real
        h *= math.sqrt(2.0) / h.sum()
        f0 *= math.sqrt(2.0) / f0.sum()
    elif name == "dd137":
        return dd137_filters()
    elif name in ("cdf53", "cdf53f"):
        q = half_band_Q(2)                      # 1 + 2y
        h = _lp_mul(_c_term(), q[0] * np.array([0, 1.0, 0]) + q[1] * _y_minus(0.0).real)
        f0 = _c_term().copy()
        gh, gf = (1.0, 2.0) if name == "cdf53" else (math.sqrt(2.0), math.sqrt(2.0))
        h *= gh / h.sum()
        f0 *= gf / f0.sum()
    else:
        raise ValueError(name)
    L = (len(f0) - 1) // 2
    g = f0 * np.array([(-1) ** abs(k) for k in range(-L, L + 1)])
    return h, g


def dd137_filters():
    """(h, g) of the Deslauriers-Dubuc 13/7 wavelet, derived without lifting.

    The synthesis low-pass is the 4-point Deslauriers-Dubuc interpolating
    filter, the closed form c^2 Q_2(y) = c^2 (1 + 2y) (7 taps); the analysis
    high-pass is its modulation.  The analysis low-pass h is the symmetric
    13-tap filter for which the product h f0 is half-band (PR: every even
    power of the product except z^0 vanishes), with a zero of order 4 at the
    Nyquist frequency; both low-pass filters get DC gain sqrt(2)."""
    q = half_band_Q(2)
    f0 = _lp_mul(_lp_mul(_c_term(), _c_term()), q[0] * np.array([0, 1.0, 0]) + q[1] * _y_minus(0.0).real)
    f0 *= math.sqrt(2.0) / f0.sum()
    # unknowns: h[0..6] (h[-k] = h[k]); 7 linear conditions
    L = 6
    rows, rhs = [], []

    def full(v):
        return np.concatenate([v[:0:-1], v])            # h[-6..6] from h[0..6]

    def prod_coeff(k):
        """Row of the linear map h[0..6] -> coefficient of z^k in h f0."""
        r = np.zeros(L + 1)
        Lf = (len(f0) - 1) // 2
        for j in range(-L, L + 1):
            i = k - j
            if -Lf <= i <= Lf:
                r[abs(j)] += f0[i + Lf]
        return r
    for k in (2, 4, 6, 8):                              # half-band: even powers vanish
        rows.append(prod_coeff(k))
        rhs.append(0.0)
    dc = np.array([1.0] + [2.0] * L)                    # sum of the taps
    rows.append(dc)
    rhs.append(math.sqrt(2.0))
    alt = np.array([1.0] + [2.0 * (-1) ** k for k in range(1, L + 1)])
    rows.append(alt)                                    # H(-1) = 0
    rhs.append(0.0)
    rows.append(np.array([0.0] + [2.0 * (-1) ** k * k * k for k in range(1, L + 1)]))
    rhs.append(0.0)                                     # H''(-1) = 0 (odd orders vanish by symmetry)
    h = full(np.linalg.solve(np.array(rows), np.array(rhs)))
    Lg = (len(f0) - 1) // 2
    g = f0 * np.array([(-1) ** abs(k) for k in range(-Lg, Lg + 1)])
    return h, g


# --------------------------------------------------------------------------
# whole-point symmetric extension and brute-force banks
# --------------------------------------------------------------------------

def wps_index(i: np.ndarray, n: int) -> np.ndarray:
    """Index into a length-n signal of the whole-point symmetric extension."""
    if n == 1:
        return np.zeros_like(i)
    period = 2 * n - 2
    j = np.mod(i, period)
    return np.where(j > n - 1, period - j, j)


def analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray):
    """Low-pass s[n] = sum_k h[k] x~[2n+k], high-pass d[n] = sum_k g[k] x~[2n+1+k]."""
    N = len(x)
    Lh, Lg = (len(h) - 1) // 2, (len(g) - 1) // 2
    s = np.zeros((N + 1) // 2)
    d = np.zeros(N // 2)
    for n in range(len(s)):
        for k in range(-Lh, Lh + 1):
            s[n] += h[k + Lh] * x[wps_index(np.array(2 * n + k), N)]
    for n in range(len(d)):
        for k in range(-Lg, Lg + 1):
            d[n] += g[k + Lg] * x[wps_index(np.array(2 * n + 1 + k), N)]
    return s, d


def separable_bank(X: np.ndarray, name: str) -> np.ndarray:
    """One scale by separable convolution N^V | N^H |, Mallat quadrants."""
    h, g = cdf_filters(name)
    H, W = X.shape
    he, we = (H + 1) // 2, (W + 1) // 2
    rows = np.zeros((H, W))
    for r in range(H):
        s, d = analysis_1d(X[r].astype(np.float64), h, g)
        rows[r, :we], rows[r, we:] = s, d
    Y = np.zeros((H, W))
    for c in range(W):
        s, d = analysis_1d(rows[:, c], h, g)
        Y[:he, c], Y[he:, c] = s, d
    return Y


def nonseparable_bank(X: np.ndarray, name: str):
    """One scale by the non-separable convolution N = N^V N^H in one step.

    Every output is a single 2-D dot product of the symmetric extension of X
    with the outer-product kernel of its subband; returns the Mallat array and
    the 2-D kernel shapes (LL, HL, LH, HH) as (rows, cols)."""
    h, g = cdf_filters(name)
    H, W = X.shape
    he, we = (H + 1) // 2, (W + 1) // 2
    kernels = {  # (vertical filter, horizontal filter, row parity, col parity)
        "LL": (h, h, 0, 0), "HL": (h, g, 0, 1), "LH": (g, h, 1, 0), "HH": (g, g, 1, 1)}
    Y = np.zeros((H, W))
    shapes = {}
    for name_, (fv, fh, pr, pc) in kernels.items():
        K = np.outer(fv, fh)
        shapes[name_] = K.shape
        Lv, Lh = (K.shape[0] - 1) // 2, (K.shape[1] - 1) // 2
        nr = (H + 1 - pr) // 2
        nc = (W + 1 - pc) // 2
        out = np.zeros((nr, nc))
        rr = 2 * np.arange(nr) + pr
        cc = 2 * np.arange(nc) + pc
        for a in range(-Lv, Lv + 1):
            ri = wps_index(rr + a, H)
            for b in range(-Lh, Lh + 1):
                ci = wps_index(cc + b, W)
                out += K[a + Lv, b + Lh] * X[np.ix_(ri, ci)]
        r0 = 0 if pr == 0 else he
        c0 = 0 if pc == 0 else we
        Y[r0:r0 + nr, c0:c0 + nc] = out
    return Y, shapes
