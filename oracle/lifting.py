"""Separable 2-D lifting DWT in FP64 and int64 -- the oracle's definition.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

What is computed
----------------
The paper (Section "Background") writes one scale of the 2-D transform as a
map of the four polyphase components of an image (the "quadruple of wavelet
coefficients") and factors it, following Sweldens, into K pairs of lifting
steps, eq. (2): predict P then update U.  In two dimensions each step becomes a
4x4 matrix acting on the column vector (x0, x1, x2, x3); the separable lifting
scheme is the sequence

    S_U^V | S_U^H | T_P^V | T_P^H |          (applied right to left)

with

    T_P^H : x1 += P x0,   x3 += P x2          (horizontal predict)
    T_P^V : x2 += P* x0,  x3 += P* x1         (vertical predict)
    S_U^H : x0 += U x1,   x2 += U x3          (horizontal update)
    S_U^V : x0 += U* x2,  x1 += U* x3         (vertical update)

(G* is G with the roles of the horizontal and vertical axes swapped.)  The
paper states that all of its schemes compute the same values, so this plain
separable form is the definition the fused GPU kernels are checked against.

Conventions fixed here (the paper leaves them open)
---------------------------------------------------
* Polyphase split of an H x W image X (row index first):
      x0 = X[0::2, 0::2]   (even row, even column)  -> LL
      x1 = X[0::2, 1::2]   (even row, odd column)   -> HL (high horizontally)
      x2 = X[1::2, 0::2]   (odd row, even column)   -> LH
      x3 = X[1::2, 1::2]   (odd row, odd column)    -> HH
  Low-pass components have ceil(N/2) samples along an axis, high-pass ones
  floor(N/2).
* Lifting polynomials: P(z) = p (1 + z) and U(z) = u (1 + z^-1), i.e.
      odd[m]  += p (even[m] + even[m+1])
      even[m] += u (odd[m-1] + odd[m]).
  This is the paper's appendix example P(z) = -1/2 (1 + z^-1) up to the
  labelling of which even neighbour is "next".
* Borders: whole-point symmetric extension of the image (X[-k] = X[k],
  X[N-1+k] = X[N-1-k]).  In the polyphase domain a lifting step then reads an
  index -1 as 0 and an index M (one past the end of that component) as M-1,
  i.e. the neighbour index is clamped into the component's own extent.
* CDF 9/7: pairs (alpha, beta), (gamma, delta) of the Daubechies-Sweldens
  factorisation, followed by a scaling of the low-pass output by zeta and the
  high-pass output by 1/zeta along each axis, zeta chosen so that the low-pass
  filter has DC gain sqrt(2) (a constant image c gives LL = 2c per level).
  In 2-D: LL * zeta^2, HL * 1, LH * 1, HH * zeta^-2.
* CDF 5/3 (real valued, as evaluated in the paper's Section "Evaluation"):
  one pair, predict p = -1/2 and update u = 1/4, then the same scaling rule
  as CDF 9/7 (low-pass DC gain sqrt(2) per axis), which here gives
  zeta = sqrt(2): LL * 2, HH * 1/2.
* Reversible integer CDF 5/3 (the paper's 5/3 is real valued; this integer
  form keeps its predict -1/2 and update 1/4 with floor rounding):
      odd[m]  -= floor((even[m] + even[m+1]) / 2)
      even[m] += floor((odd[m-1] + odd[m] + 2) / 4)
  applied in the paper's separable order T^H, T^V, S^H, S^V; no scaling.
  Valid for |x| < 2**28.
* Multi-level: Mallat pyramid in one H x W array.  Level l transforms the
  ceil(h/2) x ceil(w/2) LL of level l-1 in place of it; every transformed
  level must be at least 2 x 2.
"""
from __future__ import annotations

import math

import numpy as np

# Daubechies-Sweldens lifting factorisation of the CDF 9/7 filter pair
# (predict, update, predict, update).  Pinned against the closed-form filters
# by test_cdf97_constants_from_closed_form in tests/test_oracle_pins.py.
ALPHA = -1.586134342059924
BETA = -0.052980118572961
GAMMA = 0.882911075530934
DELTA = 0.443506852043971
# Scaling so that the composed low-pass filter has DC gain sqrt(2): a constant
# signal c becomes c * (1 + 2 beta (1 + 2 alpha)) after the lifting pairs.
ZETA = math.sqrt(2.0) / (1.0 + 2.0 * BETA * (1.0 + 2.0 * ALPHA))
# Real-valued CDF 5/3: one pair; the same rule gives zeta = sqrt(2) since
# 1 + 2p = 0.
P53 = -0.5
U53 = 0.25
ZETA53 = math.sqrt(2.0) / (1.0 + 2.0 * U53 * (1.0 + 2.0 * P53))

# Deslauriers-Dubuc 13/7 (the paper's third wavelet, Section "Evaluation"):
# one pair of 4-tap steps, the 4-point interpolating predict and its update,
#     odd[m]  -= (9 (even[m] + even[m+1]) - (even[m-1] + even[m+2])) / 16
#     even[m] += (9 (odd[m-1] + odd[m]) - (odd[m-2] + odd[m+1])) / 32
# as {offset: coefficient} taps (offset k reads sample m + k).
DD137_P = {-1: 1.0 / 16, 0: -9.0 / 16, 1: -9.0 / 16, 2: 1.0 / 16}
DD137_U = {-2: -1.0 / 32, -1: 9.0 / 32, 0: 9.0 / 32, 1: -1.0 / 32}
# The same normalisation rule (low-pass DC gain sqrt(2) per axis): the
# predict removes constants (its taps sum to -1), so the lifted low-pass has
# DC gain 1 and zeta = sqrt(2): LL * 2, HH * 1/2.
ZETA137 = math.sqrt(2.0) / (1.0 + sum(DD137_U.values()) * (1.0 + sum(DD137_P.values())))

# "cdf53" is the reversible integer transform, "cdf53f" the real-valued one
WAVELETS = ("cdf97", "cdf53", "cdf53f", "dd137")
INT_LIMIT = 1 << 28


def lifting_pairs(wavelet: str):
    """(p, u) per lifting pair of a two-tap float wavelet (eq. (2), K pairs):
    P(z) = p (1 + z), U(z) = u (1 + z^-1)."""
    if wavelet == "cdf97":
        return [(ALPHA, BETA), (GAMMA, DELTA)]
    if wavelet == "cdf53f":
        return [(P53, U53)]
    raise ValueError(f"no two-tap float lifting pairs for {wavelet!r}")


def lifting_taps(wavelet: str):
    """[(P, U), ...] per lifting pair of any float wavelet, each filter as
    {offset: coefficient}: odd[m] += sum_k P[k] even[m+k],
    even[m] += sum_k U[k] odd[m+k]."""
    if wavelet == "dd137":
        return [(dict(DD137_P), dict(DD137_U))]
    return [({0: p, 1: p}, {-1: u, 0: u}) for p, u in lifting_pairs(wavelet)]


def zeta(wavelet: str) -> float:
    """Per-axis scaling of the float wavelet (low-pass * zeta, high-pass / zeta)."""
    if wavelet == "cdf97":
        return ZETA
    if wavelet == "cdf53f":
        return ZETA53
    if wavelet == "dd137":
        return ZETA137
    raise ValueError(f"no scaling for {wavelet!r}")


def is_integer(wavelet: str) -> bool:
    if wavelet not in WAVELETS:
        raise ValueError(f"unknown wavelet {wavelet!r}")
    return wavelet == "cdf53"


# ---------------------------------------------------------------------------
# polyphase split / merge and the Mallat quadrant layout
# ---------------------------------------------------------------------------

def split(X: np.ndarray):
    """The four polyphase components (x0, x1, x2, x3) of X, as copies."""
    return (X[0::2, 0::2].copy(), X[0::2, 1::2].copy(),
            X[1::2, 0::2].copy(), X[1::2, 1::2].copy())


def merge(x0, x1, x2, x3, h: int, w: int) -> np.ndarray:
    """Interleave four polyphase components back into an h x w image."""
    X = np.empty((h, w), dtype=x0.dtype)
    X[0::2, 0::2] = x0
    X[0::2, 1::2] = x1
    X[1::2, 0::2] = x2
    X[1::2, 1::2] = x3
    return X


def quadrants(x0, x1, x2, x3, h: int, w: int) -> np.ndarray:
    """Place LL, HL, LH, HH of one level into an h x w array (Mallat)."""
    he, we = (h + 1) // 2, (w + 1) // 2
    Y = np.empty((h, w), dtype=x0.dtype)
    Y[:he, :we] = x0
    Y[:he, we:] = x1
    Y[he:, :we] = x2
    Y[he:, we:] = x3
    return Y


def unquadrants(Y: np.ndarray):
    """Inverse of quadrants(): (LL, HL, LH, HH) copies of an h x w array."""
    h, w = Y.shape
    he, we = (h + 1) // 2, (w + 1) // 2
    return (Y[:he, :we].copy(), Y[:he, we:].copy(),
            Y[he:, :we].copy(), Y[he:, we:].copy())


# ---------------------------------------------------------------------------
# 1-D lifting operators with symmetric borders, applied along one axis
# ---------------------------------------------------------------------------

def _predict_operands(even: np.ndarray, n_odd: int, axis: int):
    """even[m] and even[m+1] for m = 0..n_odd-1, index clamped to the extent."""
    ne = even.shape[axis]
    m = np.arange(n_odd)
    return (np.take(even, m, axis=axis),
            np.take(even, np.minimum(m + 1, ne - 1), axis=axis))


def _update_operands(odd: np.ndarray, n_even: int, axis: int):
    """odd[m-1] and odd[m] for m = 0..n_even-1, indices clamped to the extent."""
    no = odd.shape[axis]
    m = np.arange(n_even)
    return (np.take(odd, np.clip(m - 1, 0, no - 1), axis=axis),
            np.take(odd, np.minimum(m, no - 1), axis=axis))


def _predict(even, odd, p, axis, integer, sign=+1):
    a, b = _predict_operands(even, odd.shape[axis], axis)
    if integer:
        odd -= sign * ((a + b) // 2)
    else:
        odd += (sign * p) * (a + b)


def _update(odd, even, u, axis, integer, sign=+1):
    a, b = _update_operands(odd, even.shape[axis], axis)
    if integer:
        even += sign * ((a + b + 2) // 4)
    else:
        even += (sign * u) * (a + b)


# axis 1 = horizontal (m, columns), axis 0 = vertical (n, rows)
H_AXIS, V_AXIS = 1, 0


# ---------------------------------------------------------------------------
# lifting steps with taps beyond the nearest neighbours (DD 13/7)
# ---------------------------------------------------------------------------
# With longer filters the symmetric extension is no longer a clamp of the
# component index: the sample two places before the first even sample is the
# second even sample (X[-2] = X[2]).  The general rule reflects the pixel
# position 2k + q of component sample k (q = 0 even, 1 odd) into [0, n) and
# maps it back; a reflection keeps the parity of the position, so the sample
# read is always one of the same component.

def reflect_component(k: np.ndarray, q: int, n: int) -> np.ndarray:
    """Component index of sample k (any integer) of the parity-q component of
    a length-n signal under whole-point symmetric extension."""
    p = 2 * np.asarray(k) + q
    if n == 1:
        return np.zeros_like(p)
    period = 2 * (n - 1)
    p = np.mod(p, period)
    p = np.where(p > n - 1, period - p, p)
    assert np.all(p % 2 == q)
    return (p - q) // 2


def _lift_taps(src, dst, taps, axis, n, q_src, sign=+1):
    """dst[m] += sign * sum_k taps[k] * src[m + k] along `axis`, the source
    (a component of parity q_src of a length-n signal) read through the
    symmetric extension."""
    m = np.arange(dst.shape[axis])
    for k, c in sorted(taps.items()):
        dst += (sign * c) * np.take(src, reflect_component(m + k, q_src, n), axis=axis)


def _forward_pair_taps(x, P, U, h, w):
    x0, x1, x2, x3 = x
    # T_P^H, T_P^V, S_U^H, S_U^V (the order of the two-tap pairs)
    _lift_taps(x0, x1, P, H_AXIS, w, 0)
    _lift_taps(x2, x3, P, H_AXIS, w, 0)
    _lift_taps(x0, x2, P, V_AXIS, h, 0)
    _lift_taps(x1, x3, P, V_AXIS, h, 0)
    _lift_taps(x1, x0, U, H_AXIS, w, 1)
    _lift_taps(x3, x2, U, H_AXIS, w, 1)
    _lift_taps(x2, x0, U, V_AXIS, h, 1)
    _lift_taps(x3, x1, U, V_AXIS, h, 1)


def _inverse_pair_taps(x, P, U, h, w):
    x0, x1, x2, x3 = x
    _lift_taps(x2, x0, U, V_AXIS, h, 1, sign=-1)
    _lift_taps(x3, x1, U, V_AXIS, h, 1, sign=-1)
    _lift_taps(x1, x0, U, H_AXIS, w, 1, sign=-1)
    _lift_taps(x3, x2, U, H_AXIS, w, 1, sign=-1)
    _lift_taps(x0, x2, P, V_AXIS, h, 0, sign=-1)
    _lift_taps(x1, x3, P, V_AXIS, h, 0, sign=-1)
    _lift_taps(x0, x1, P, H_AXIS, w, 0, sign=-1)
    _lift_taps(x2, x3, P, H_AXIS, w, 0, sign=-1)


def _forward_pair(x, p, u, integer):
    x0, x1, x2, x3 = x
    # T_P^H
    _predict(x0, x1, p, H_AXIS, integer)
    _predict(x2, x3, p, H_AXIS, integer)
    # T_P^V
    _predict(x0, x2, p, V_AXIS, integer)
    _predict(x1, x3, p, V_AXIS, integer)
    # S_U^H
    _update(x1, x0, u, H_AXIS, integer)
    _update(x3, x2, u, H_AXIS, integer)
    # S_U^V
    _update(x2, x0, u, V_AXIS, integer)
    _update(x3, x1, u, V_AXIS, integer)


def _inverse_pair(x, p, u, integer):
    x0, x1, x2, x3 = x
    # undo S_U^V, S_U^H, T_P^V, T_P^H in that order
    _update(x2, x0, u, V_AXIS, integer, sign=-1)
    _update(x3, x1, u, V_AXIS, integer, sign=-1)
    _update(x1, x0, u, H_AXIS, integer, sign=-1)
    _update(x3, x2, u, H_AXIS, integer, sign=-1)
    _predict(x0, x2, p, V_AXIS, integer, sign=-1)
    _predict(x1, x3, p, V_AXIS, integer, sign=-1)
    _predict(x0, x1, p, H_AXIS, integer, sign=-1)
    _predict(x2, x3, p, H_AXIS, integer, sign=-1)


def _pairs(wavelet):
    if is_integer(wavelet):
        return [(None, None)]
    return lifting_pairs(wavelet)


def _prepare(X: np.ndarray, wavelet: str) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("expected a 2-D image")
    if is_integer(wavelet):
        if not np.issubdtype(X.dtype, np.integer):
            raise TypeError("the reversible 5/3 transform takes integer input")
        Y = X.astype(np.int64)
        if Y.size and np.abs(Y).max() >= INT_LIMIT:
            raise ValueError("integer input outside |x| < 2**28")
        return Y
    return X.astype(np.float64)


def fwd_level(X: np.ndarray, wavelet: str) -> np.ndarray:
    """One scale: image (h x w) -> LL/HL/LH/HH quadrants (h x w)."""
    h, w = X.shape
    if h < 2 or w < 2:
        raise ValueError("every transformed level must be at least 2 x 2")
    integer = is_integer(wavelet)
    x = split(X)
    if wavelet == "dd137":
        for P, U in lifting_taps(wavelet):
            _forward_pair_taps(x, P, U, h, w)
    else:
        for p, u in _pairs(wavelet):
            _forward_pair(x, p, u, integer)
    x0, x1, x2, x3 = x
    if not integer:
        z = zeta(wavelet)
        x0 *= z * z
        x3 *= 1.0 / (z * z)
    return quadrants(x0, x1, x2, x3, h, w)


def inv_level(Y: np.ndarray, wavelet: str) -> np.ndarray:
    """One scale: LL/HL/LH/HH quadrants (h x w) -> image (h x w)."""
    h, w = Y.shape
    if h < 2 or w < 2:
        raise ValueError("every transformed level must be at least 2 x 2")
    integer = is_integer(wavelet)
    x = list(unquadrants(Y))
    if not integer:
        z = zeta(wavelet)
        x[0] *= 1.0 / (z * z)
        x[3] *= z * z
    if wavelet == "dd137":
        for P, U in reversed(lifting_taps(wavelet)):
            _inverse_pair_taps(x, P, U, h, w)
    else:
        for p, u in reversed(_pairs(wavelet)):
            _inverse_pair(x, p, u, integer)
    return merge(*x, h, w)


def level_shapes(h: int, w: int, levels: int):
    """Shape of the array each level transforms: (h, w), (ceil(h/2), ...)."""
    shapes = []
    for _ in range(levels):
        shapes.append((h, w))
        h, w = (h + 1) // 2, (w + 1) // 2
    return shapes


def max_levels(h: int, w: int) -> int:
    """Largest level count for which every transformed level is >= 2 x 2."""
    n = 0
    while h >= 2 and w >= 2:
        n += 1
        h, w = (h + 1) // 2, (w + 1) // 2
    return n


def fwd(X: np.ndarray, wavelet: str = "cdf97", levels: int = 1) -> np.ndarray:
    """Multi-level forward transform; returns the Mallat pyramid (H x W)."""
    Y = _prepare(X, wavelet)
    if not 1 <= levels <= max_levels(*Y.shape):
        raise ValueError("level count out of range for this image size")
    for h, w in level_shapes(*Y.shape, levels):
        Y[:h, :w] = fwd_level(Y[:h, :w], wavelet)
    return Y


def inv(Y: np.ndarray, wavelet: str = "cdf97", levels: int = 1) -> np.ndarray:
    """Multi-level inverse transform of a Mallat pyramid."""
    X = _prepare(Y, wavelet) if is_integer(wavelet) else np.asarray(Y, np.float64).copy()
    if not 1 <= levels <= max_levels(*X.shape):
        raise ValueError("level count out of range for this image size")
    for h, w in reversed(level_shapes(*X.shape, levels)):
        X[:h, :w] = inv_level(X[:h, :w], wavelet)
    return X
