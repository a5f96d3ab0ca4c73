"""The paper's fused non-separable lifting steps, as a CPU cross-check.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Proposed Schemes" fuses each horizontal/vertical pair of separable
steps into one spatial step per barrier:

    T_P = T_P^V T_P^H :  x1 += P x0
                         x2 += P* x0
                         x3 += P P* x0 + P* x1 + P x2
    S_U = S_U^V S_U^H :  x0 += U x1 + U* x2 + U U* x3
                         x1 += U* x3
                         x2 += U x3

(all right-hand sides are the values before the step).  Section "Optimization
Approach" splits P = P0 + P1 and U = U0 + U1 with P0, U0 the constant
(z^0) terms: the constant parts are applied as separable lifting steps that
never touch a neighbour, the remaining parts keep the fused form and are the
only ones that need the barrier.

Here each term is a whole-plane 2-D gather with the symmetric-border index
clamp applied per axis.  For CDF filters P(z) = p (1 + z_m), so P x0 at block
(n, m) is p (x0[n, m] + x0[n, m+1]); U(z) = u (1 + z_m^-1), so U x1 is
u (x1[n, m-1] + x1[n, m]).

The reversible integer 5/3 cannot be fused linearly because of its floors: the
fused step recomputes the neighbour's intermediate value (e.g. the vertical
predict of x3 needs x1 after the horizontal predict one row down) from that
neighbour's pre-step inputs, as a GPU work item that owns one block must.
"""
from __future__ import annotations

import numpy as np

from .lifting import is_integer, lifting_pairs, merge, quadrants, split, zeta


def nb(a: np.ndarray, dn: int, dm: int, shape) -> np.ndarray:
    """a[clamp(n+dn), clamp(m+dm)] over an output grid of `shape`."""
    rows = np.clip(np.arange(shape[0]) + dn, 0, a.shape[0] - 1)
    cols = np.clip(np.arange(shape[1]) + dm, 0, a.shape[1] - 1)
    return a[np.ix_(rows, cols)]


# --------------------------------------------------------------------------
# real-valued fused steps
# --------------------------------------------------------------------------

def T_fused(x, p):
    """Spatial predict T_P with all right-hand sides taken before the step."""
    x0, x1, x2, x3 = x
    s1, s2, s3 = x1.shape, x2.shape, x3.shape
    y1 = x1 + p * (nb(x0, 0, 0, s1) + nb(x0, 0, 1, s1))
    y2 = x2 + p * (nb(x0, 0, 0, s2) + nb(x0, 1, 0, s2))
    y3 = (x3 + p * p * (nb(x0, 0, 0, s3) + nb(x0, 0, 1, s3) + nb(x0, 1, 0, s3) + nb(x0, 1, 1, s3))
          + p * (nb(x1, 0, 0, s3) + nb(x1, 1, 0, s3))
          + p * (nb(x2, 0, 0, s3) + nb(x2, 0, 1, s3)))
    return [x0, y1, y2, y3]


def S_fused(x, u):
    """Spatial update S_U with all right-hand sides taken before the step."""
    x0, x1, x2, x3 = x
    s0, s1, s2 = x0.shape, x1.shape, x2.shape
    y0 = (x0 + u * (nb(x1, 0, -1, s0) + nb(x1, 0, 0, s0))
          + u * (nb(x2, -1, 0, s0) + nb(x2, 0, 0, s0))
          + u * u * (nb(x3, 0, 0, s0) + nb(x3, 0, -1, s0) + nb(x3, -1, 0, s0) + nb(x3, -1, -1, s0)))
    y1 = x1 + u * (nb(x3, 0, 0, s1) + nb(x3, -1, 0, s1))
    y2 = x2 + u * (nb(x3, 0, 0, s2) + nb(x3, 0, -1, s2))
    return [y0, y1, y2, x3]


def T_local(x, p):
    """Constant part P0 = p, as separable lifting (horizontal then vertical)."""
    x0, x1, x2, x3 = x
    x1 = x1 + p * nb(x0, 0, 0, x1.shape)
    x3 = x3 + p * nb(x2, 0, 0, x3.shape)
    x2 = x2 + p * nb(x0, 0, 0, x2.shape)
    x3 = x3 + p * nb(x1, 0, 0, x3.shape)
    return [x0, x1, x2, x3]


def T_nonlocal(x, p):
    """The P1 = p z part in fused form (reads the post-local values)."""
    x0, x1, x2, x3 = x
    s1, s2, s3 = x1.shape, x2.shape, x3.shape
    y1 = x1 + p * nb(x0, 0, 1, s1)
    y2 = x2 + p * nb(x0, 1, 0, s2)
    y3 = x3 + p * p * nb(x0, 1, 1, s3) + p * nb(x1, 1, 0, s3) + p * nb(x2, 0, 1, s3)
    return [x0, y1, y2, y3]


def S_local(x, u):
    """Constant part U0 = u, as separable lifting (horizontal then vertical)."""
    x0, x1, x2, x3 = x
    x0 = x0 + u * nb(x1, 0, 0, x0.shape)
    x2 = x2 + u * nb(x3, 0, 0, x2.shape)
    x0 = x0 + u * nb(x2, 0, 0, x0.shape)
    x1 = x1 + u * nb(x3, 0, 0, x1.shape)
    return [x0, x1, x2, x3]


def S_nonlocal(x, u):
    """The U1 = u z^-1 part in fused form (reads the post-local values)."""
    x0, x1, x2, x3 = x
    s0, s1, s2 = x0.shape, x1.shape, x2.shape
    y0 = x0 + u * nb(x1, 0, -1, s0) + u * nb(x2, -1, 0, s0) + u * u * nb(x3, -1, -1, s0)
    y1 = x1 + u * nb(x3, -1, 0, s1)
    y2 = x2 + u * nb(x3, 0, -1, s2)
    return [y0, y1, y2, x3]


# --------------------------------------------------------------------------
# reversible integer 5/3 fused steps (with neighbour recomputation)
# --------------------------------------------------------------------------

def T_int(x):
    """Fused T for the integer 5/3: T^H then T^V inside one step.

    The vertical predict of x3 needs x1' = x1 - floor((x0 + x0->)/2) one row
    down; that value is recomputed from the neighbour's pre-step inputs."""
    x0, x1, x2, x3 = x
    s1, s2, s3 = x1.shape, x2.shape, x3.shape
    x1h = x1 - (nb(x0, 0, 0, s1) + nb(x0, 0, 1, s1)) // 2
    x1h_own = nb(x1, 0, 0, s3) - (nb(x0, 0, 0, s3) + nb(x0, 0, 1, s3)) // 2
    x1h_dn = nb(x1, 1, 0, s3) - (nb(x0, 1, 0, s3) + nb(x0, 1, 1, s3)) // 2
    x3h = x3 - (nb(x2, 0, 0, s3) + nb(x2, 0, 1, s3)) // 2
    x2v = x2 - (nb(x0, 0, 0, s2) + nb(x0, 1, 0, s2)) // 2
    x3v = x3h - (x1h_own + x1h_dn) // 2
    return [x0, x1h, x2v, x3v]


def S_int(x):
    """Fused S for the integer 5/3: S^H then S^V inside one step.

    The vertical update of x0 needs x2'' = x2 + floor((x3 + x3<- + 2)/4) one
    row up; that value is recomputed from the neighbour's inputs."""
    x0, x1, x2, x3 = x
    s0, s1, s2 = x0.shape, x1.shape, x2.shape
    x2h = x2 + (nb(x3, 0, 0, s2) + nb(x3, 0, -1, s2) + 2) // 4
    x2h_own = nb(x2, 0, 0, s0) + (nb(x3, 0, 0, s0) + nb(x3, 0, -1, s0) + 2) // 4
    x2h_up = nb(x2, -1, 0, s0) + (nb(x3, -1, 0, s0) + nb(x3, -1, -1, s0) + 2) // 4
    x0h = x0 + (nb(x1, 0, -1, s0) + nb(x1, 0, 0, s0) + 2) // 4
    x0v = x0h + (x2h_own + x2h_up + 2) // 4
    x1v = x1 + (nb(x3, 0, 0, s1) + nb(x3, -1, 0, s1) + 2) // 4
    return [x0v, x1v, x2h, x3]


# --------------------------------------------------------------------------
# one scale with the fused schemes
# --------------------------------------------------------------------------

def nonsep_fwd_level(X: np.ndarray, wavelet: str = "cdf97", split_consts: bool = False) -> np.ndarray:
    """One forward scale with the non-separable lifting scheme  S_U | T_P |."""
    h, w = X.shape
    if is_integer(wavelet):
        x = list(split(np.asarray(X).astype(np.int64)))
        x = S_int(T_int(x))
        return quadrants(*x, h, w)
    x = list(split(np.asarray(X, dtype=np.float64)))
    for p, u in lifting_pairs(wavelet):
        if split_consts:
            x = S_nonlocal(S_local(T_nonlocal(T_local(x, p), p), u), u)
        else:
            x = S_fused(T_fused(x, p), u)
    z = zeta(wavelet)
    x[0] = x[0] * z ** 2
    x[3] = x[3] * z ** -2
    return quadrants(*x, h, w)


# --------------------------------------------------------------------------
# schemes written as 4x4 step matrices, evaluated on the symmetrically
# extended image: the non-separable polyconvolution N_{P,U}, and the fused
# lifting steps T_P, S_U with filters of any length (DD 13/7)
# --------------------------------------------------------------------------
# A matrix entry G*(z_n) H(z_m) -- a vertical 1-D filter times a horizontal
# one -- is the pair (vertical taps, horizontal taps); taps are
# {offset: coefficient}, offset k reading sample n + k (m + k).  ONE is the
# unit filter.  The image is extended by the whole-point symmetric extension
# (wide enough for every step's reach), split into its four polyphase
# components, every step applied to whole planes with no border rule at all,
# and the image's part cut out: lifting on the extended signal equals the
# oracle's per-step reflection inside the image.

ONE = {0: 1.0}


def _compose(a: dict, b: dict) -> dict:
    """The filter a b (apply b, then a): offsets add."""
    out = {}
    for i, x in a.items():
        for j, y in b.items():
            out[i + j] = out.get(i + j, 0.0) + x * y
    return out


def _plus(a: dict, b: dict) -> dict:
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0.0) + v
    return out


def _neg(a: dict) -> dict:
    return {k: -v for k, v in a.items()}


def polyconv_matrix(P: dict, U: dict):
    """N_{P,U} of Section "Proposed Schemes" (one lifting pair in one step):

        [ V*V  V*U  U*V  U*U ]
        [ V*P  V*   U*P  U*  ]      V = P U + 1
        [ P*V  P*U  V    U   ]
        [ P*P  P*   P    1   ]

    as (vertical, horizontal) filter pairs, rows = output component."""
    V = _plus(_compose(P, U), ONE)
    return [[(V, V), (V, U), (U, V), (U, U)],
            [(V, P), (V, ONE), (U, P), (U, ONE)],
            [(P, V), (P, U), (ONE, V), (ONE, U)],
            [(P, P), (P, ONE), (ONE, P), (ONE, ONE)]]


def polyconv_inverse_matrix(P: dict, U: dict):
    """The inverse of N_{P,U}: per axis the inverse of the pair matrix
    [[V, U], [P, 1]] is [[1, -U], [-P, V]] (determinant V - U P = 1), and the
    2-D matrix is again the product of the vertical and horizontal ones."""
    V = _plus(_compose(P, U), ONE)
    m1 = [[ONE, _neg(U)], [_neg(P), V]]
    return [[(m1[c >> 1][k >> 1], m1[c & 1][k & 1]) for k in range(4)] for c in range(4)]


def fused_T_matrix(P: dict):
    """T_P of Section "Proposed Schemes" (None: no term; the diagonal is 1)."""
    return [[(ONE, ONE), None, None, None],
            [(ONE, P), (ONE, ONE), None, None],
            [(P, ONE), None, (ONE, ONE), None],
            [(P, P), (P, ONE), (ONE, P), (ONE, ONE)]]


def fused_S_matrix(U: dict):
    """S_U of Section "Proposed Schemes"."""
    return [[(ONE, ONE), (ONE, U), (U, ONE), (U, U)],
            [None, (ONE, ONE), None, (U, ONE)],
            [None, None, (ONE, ONE), (ONE, U)],
            [None, None, None, (ONE, ONE)]]


def apply_matrix(x, M):
    """One step: out_c = sum_k M[c][k] x_k over whole planes of equal shape.
    Samples near the planes' edges read wrapped-around values; the callers'
    margins keep that garbage outside the image."""
    out = []
    for c in range(4):
        acc = np.zeros_like(x[0])
        for k in range(4):
            if M[c][k] is None:
                continue
            vt, ht = M[c][k]
            for i, a in vt.items():
                for j, b in ht.items():
                    acc += (a * b) * np.roll(x[k], (-i, -j), axis=(0, 1))
        out.append(acc)
    return out


def _reach(M) -> int:
    return max(abs(k) for row in M for e in row if e is not None for t in e for k in t)


def _extended_components(X: np.ndarray, margin: int):
    """The four polyphase components of X extended symmetrically by `margin`
    blocks on every side (one more sample at the end of an odd side, so that
    all four components have the same shape); block (n, m) of a component
    is block (n - margin, m - margin) of the image's."""
    from .filterbank import wps_index
    h, w = X.shape
    rows = wps_index(np.arange(-2 * margin, h + 2 * margin + h % 2), h)
    cols = wps_index(np.arange(-2 * margin, w + 2 * margin + w % 2), w)
    return list(split(np.asarray(X, dtype=np.float64)[np.ix_(rows, cols)]))


def _cut(x, margin: int, h: int, w: int):
    he, ho, we, wo = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    sl = lambda n, m: (slice(margin, margin + n), slice(margin, margin + m))
    return [x[0][sl(he, we)], x[1][sl(he, wo)], x[2][sl(ho, we)], x[3][sl(ho, wo)]]


def matrix_scheme_fwd_level(X: np.ndarray, wavelet: str, scheme: str) -> np.ndarray:
    """One forward scale of a float wavelet, every lifting pair applied as
    one polyconvolution step N_{P,U} (scheme "polyconv") or as the two fused
    steps T_P then S_U (scheme "fused"), on the extended image."""
    from .lifting import lifting_taps
    h, w = X.shape
    pairs = lifting_taps(wavelet)
    if scheme == "polyconv":
        steps = [polyconv_matrix(P, U) for P, U in pairs]
    elif scheme == "fused":
        steps = [M for P, U in pairs for M in (fused_T_matrix(P), fused_S_matrix(U))]
    else:
        raise ValueError(scheme)
    margin = sum(_reach(M) for M in steps) + 2
    x = _extended_components(X, margin)
    for M in steps:
        x = apply_matrix(x, M)
    x = _cut(x, margin, h, w)
    z = zeta(wavelet)
    x[0] = x[0] * z ** 2
    x[3] = x[3] * z ** -2
    return quadrants(*x, h, w)


def matrix_scheme_inv_level(Y: np.ndarray, wavelet: str, scheme: str = "polyconv") -> np.ndarray:
    """One inverse scale: the inverse polyconvolution of every pair, last
    pair first, on the symmetric extension of the image the pyramid level
    belongs to.  The extension of a subband is taken at the reflected pixel
    position of each of its samples, the same extension the forward
    transform of the extended image has."""
    from .filterbank import wps_index
    from .lifting import lifting_taps, unquadrants
    if scheme != "polyconv":
        raise ValueError(scheme)
    h, w = Y.shape
    steps = [polyconv_inverse_matrix(P, U) for P, U in reversed(lifting_taps(wavelet))]
    margin = sum(_reach(M) for M in steps) + 2
    q = list(unquadrants(np.asarray(Y, dtype=np.float64)))
    z = zeta(wavelet)
    q[0] = q[0] * z ** -2
    q[3] = q[3] * z ** 2
    x = []
    for k in range(4):
        pr, pc = k >> 1, k & 1
        r = (wps_index(2 * np.arange(-margin, (h + 1) // 2 + margin) + pr, h) - pr) // 2
        c = (wps_index(2 * np.arange(-margin, (w + 1) // 2 + margin) + pc, w) - pc) // 2
        x.append(q[k][np.ix_(r, c)])
    for M in steps:
        x = apply_matrix(x, M)
    return merge(*_cut(x, margin, h, w), h, w)


def polyconv_fwd(X: np.ndarray, wavelet: str = "cdf97", levels: int = 1) -> np.ndarray:
    """Multi-level forward transform with the polyconvolution scheme."""
    from .lifting import level_shapes
    Y = np.asarray(X, dtype=np.float64).copy()
    for h, w in level_shapes(*Y.shape, levels):
        Y[:h, :w] = matrix_scheme_fwd_level(Y[:h, :w], wavelet, "polyconv")
    return Y


def polyconv_inv(Y: np.ndarray, wavelet: str = "cdf97", levels: int = 1) -> np.ndarray:
    """Multi-level inverse with the inverse polyconvolution scheme."""
    from .lifting import level_shapes
    X = np.asarray(Y, dtype=np.float64).copy()
    for h, w in reversed(level_shapes(*X.shape, levels)):
        X[:h, :w] = matrix_scheme_inv_level(X[:h, :w], wavelet)
    return X
