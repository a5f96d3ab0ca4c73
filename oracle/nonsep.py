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

from .lifting import lifting_pairs, is_integer, quadrants, split, zeta


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
