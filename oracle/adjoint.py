"""Transpose W^T of the forward 2-D lifting DWT, from explicit step matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward transform of one scale is a product of the separable lifting step
matrices T_P^H, T_P^V, S_U^H, S_U^V (Section "Background"), then a diagonal
scaling and a permutation into the Mallat layout.  Each step adds a 1-D
operator applied along one axis of one polyphase component to another
component, e.g.  x1 += P x0  along rows.  Here every such 1-D operator is
built as an explicit sparse matrix (with the symmetric-border index clamp of
the forward definition baked into its entries), and the adjoint applies the
*transposed* matrices to the steps in reverse order:

    forward   x_dst += A x_src          adjoint   x_src += A^T x_dst

Levels run from the coarsest to the finest.  Because the transpose of a
clamped neighbour access is not itself a clamped neighbour access, this module
deliberately shares nothing with the index helpers of `lifting` beyond the
lifting constants.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .lifting import ZETA, lifting_pairs, level_shapes, max_levels


def predict_matrix(n_even: int, n_odd: int) -> sp.csr_matrix:
    """(n_odd x n_even) matrix of  odd[m] += even[m] + even[min(m+1, n_even-1)]."""
    rows, cols = [], []
    for m in range(n_odd):
        rows += [m, m]
        cols += [m, min(m + 1, n_even - 1)]
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n_odd, n_even))


def update_matrix(n_odd: int, n_even: int) -> sp.csr_matrix:
    """(n_even x n_odd) matrix of  even[m] += odd[clip(m-1)] + odd[min(m, n_odd-1)]."""
    rows, cols = [], []
    for m in range(n_even):
        rows += [m, m]
        cols += [min(max(m - 1, 0), n_odd - 1), min(m, n_odd - 1)]
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n_even, n_odd))


def _h_apply(A, x):
    """Apply a 1-D operator along rows: y[r, :] = A @ x[r, :]."""
    return (A @ x.T).T


def _v_apply(A, x):
    """Apply a 1-D operator along columns: y[:, c] = A @ x[:, c]."""
    return A @ x


def _step_list(h: int, w: int, wavelet: str):
    """The forward step sequence of one scale as (dst, src, axis, coeff, A)."""
    he, ho, we, wo = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    PH, PV = predict_matrix(we, wo), predict_matrix(he, ho)
    UH, UV = update_matrix(wo, we), update_matrix(ho, he)
    steps = []
    for p, u in lifting_pairs(wavelet):
        steps += [(1, 0, "h", p, PH), (3, 2, "h", p, PH),     # T_P^H
                  (2, 0, "v", p, PV), (3, 1, "v", p, PV),     # T_P^V
                  (0, 1, "h", u, UH), (2, 3, "h", u, UH),     # S_U^H
                  (0, 2, "v", u, UV), (1, 3, "v", u, UV)]     # S_U^V
    return steps


def _fwd_level_matrix_form(X: np.ndarray, wavelet: str) -> np.ndarray:
    """Forward scale written with the same explicit matrices (for self-checks)."""
    h, w = X.shape
    x = [X[0::2, 0::2].astype(np.float64), X[0::2, 1::2].astype(np.float64),
         X[1::2, 0::2].astype(np.float64), X[1::2, 1::2].astype(np.float64)]
    for dst, src, axis, c, A in _step_list(h, w, wavelet):
        x[dst] = x[dst] + c * (_h_apply(A, x[src]) if axis == "h" else _v_apply(A, x[src]))
    x[0] = x[0] * ZETA ** 2
    x[3] = x[3] * ZETA ** -2
    he, we = (h + 1) // 2, (w + 1) // 2
    Y = np.empty((h, w))
    Y[:he, :we], Y[:he, we:], Y[he:, :we], Y[he:, we:] = x
    return Y


def adj_level(G: np.ndarray, wavelet: str) -> np.ndarray:
    """W^T of one scale: Mallat-layout cotangent (h x w) -> image cotangent."""
    h, w = G.shape
    he, we = (h + 1) // 2, (w + 1) // 2
    # transpose of the Mallat permutation
    x = [G[:he, :we].astype(np.float64), G[:he, we:].astype(np.float64),
         G[he:, :we].astype(np.float64), G[he:, we:].astype(np.float64)]
    # the scaling is diagonal, hence its own transpose
    x[0] = x[0] * ZETA ** 2
    x[3] = x[3] * ZETA ** -2
    for dst, src, axis, c, A in reversed(_step_list(h, w, wavelet)):
        At = A.T.tocsr()
        x[src] = x[src] + c * (_h_apply(At, x[dst]) if axis == "h" else _v_apply(At, x[dst]))
    # transpose of the polyphase split is the interleave
    X = np.empty((h, w))
    X[0::2, 0::2], X[0::2, 1::2], X[1::2, 0::2], X[1::2, 1::2] = x
    return X


def adj(G: np.ndarray, wavelet: str = "cdf97", levels: int = 1) -> np.ndarray:
    """W^T of the multi-level forward transform (Mallat pyramid in, image out)."""
    if wavelet != "cdf97":
        raise ValueError("the adjoint is defined for the linear CDF 9/7 transform")
    X = np.asarray(G, dtype=np.float64).copy()
    if not 1 <= levels <= max_levels(*X.shape):
        raise ValueError("level count out of range for this image size")
    for h, w in reversed(level_shapes(*X.shape, levels)):
        X[:h, :w] = adj_level(X[:h, :w], wavelet)
    return X
