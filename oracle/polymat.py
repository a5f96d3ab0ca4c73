"""Exact 4x4 matrices of bivariate Laurent polynomials and the op/step count.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Background" describes every scheme as a sequence of 4x4 polyphase
matrices acting on the column vector (x0, x1, x2, x3), each matrix one
calculation step, barriers written as `|`.  The operation count is the number
of distinct polynomial terms in all matrices, not counting the unit diagonal.
This module builds those matrices with exact rational coefficients so that:

* the paper's fused matrices can be checked against products of separable
  ones:  T_P = T_P^V T_P^H,  S_U = S_U^V S_U^H  (Section "Proposed Schemes"),
  and the polyconvolution N_{P,U} = S_U T_P with V = P U + 1;
* the step and operation counts of the lifting rows of Table 1 follow from
  the step lists of the schemes, including the split P = P0 + P1,
  U = U0 + U1 of Section "Optimization Approach".

A polynomial is a dict {(a, b): coefficient} for the term z_m^a z_n^b
(m horizontal, n vertical); the transposed polynomial G* swaps a and b.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Tuple

Poly = Dict[Tuple[int, int], Fraction]


def poly(terms) -> Poly:
    out: Poly = {}
    for (a, b), c in terms:
        c = Fraction(c)
        out[(a, b)] = out.get((a, b), Fraction(0)) + c
    return {k: v for k, v in out.items() if v != 0}


def horizontal(taps) -> Poly:
    """1-D filter along m: taps = [(exponent, coefficient), ...]."""
    return poly(((e, 0), c) for e, c in taps)


def padd(p: Poly, q: Poly) -> Poly:
    return poly(list(p.items()) + list(q.items()))


def pmul(p: Poly, q: Poly) -> Poly:
    return poly(((a1 + a2, b1 + b2), c1 * c2)
                for (a1, b1), c1 in p.items() for (a2, b2), c2 in q.items())


def star(p: Poly) -> Poly:
    """G*(z_m, z_n) = G(z_n, z_m)."""
    return {(b, a): c for (a, b), c in p.items()}


ZERO: Poly = {}
ONE: Poly = {(0, 0): Fraction(1)}

Mat = List[List[Poly]]


def eye() -> Mat:
    return [[dict(ONE) if i == j else {} for j in range(4)] for i in range(4)]


def matmul(A: Mat, B: Mat) -> Mat:
    C = [[{} for _ in range(4)] for _ in range(4)]
    for i in range(4):
        for j in range(4):
            acc: Poly = {}
            for k in range(4):
                acc = padd(acc, pmul(A[i][k], B[k][j]))
            C[i][j] = acc
    return C


def mat(entries) -> Mat:
    """Build from a 4x4 nested list whose items are Poly, 0 or 1."""
    def conv(e):
        if isinstance(e, dict):
            return dict(e)
        return dict(ONE) if e == 1 else {}
    return [[conv(e) for e in row] for row in entries]


# ---- the step matrices of the paper --------------------------------------

def T_H(P: Poly) -> Mat:
    return mat([[1, 0, 0, 0], [P, 1, 0, 0], [0, 0, 1, 0], [0, 0, P, 1]])


def T_V(P: Poly) -> Mat:
    Ps = star(P)
    return mat([[1, 0, 0, 0], [0, 1, 0, 0], [Ps, 0, 1, 0], [0, Ps, 0, 1]])


def S_H(U: Poly) -> Mat:
    return mat([[1, U, 0, 0], [0, 1, 0, 0], [0, 0, 1, U], [0, 0, 0, 1]])


def S_V(U: Poly) -> Mat:
    Us = star(U)
    return mat([[1, 0, Us, 0], [0, 1, 0, Us], [0, 0, 1, 0], [0, 0, 0, 1]])


def T_fused(P: Poly) -> Mat:
    """Spatial predict of the non-separable lifting scheme."""
    Ps = star(P)
    return mat([[1, 0, 0, 0], [P, 1, 0, 0], [Ps, 0, 1, 0], [pmul(P, Ps), Ps, P, 1]])


def S_fused(U: Poly) -> Mat:
    """Spatial update of the non-separable lifting scheme."""
    Us = star(U)
    return mat([[1, U, Us, pmul(U, Us)], [0, 1, 0, Us], [0, 0, 1, U], [0, 0, 0, 1]])


def N_polyconv(P: Poly, U: Poly) -> Mat:
    """Non-separable polyconvolution N_{P,U} with V = P U + 1."""
    V = padd(pmul(P, U), ONE)
    Vs, Us, Ps = star(V), star(U), star(P)
    return mat([[pmul(Vs, V), pmul(Vs, U), pmul(Us, V), pmul(Us, U)],
                [pmul(Vs, P), Vs, pmul(Us, P), Us],
                [pmul(Ps, V), pmul(Ps, U), V, U],
                [pmul(Ps, P), Ps, P, 1]])


def equal(A: Mat, B: Mat) -> bool:
    return all(poly(A[i][j].items()) == poly(B[i][j].items()) for i in range(4) for j in range(4))


def ops(M: Mat) -> int:
    """Polynomial terms of a matrix, excluding the unit diagonal."""
    n = 0
    for i in range(4):
        for j in range(4):
            terms = dict(M[i][j])
            if i == j and terms.get((0, 0)) == 1:
                del terms[(0, 0)]
            n += len(terms)
    return n


# ---- the lifting polynomials of the paper's three wavelets ---------------

def wavelet_pairs(name: str):
    """[(P, U), ...] with P(z) acting on even samples to predict odd ones.

    CDF 5/3 and DD 13/7 use their textbook lifting filters; for CDF 9/7 only
    the term structure matters for counting (two 2-tap pairs), so symbolic
    unit coefficients are used."""
    if name == "cdf53":
        return [(horizontal([(0, Fraction(-1, 2)), (1, Fraction(-1, 2))]),
                 horizontal([(0, Fraction(1, 4)), (-1, Fraction(1, 4))]))]
    if name == "cdf97":
        P = horizontal([(0, 1), (1, 1)])
        U = horizontal([(0, 1), (-1, 1)])
        return [(P, U), (P, U)]
    if name == "dd137":
        P = horizontal([(-1, Fraction(-1, 16)), (0, Fraction(9, 16)),
                        (1, Fraction(9, 16)), (2, Fraction(-1, 16))])
        U = horizontal([(-2, Fraction(-1, 32)), (-1, Fraction(9, 32)),
                        (0, Fraction(9, 32)), (1, Fraction(-1, 32))])
        return [(P, U)]
    raise ValueError(name)


def split_constant(G: Poly):
    """G = G0 + G1 with G0 the constant (z^0) term."""
    G0 = {k: v for k, v in G.items() if k == (0, 0)}
    G1 = {k: v for k, v in G.items() if k != (0, 0)}
    return G0, G1


def scheme_steps(scheme: str, name: str):
    """A scheme as a list of steps; each step is the list of matrices that
    run between two barriers."""
    steps = []
    pairs = wavelet_pairs(name)
    if scheme == "separable-lifting":
        for P, U in pairs:
            steps += [[T_H(P)], [T_V(P)], [S_H(U)], [S_V(U)]]
    elif scheme == "nonseparable-lifting":
        for P, U in pairs:
            steps += [[T_fused(P)], [S_fused(U)]]
    elif scheme == "nonseparable-lifting-optimized":
        # The constant parts are separable lifting with no neighbour access:
        # they run inside the step that precedes the next barrier.
        for P, U in pairs:
            P0, P1 = split_constant(P)
            U0, U1 = split_constant(U)
            steps += [[T_H(P0), T_V(P0), T_fused(P1)],
                      [S_H(U0), S_V(U0), S_fused(U1)]]
    else:
        raise ValueError(scheme)
    return steps


def count(scheme: str, name: str):
    """(steps, operations) of a scheme."""
    st = scheme_steps(scheme, name)
    return len(st), sum(ops(M) for step in st for M in step)


def product(step_list) -> Mat:
    """The overall matrix of a step list (later steps multiply on the left)."""
    M = eye()
    for step in step_list:
        for A in step:
            M = matmul(A, M)
    return M
