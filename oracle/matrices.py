"""One-dimensional Gram matrices of B-splines (paper eqs. space_mat, time_mat and Section 5).

Test infrastructure: see the package docstring.

All integrals use the element-wise Gauss-Legendre rule with q points per
non-empty knot interval (q = p + 1 by default, which integrates every product
of two degree-p spline derivatives exactly).
"""
from __future__ import annotations

import numpy as np

from .bspline import basis, gauss_rule


def gram_1d(knots, p: int, q: int | None = None) -> dict:
    """Full m x m matrices X[a,b][i,j] = int b_i^(a) b_j^(b) for a, b in {0, 1, 2}.

    Keys: "M" = (0,0) mass, "L" = (1,1) stiffness, "J" = (2,2) second-derivative
    Gram matrix, "G" with G[i,j] = int b_j' b_i (so that the time matrix
    W_t of eq. time_mat equals i*G), and "D20"/"D02" with D20[i,j] = int b_i'' b_j.
    """
    q = p + 1 if q is None else q
    x, w, _ = gauss_rule(knots, q)
    B = basis(knots, p, x, nder=2)

    def g(a, b):
        return (B[a] * w[None, :]) @ B[b].T

    return {"M": g(0, 0), "L": g(1, 1), "J": g(2, 2), "G": g(0, 1),
            "D20": g(2, 0), "D02": g(0, 2)}


def space_1d(knots, p: int, q: int | None = None) -> dict:
    """Dirichlet-reduced spatial matrices (Section 3.2: drop the first and last function).

    Returns M, L, J and D20 restricted to indices 2..m-1 (1-based), i.e. the
    hat-matrices of eq. prec_definition for one direction.
    """
    full = gram_1d(knots, p, q)
    s = slice(1, -1)
    return {k: v[s, s].copy() for k, v in full.items()}


def time_1d(knots_t, p_t: int, q: int | None = None, final: bool = False) -> dict:
    """Reduced time matrices of eq. time_mat (Section 3.2: drop the first function, u(0) = 0;
    final=True: drop the last one, w(T) = 0, the test space of the ultraweak method of Section 4.4).

    M_t[i,j] = int b_i b_j, L_t[i,j] = int b_j' b_i', W_t[i,j] = i int b_j' b_i,
    and T3 = W_t + W_t^* (the time factor of the third Kronecker term).
    """
    full = gram_1d(knots_t, p_t, q)
    s = slice(None, -1) if final else slice(1, None)
    M, L, G = full["M"][s, s], full["L"][s, s], full["G"][s, s]
    W = 1j * G
    return {"M": M.copy(), "L": L.copy(), "W": W, "T3": W + W.conj().T}
