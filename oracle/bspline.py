"""B-spline basis by the Cox-de Boor recursion (paper Section 3.1).

Test infrastructure: see the package docstring.
"""
from __future__ import annotations

import numpy as np


def _ratio(num, den):
    """num/den with the Cox-de Boor convention 0/0 = 0 (den == 0 only for repeated knots)."""
    out = np.zeros(np.broadcast(num, den).shape)
    nz = den != 0
    out[..., nz] = (num[..., nz] if np.ndim(num) else num) / den[nz]
    return out


def basis(knots, p: int, x, nder: int = 2) -> np.ndarray:
    """Values and derivatives of all B-splines of degree p at points x.

    Section 3.1: degree-0 functions are interval indicators, degree k functions
    follow the Cox-de Boor recursion
        N_{i,k} = (x - xi_i)/(xi_{i+k} - xi_i) N_{i,k-1}
                + (xi_{i+k+1} - x)/(xi_{i+k+1} - xi_{i+1}) N_{i+1,k-1},
    and derivatives follow de Boor's formula
        N'_{i,k} = k/(xi_{i+k} - xi_i) N_{i,k-1} - k/(xi_{i+k+1} - xi_{i+1}) N_{i+1,k-1}
    applied recursively for higher derivatives.

    Returns an array of shape (nder+1, m, len(x)), m = len(knots) - p - 1.
    Points must lie in [knots[0], knots[-1]]; the right end point is assigned to
    the last non-empty knot interval.
    """
    kn = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nk = len(kn)
    # degree 0 indicators
    N0 = ((kn[:-1, None] <= x[None, :]) & (x[None, :] < kn[1:, None])).astype(np.float64)
    last = np.max(np.nonzero(kn[1:] > kn[:-1])[0])
    N0[last, x == kn[-1]] = 1.0
    # table[k] = (nk - 1 - k, nx) values of degree k
    table = [N0]
    for k in range(1, p + 1):
        prev = table[-1]
        i = np.arange(nk - 1 - k)
        left = _ratio(x[None, :] - kn[i, None], (kn[i + k] - kn[i])[:, None] + 0 * x[None, :])
        right = _ratio(kn[i + k + 1, None] - x[None, :], (kn[i + k + 1] - kn[i + 1])[:, None] + 0 * x[None, :])
        table.append(left * prev[:-1] + right * prev[1:])
    m = nk - p - 1
    out = np.zeros((nder + 1, m, len(x)))
    out[0] = table[p]
    # The r-th derivative of N_{i,p} is a combination sum_j a_j[i] N_{i+j,p-r};
    # each differentiation step applies de Boor's formula to every term.
    a = [np.ones(m)]
    for r in range(1, min(nder, p) + 1):
        k = p - r + 1  # degree of the terms being differentiated
        new = [np.zeros(m) for _ in range(r + 1)]
        for j, aj in enumerate(a):
            idx = np.arange(m) + j
            d1 = kn[idx + k] - kn[idx]
            d2 = kn[idx + k + 1] - kn[idx + 1]
            new[j] += aj * np.where(d1 != 0, k / np.where(d1 != 0, d1, 1.0), 0.0)
            new[j + 1] -= aj * np.where(d2 != 0, k / np.where(d2 != 0, d2, 1.0), 0.0)
        a = new
        low = table[p - r]
        out[r] = sum(aj[:, None] * low[np.arange(m) + j] for j, aj in enumerate(a))
    return out


def breakpoints(knots) -> np.ndarray:
    """Knots without repetition (the breakpoints Z of Section 3.1)."""
    return np.unique(np.asarray(knots, dtype=np.float64))


def greville(knots, p: int) -> np.ndarray:
    """Greville abscissae (mean of p consecutive interior knots) for each basis function."""
    kn = np.asarray(knots, dtype=np.float64)
    m = len(kn) - p - 1
    return np.array([kn[i + 1:i + p + 1].mean() for i in range(m)])


def gauss_rule(knots, q: int):
    """Element-wise Gauss-Legendre rule with q points on every non-empty knot interval.

    Returns points (n_el*q,), weights (n_el*q,) and the element index of each point.
    """
    z = breakpoints(knots)
    xg, wg = np.polynomial.legendre.leggauss(q)
    a, b = z[:-1], z[1:]
    pts = (0.5 * (a + b))[:, None] + (0.5 * (b - a))[:, None] * xg[None, :]
    wts = (0.5 * (b - a))[:, None] * wg[None, :]
    el = np.repeat(np.arange(len(a)), q)
    return pts.ravel(), wts.ravel(), el
