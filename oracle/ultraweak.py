"""Ultraweak space-time method (Section 4.4, eq. uw-discrete-system).

Test infrastructure: see the package docstring.

Test space W_h: the isogeometric space with homogeneous Dirichlet data on the spatial boundary and
the final condition w(T) = 0 (time basis without its last function).  Trial space V_h = S_V(W_h):
the discrete solution is u_h = S_V z_h with z_h in W_h, and for every test function w_h

    (S_V z_h, S_V w_h) = (f, w_h) + i (u_0, w_h(., 0))_{L2(Omega)},

which follows from (S v, w) = (v, S w) - i (v(0), w(0)) for w(T) = 0 applied to the exact
solution.  The left side is the matrix of eq. syst_mat (with the potential terms) on the
final-condition time basis (oracle.operators.Problem(..., final=True)); the right side carries
the initial data instead of a lifting.  u_h is the L2(Q)-orthogonal projection of u onto
S_V(W_h) (the test in tests/test_oracle_ultraweak.py pins both sides against brute-force
quadrature of that projection).
"""
from __future__ import annotations

import numpy as np

from .rhs import SpaceTimeBasis, apply_axes


def free_rows(stb: SpaceTimeBasis):
    """Free functions of W_h: time without the last function, space without the boundary ones."""
    r = {"t": slice(None, -1)}
    for l in range(stb.d):
        r[l] = slice(1, -1)
    return r


def load_vector(stb: SpaceTimeBasis, f=None, u0=None):
    """F_I = (f, B_I) + i (u_0, B_I(., 0)) over the free basis of W_h (eq. uw-discrete-system).

    f(t, x_1..x_d) and u0(x_1..x_d) are callables or None (zero data); B-splines are real, so
    the conjugate of the test function is the function itself.  Of the time functions only the
    first is non-zero at t = 0 (open knot vector, value 1 there).  Returns (n_d, ..., n_1, n_t).
    """
    if stb.geometry is not None:
        raise NotImplementedError("ultraweak method: unit cube only")
    rows = free_rows(stb)
    shape = tuple(stb.m[l] - 2 for l in reversed(range(stb.d))) + (stb.m[stb.d] - 1,)
    out = np.zeros(shape, dtype=np.complex128)
    if f is not None:
        Fw = f(*stb.grid()) * stb.weights()
        out = out + apply_axes(Fw, stb.mats({}, rows))
    if u0 is not None:
        d = stb.d
        ws = np.ones([1] * d)
        for l in range(d):
            s = [1] * d
            s[d - 1 - l] = len(stb.wts[l])
            ws = ws * stb.wts[l].reshape(s)
        vals = u0(*stb.space_grid()) * ws
        out[..., 0] += 1j * apply_axes(vals, [stb.B[l][0][1:-1] for l in reversed(range(d))])
    return out


def full_tensor(stb: SpaceTimeBasis, z_free):
    """Coefficients of z_h over the full basis (zero on the Dirichlet and final-time functions)."""
    d = stb.d
    Z = np.zeros(tuple(stb.m[l] for l in reversed(range(d))) + (stb.m[d],), dtype=np.complex128)
    sl = tuple([slice(1, -1)] * d) + (slice(None, -1),)
    Z[sl] = np.asarray(z_free).reshape(Z[sl].shape)
    return Z


def solution_values(stb: SpaceTimeBasis, z_free, nu, Vq=None):
    """u_h = S_V z_h = i d_t z_h - nu Lap z_h + V z_h at the grid of stb (Vq on its spatial grid)."""
    Z = full_tensor(stb, z_free)
    u = 1j * apply_axes(Z, stb.mats({"t": 1}, transpose=True))
    for coef, orders in stb.laplacian_terms():
        u = u - nu * coef * apply_axes(Z, stb.mats(orders, transpose=True))
    if Vq is not None:
        u = u + Vq[..., None] * apply_axes(Z, stb.mats({}, transpose=True))
    return u


def l2_error(knots_t, knots_s, p_t, p_s, z_free, nu, exact_u, V=None, q_extra=1):
    """||u - S_V z_h||_{L2(Q)} with p+1+q_extra Gauss points per element and direction."""
    stb = SpaceTimeBasis(knots_t, knots_s, p_t, p_s, q=max(p_t, p_s) + 1 + q_extra)
    Vq = V(*stb.space_grid()) if V is not None else None
    uh = solution_values(stb, z_free, nu, Vq)
    e = exact_u(*stb.grid()) - uh
    return float(np.sqrt(np.sum(stb.weights() * np.abs(e) ** 2)))
