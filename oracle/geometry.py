"""Mapped spatial domains: the quarter annulus and the physical Laplacian in parametric form.

Test infrastructure: see the package docstring.

Section 3.1 allows a physical domain Omega = F(Omega_hat) given by a map from the
parametric square; the paper's tests all use F = Id.  Here F is the quarter annulus
x = (r0 + (r1 - r0) xi_1) c(xi_2), with c the quarter circle written as a rational
quadratic curve (control points (1,0), (1,1), (0,1), weights 1, 1/sqrt(2), 1), which
is exact.

The physical derivatives of a function u(F(xi)) follow from the general chain rule
(no use of the orthogonality of this particular map):
    grad_x u = DF^{-T} grad_xi u,
    Hess_x u = DF^{-T} (Hess_xi u - sum_k (grad_x u)_k Hess_xi F_k) DF^{-1},
so Lap_x u = sum_{ab} G_ab u_{xi_a xi_b} + sum_a beta_a u_{xi_a} with the inverse metric
G = DF^{-1} DF^{-T} and beta_a = - sum_k (DF^{-1})_{ak} tr(G Hess_xi F_k).

Spatial factors on the mapped domain (reading: the cross term with the time
derivative is written with int grad phi_I . grad phi_J dx, the form that integration
by parts gives for functions vanishing on the boundary):
    S_1 = int phi_I phi_J dx,  S_3 = nu int grad phi_I . grad phi_J dx + int V phi_I phi_J dx,
    S_2 = nu^2 int Lap phi_I Lap phi_J dx - nu int V (phi_I Lap phi_J + Lap phi_I phi_J) dx
          + int V^2 phi_I phi_J dx,
all with the element Gauss rule on the parametric square and dx = |det DF| dxi.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .spatial import _direction_data, interior_indices


class QuarterAnnulus:
    """x = (r0 + (r1 - r0) xi_1) c(xi_2), c the exact quadratic rational quarter circle."""

    def __init__(self, r0=1.0, r1=2.0):
        self.r0, self.r1 = float(r0), float(r1)
        w = 1.0 / np.sqrt(2.0)
        # homogeneous control points (w_i P_i, w_i) of the arc
        self.Pw = np.array([[1.0, 0.0, 1.0], [w, w, w], [0.0, 1.0, 1.0]])

    def _arc(self, t):
        """c(t), c'(t), c''(t) from the homogeneous Bernstein form C(t) = sum B_i(t) Pw_i."""
        t = np.asarray(t, dtype=np.float64)
        B = [(1 - t) ** 2, 2 * t * (1 - t), t ** 2]
        dB = [-2 * (1 - t), 2 - 4 * t, 2 * t]
        ddB = [2.0 + 0 * t, -4.0 + 0 * t, 2.0 + 0 * t]
        C = sum(B[i][..., None] * self.Pw[i] for i in range(3))
        dC = sum(dB[i][..., None] * self.Pw[i] for i in range(3))
        ddC = sum(ddB[i][..., None] * self.Pw[i] for i in range(3))
        A, W = C[..., :2], C[..., 2:]
        dA, dW = dC[..., :2], dC[..., 2:]
        ddA, ddW = ddC[..., :2], ddC[..., 2:]
        c = A / W
        dc = (dA - c * dW) / W
        ddc = (ddA - 2 * dc * dW - c * ddW) / W
        return c, dc, ddc

    def F(self, xi1, xi2):
        c, _, _ = self._arc(xi2)
        r = self.r0 + (self.r1 - self.r0) * np.asarray(xi1)
        return r[..., None] * c

    def derivatives(self, xi1, xi2):
        """F, DF[..., k, a] = dF_k/dxi_a, D2F[..., k, a, b] = d2F_k/dxi_a dxi_b."""
        xi1, xi2 = np.broadcast_arrays(np.asarray(xi1, float), np.asarray(xi2, float))
        c, dc, ddc = self._arc(xi2)
        dr = self.r1 - self.r0
        r = self.r0 + dr * xi1
        F = r[..., None] * c
        DF = np.stack([dr * c, r[..., None] * dc], axis=-1)
        D2F = np.zeros(xi1.shape + (2, 2, 2))
        D2F[..., :, 0, 1] = dr * dc
        D2F[..., :, 1, 0] = dr * dc
        D2F[..., :, 1, 1] = r[..., None] * ddc
        return F, DF, D2F


def laplacian_coefficients(geom, xi1, xi2):
    """Coefficients of Lap_x u = a11 u_11 + a12 u_12 + a22 u_22 + b1 u_1 + b2 u_2 and the
    gradient metric G (inverse metric) and J = |det DF| at parametric points (general chain rule)."""
    _, DF, D2F = geom.derivatives(xi1, xi2)
    Dinv = np.linalg.inv(DF)                          # [..., a, k]
    G = np.einsum("...ak,...bk->...ab", Dinv, Dinv)   # DF^{-1} DF^{-T}
    L = np.einsum("...ab,...kab->...k", G, D2F)       # tr(G Hess F_k)
    beta = -np.einsum("...ak,...k->...a", Dinv, L)
    J = np.abs(np.linalg.det(DF))
    return {"a11": G[..., 0, 0], "a12": 2 * G[..., 0, 1], "a22": G[..., 1, 1],
            "b1": beta[..., 0], "b2": beta[..., 1], "G": G, "J": J}


def mapped_spatial_factors(knots_list, p: int, nu: float, geom, V=None, q: int | None = None):
    """S_1, S_2, S_3 (sparse, Dirichlet-reduced) on the mapped 2D domain, by element quadrature.

    V: callable V(x, y) in physical coordinates, or None.
    """
    assert len(knots_list) == 2
    q = p + 1 if q is None else q
    dirs = [_direction_data(kn, p, q) for kn in knots_list]
    m = [len(kn) - p - 1 for kn in knots_list]
    n_el = [dd[1].shape[0] for dd in dirs]
    nl = p + 1
    blocks = {0: [], 1: [], 2: []}
    for e2, e1 in itertools.product(range(n_el[1]), range(n_el[0])):
        (f1, B1, x1, w1), (f2, B2, x2, w2) = dirs[0], dirs[1]
        X1, X2 = np.meshgrid(x1[e1], x2[e2], indexing="xy")        # (q2, q1) arrays, xi_1 fastest
        W = np.outer(w2[e2], w1[e1])
        cf = laplacian_coefficients(geom, X1, X2)
        Jw = (W * cf["J"]).ravel()
        # local functions phi_{a1, a2} = b1_a1 b2_a2, index a2 * nl + a1; derivatives (o1, o2)
        def D(o1, o2):
            return np.einsum("ai,bj->baji", B1[e1][o1], B2[e2][o2]).reshape(nl * nl, q * q)
        val = D(0, 0)
        d1, d2 = D(1, 0), D(0, 1)
        lap = (cf["a11"].ravel() * D(2, 0) + cf["a12"].ravel() * D(1, 1) + cf["a22"].ravel() * D(0, 2)
               + cf["b1"].ravel() * d1 + cf["b2"].ravel() * d2)
        G = cf["G"].reshape(-1, 2, 2)
        grad_dot = (d1 * (G[:, 0, 0] * Jw)) @ d1.T + (d1 * (G[:, 0, 1] * Jw)) @ d2.T \
            + (d2 * (G[:, 1, 0] * Jw)) @ d1.T + (d2 * (G[:, 1, 1] * Jw)) @ d2.T
        S1 = (val * Jw) @ val.T
        S3 = nu * grad_dot
        S2 = nu * nu * (lap * Jw) @ lap.T
        if V is not None:
            Fx = geom.F(X1, X2)
            Vq = np.asarray(V(Fx[..., 0], Fx[..., 1]), dtype=np.float64).ravel()
            S3 = S3 + (val * (Vq * Jw)) @ val.T
            KV = (val * (Vq * Jw)) @ lap.T        # int V phi_I Lap phi_J
            S2 = S2 - nu * (KV + KV.T) + (val * (Vq * Vq * Jw)) @ val.T
        a1 = f1[e1] + np.tile(np.arange(nl), nl)
        a2 = f2[e2] + np.repeat(np.arange(nl), nl)
        gidx = a1 + m[0] * a2
        for k, Sk in enumerate((S1, S2, S3)):
            blocks[k].append((np.repeat(gidx, len(gidx)), np.tile(gidx, len(gidx)), Sk.ravel()))
    N = m[0] * m[1]
    keep = interior_indices(m)
    out = []
    for k in range(3):
        r = np.concatenate([b[0] for b in blocks[k]])
        c = np.concatenate([b[1] for b in blocks[k]])
        v = np.concatenate([b[2] for b in blocks[k]])
        A = sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()
        out.append(A[keep][:, keep])
    return out
