"""Load vector, lifting of initial/boundary data, and error norms (Sections 2.2, 4.3).

Test infrastructure: see the package docstring.

Space-time fields sampled at quadrature points are arrays of shape
(Q_d, ..., Q_1, Q_t) and coefficient tensors have shape (m_d, ..., m_1, m_t)
(full basis) or (n_d, ..., n_1, n_t) (free basis), so that a C-order ravel
puts time fastest as in the paper's vec operator.

Lifting reading (the paper only states u = u_bar + u_bar_0, f_bar = f - S u_bar_0):
the fixed coefficients are those of every B-spline that does not vanish on
the Dirichlet part Gamma = {t = 0} x Omega  U  (0,T) x boundary(Omega); they are the
joint L2(Gamma) projection of the data (u0 on the initial face, the Dirichlet
trace on the lateral faces).  The free problem is then A u = (f - S u_bar, S B_I).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bspline import basis, gauss_rule
from .matrices import gram_1d
from .spatial import kron_seq


def along(X, axis, mat):
    """X x_axis mat: contract axis of X with the columns of mat (mat: new x old)."""
    return np.moveaxis(np.tensordot(mat, X, axes=([1], [axis])), 0, axis)


def apply_axes(X, mats):
    """Apply mats[a] along axis a for every axis with a matrix (None = identity)."""
    for a, m in enumerate(mats):
        if m is not None:
            X = along(X, a, m)
    return X


class SpaceTimeBasis:
    """Basis values at the tensor Gauss grid (q points per element and direction)."""

    def __init__(self, knots_t, knots_s, p_t, p_s, q=None, geometry=None):
        self.geometry = geometry
        self.d = len(knots_s)
        self.knots = [np.asarray(k, dtype=np.float64) for k in knots_s] + [np.asarray(knots_t, dtype=np.float64)]
        self.deg = [p_s] * self.d + [p_t]
        self.q = [(dg + 1 if q is None else q) for dg in self.deg]
        self.pts, self.wts, self.B = [], [], []
        for kn, dg, qq in zip(self.knots, self.deg, self.q):
            x, w, _ = gauss_rule(kn, qq)
            self.pts.append(x)
            self.wts.append(w)
            self.B.append(basis(kn, dg, x, nder=2))  # (3, m, Q)
        self.m = [b.shape[1] for b in self.B]

    # axis a of an array (x_d ... x_1 t): direction index dir_of_axis
    def axis(self, direction):
        """Array axis of spatial direction l (0-based) or of time (direction == 't')."""
        return self.d if direction == "t" else self.d - 1 - direction

    def grid(self):
        """Point arrays (t, x_1, ..., x_d) broadcast to shape (Q_d, ..., Q_1, Q_t)."""
        shape = [len(self.pts[l]) for l in reversed(range(self.d))] + [len(self.pts[self.d])]
        out = []
        for direction in ["t"] + list(range(self.d)):
            a = self.axis(direction)
            src = self.pts[self.d] if direction == "t" else self.pts[direction]
            s = [1] * (self.d + 1)
            s[a] = len(src)
            out.append(np.broadcast_to(src.reshape(s), shape))
        return out

    def space_grid(self):
        shape = [len(self.pts[l]) for l in reversed(range(self.d))]
        out = []
        for l in range(self.d):
            s = [1] * self.d
            s[self.d - 1 - l] = len(self.pts[l])
            out.append(np.broadcast_to(self.pts[l].reshape(s), shape))
        return out

    def physical_space_grid(self):
        """Physical coordinates of the spatial grid (the parametric ones when F = Id)."""
        xs = self.space_grid()
        if self.geometry is None:
            return xs
        Fx = self.geometry.F(xs[0], xs[1])
        return [Fx[..., 0], Fx[..., 1]]

    def jacobian(self):
        """|det DF| on the spatial grid, shape (Q_d, ..., Q_1, 1) (1 when F = Id)."""
        if self.geometry is None:
            return 1.0
        from .geometry import laplacian_coefficients
        xs = self.space_grid()
        return laplacian_coefficients(self.geometry, xs[0], xs[1])["J"][..., None]

    def laplacian_terms(self):
        """[(coefficient on the grid (broadcast over time), {direction: order})] with
        Lap_x = sum coefficient * derivative (parametric Laplacian when F = Id)."""
        if self.geometry is None:
            return [(1.0, {l: 2}) for l in range(self.d)]
        from .geometry import laplacian_coefficients
        xs = self.space_grid()
        cf = laplacian_coefficients(self.geometry, xs[0], xs[1])
        return [(cf["a11"][..., None], {0: 2}), (cf["a12"][..., None], {0: 1, 1: 1}),
                (cf["a22"][..., None], {1: 2}), (cf["b1"][..., None], {0: 1}), (cf["b2"][..., None], {1: 1})]

    def weights(self):
        W = np.ones([1] * (self.d + 1))
        for direction in ["t"] + list(range(self.d)):
            a = self.axis(direction)
            w = self.wts[self.d] if direction == "t" else self.wts[direction]
            s = [1] * (self.d + 1)
            s[a] = len(w)
            W = W * w.reshape(s)
        return W

    def mats(self, orders, rows=None, transpose=False):
        """Per-axis matrices: derivative orders (dict direction->order, default 0)."""
        out = [None] * (self.d + 1)
        for direction in ["t"] + list(range(self.d)):
            idx = self.d if direction == "t" else direction
            Bm = self.B[idx][orders.get(direction, 0)]
            if rows is not None:
                Bm = Bm[rows[direction]]
            out[self.axis(direction)] = Bm.T if transpose else Bm
        return out

    def free_rows(self):
        r = {"t": slice(1, None)}
        for l in range(self.d):
            r[l] = slice(1, -1)
        return r


def load_vector(stb: SpaceTimeBasis, Fq, nu, Vq=None):
    """f_I = (F, S_V B_I) over the free basis (Section 4.3, load vector with S_V = S + V).

    conj(S_V B_I) = -i b_t' phi - nu b_t Lap phi + V b_t phi (B-splines are real).
    Fq: samples at the tensor grid, shape (Q_d, ..., Q_1, Q_t).  Vq: (Q_d, ..., Q_1) or None.
    Returns an array of shape (n_d, ..., n_1, n_t).
    """
    Fw = Fq * stb.weights() * stb.jacobian()
    rows = stb.free_rows()
    out = -1j * apply_axes(Fw, stb.mats({"t": 1}, rows))
    for coef, orders in stb.laplacian_terms():
        out = out - nu * apply_axes(coef * Fw, stb.mats(orders, rows))
    if Vq is not None:
        out = out + apply_axes(Fw * Vq[..., None], stb.mats({}, rows))
    return out


def evaluate(stb: SpaceTimeBasis, C, nu, Vq=None):
    """Values of u = sum C_I B_I and of S_V u at the grid (C over the full basis)."""
    u = apply_axes(C, stb.mats({}, transpose=True))
    Su = 1j * apply_axes(C, stb.mats({"t": 1}, transpose=True))
    for coef, orders in stb.laplacian_terms():
        Su = Su - nu * coef * apply_axes(C, stb.mats(orders, transpose=True))
    if Vq is not None:
        Su = Su + Vq[..., None] * u
    return u, Su


def fixed_mask(m_space, m_t):
    """Boolean tensor (m_d, ..., m_1, m_t): basis functions not vanishing on Gamma."""
    d = len(m_space)
    mask = np.zeros(tuple(reversed(m_space)) + (m_t,), dtype=bool)
    mask[..., 0] = True
    for l in range(d):
        a = d - 1 - l
        idx = [slice(None)] * (d + 1)
        idx[a] = 0
        mask[tuple(idx)] = True
        idx[a] = m_space[l] - 1
        mask[tuple(idx)] = True
    return mask


def lifting(stb: SpaceTimeBasis, u0=None, dirichlet=None):
    """Joint L2(Gamma) projection of the initial and Dirichlet data (reading stated above).

    u0(x_1..x_d) and dirichlet(t, x_1..x_d) are callables or None (zero data).
    Returns the full coefficient tensor with zeros at free positions.
    """
    d = stb.d
    m_s, m_t = stb.m[:d], stb.m[d]
    Mfull = [gram_1d(stb.knots[l], stb.deg[l], stb.q[l])["M"] for l in range(d + 1)]
    N = int(np.prod(m_s)) * m_t
    E0 = sp.csr_matrix(([1.0], ([0], [0])), shape=(m_t, m_t))
    Mg = sp.kron(kron_seq(Mfull[:d], sparse=True), E0, format="csr")
    rhs = np.zeros(tuple(reversed(m_s)) + (m_t,), dtype=np.complex128)
    # initial face t = 0: traces phi_I for i_t = 0
    if u0 is not None:
        xs = stb.physical_space_grid()
        ws = np.ones([1] * d)
        for l in range(d):
            s = [1] * d
            s[d - 1 - l] = len(stb.wts[l])
            ws = ws * stb.wts[l].reshape(s)
        vals = u0(*xs) * ws
        rhs[..., 0] += apply_axes(vals, [stb.B[l][0] for l in reversed(range(d))])
    # lateral faces x_l = side
    for l in range(d):
        for side, end in ((0, 0), (1, m_s[l] - 1)):
            El = sp.csr_matrix(([1.0], ([end], [end])), shape=(m_s[l], m_s[l]))
            factors = [El if k == l else Mfull[k] for k in range(d)]
            Mg = Mg + sp.kron(kron_seq(factors, sparse=True), sp.csr_matrix(Mfull[d]), format="csr")
            if dirichlet is None:
                continue
            # face grid: (Q_d..Q_1 without l, Q_t)
            tgrid = stb.grid()
            sl = [slice(None)] * (d + 1)
            sl[d - 1 - l] = slice(0, 1)
            pts = [g[tuple(sl)] for g in tgrid]
            pts[1 + l] = np.full_like(pts[1 + l], float(side) * stb.knots[l][-1])
            # face weights: every direction except l
            W = np.ones([1] * (d + 1))
            for direction in ["t"] + [k for k in range(d) if k != l]:
                a = stb.axis(direction)
                w = stb.wts[d] if direction == "t" else stb.wts[direction]
                s = [1] * (d + 1)
                s[a] = len(w)
                W = W * w.reshape(s)
            vals = dirichlet(*pts) * W
            mats = stb.mats({})
            mats[d - 1 - l] = np.zeros((m_s[l], 1))
            mats[d - 1 - l][end, 0] = 1.0
            rhs += apply_axes(vals, mats)
    mask = fixed_mask(m_s, m_t).ravel()
    idx = np.nonzero(mask)[0]
    Mff = Mg[idx][:, idx].tocsc()
    g = spla.spsolve(Mff, rhs.ravel()[idx])
    G = np.zeros(N, dtype=np.complex128)
    G[idx] = g
    return G.reshape(rhs.shape)


def assemble_rhs(stb: SpaceTimeBasis, nu, f=None, u0=None, dirichlet=None, V=None):
    """Free right-hand side f_bar = (f - S_V u_bar, S_V B_I) and the lifting tensor.

    f(t, x_1..x_d), u0, dirichlet and V(x_1..x_d) are callables or None.
    Returns (f_bar flattened time-fastest, lifting tensor G).
    """
    tg = stb.grid()
    if stb.geometry is not None and (f is not None or dirichlet is not None):
        raise NotImplementedError("mapped domains: f = 0 and homogeneous Dirichlet data only")
    Fq = f(*tg) if f is not None else np.zeros(tg[0].shape, dtype=np.complex128)
    Vq = V(*stb.physical_space_grid()) if V is not None else None
    G = lifting(stb, u0, dirichlet)
    _, SG = evaluate(stb, G, nu, Vq)
    fbar = load_vector(stb, Fq - SG, nu, Vq)
    return fbar.reshape(-1), G


def full_coefficients(G, x_free, n_s, n_t):
    """Full tensor = lifting G plus the free solution scattered into the interior."""
    C = G.copy()
    d = C.ndim - 1
    sl = tuple([slice(1, -1)] * d) + (slice(1, None),)
    C[sl] += np.asarray(x_free).reshape(tuple(reversed(n_s)) + (n_t,))
    return C


def errors_separable(knots_t, knots_s, p_t, p_s, C, nu, space_factors, time_u, time_f, q_extra=1):
    """errors() for one space dimension (V = 0) and an exact solution given as a finite series
    u = sum_k a_k(t) e_k(x), S u = f = sum_k c_k(t) e_k(x): space_factors(x) -> e_k(x_q) (Q_x x M),
    time_u(t) / time_f(t) -> a_k(t_q) / c_k(t_q) (Q_t x M).  The exact values on the tensor grid
    are the products E_x A_t^T and E_x C_t^T; everything else is errors().
    """
    assert len(knots_s) == 1
    stb = SpaceTimeBasis(knots_t, knots_s, p_t, p_s, q=max(p_t, p_s) + 1 + q_extra)
    uh, Suh = evaluate(stb, C, nu, None)
    Ex = space_factors(stb.pts[0])
    W = stb.weights()
    e = Ex @ time_u(stb.pts[1]).T - uh
    l2 = np.sqrt(np.sum(W * np.abs(e) ** 2))
    del e
    Se = Ex @ time_f(stb.pts[1]).T - Suh
    vn = np.sqrt(l2 ** 2 + np.sum(W * np.abs(Se) ** 2))
    return l2, vn


def errors(knots_t, knots_s, p_t, p_s, C, nu, exact_u, exact_f, V=None, q_extra=1):
    """L2(Q) error and V-norm error ||e||_V^2 = ||e||^2 + ||S_V e||^2 (Section 2.1).

    Evaluated with p+1+q_extra Gauss points per element; exact_f = S_V u_exact.
    """
    stb = SpaceTimeBasis(knots_t, knots_s, p_t, p_s, q=max(p_t, p_s) + 1 + q_extra)
    Vq = V(*stb.space_grid()) if V is not None else None
    uh, Suh = evaluate(stb, C, nu, Vq)
    tg = stb.grid()
    W = stb.weights()
    e = exact_u(*tg) - uh
    Se = exact_f(*tg) - Suh
    l2 = np.sqrt(np.sum(W * np.abs(e) ** 2))
    vn = np.sqrt(l2 ** 2 + np.sum(W * np.abs(Se) ** 2))
    return l2, vn
