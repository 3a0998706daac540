"""Pins of the oracle's mapped-domain operators (quarter annulus, Section 3.1 mapped domains).

The map and its derivatives are pinned by closed forms and finite differences, the chain
rule by functions with known Laplacians, the assembly by the identity map (where it must
equal the unit-square operators) and by the integration-by-parts identity that links the
gradient form of S_3 to the Laplacian form of K_V.
"""
import numpy as np
import pytest

from oracle.bspline import basis, gauss_rule
from oracle.geometry import QuarterAnnulus, laplacian_coefficients, mapped_spatial_factors
from oracle.operators import Problem
from oracle.spatial import system_spatial_factors
from paper_2311_18461_amd import inputs


class IdentityMap:
    """F = Id on the unit square."""

    def F(self, xi1, xi2):
        return np.stack(np.broadcast_arrays(np.asarray(xi1, float), np.asarray(xi2, float)), axis=-1)

    def derivatives(self, xi1, xi2):
        F = self.F(xi1, xi2)
        DF = np.zeros(F.shape[:-1] + (2, 2))
        DF[..., 0, 0] = DF[..., 1, 1] = 1.0
        return F, DF, np.zeros(F.shape[:-1] + (2, 2, 2))


def test_arc_is_the_quarter_circle():
    g = QuarterAnnulus(1.0, 2.0)
    t = np.linspace(0.0, 1.0, 101)
    c, _, _ = g._arc(t)
    assert np.max(np.abs(np.linalg.norm(c, axis=-1) - 1.0)) < 1e-15
    ang = np.arctan2(c[:, 1], c[:, 0])
    assert np.all(np.diff(ang) > 0) and abs(ang[0]) < 1e-15 and abs(ang[-1] - np.pi / 2) < 1e-15
    assert np.allclose(g.F(0.0, 0.0), [1, 0]) and np.allclose(g.F(1.0, 0.0), [2, 0])
    assert np.allclose(g.F(0.0, 1.0), [0, 1]) and np.allclose(g.F(1.0, 1.0), [0, 2])
    assert np.allclose(g.F(0.5, 0.5), 1.5 * np.array([1, 1]) / np.sqrt(2))  # symmetric weights


def test_map_derivatives_match_finite_differences():
    g = QuarterAnnulus(1.0, 2.0)
    rng = np.random.default_rng(0)
    h = 1e-4
    for _ in range(10):
        x1, x2 = rng.uniform(0.05, 0.95, 2)
        _, DF, D2F = g.derivatives(np.array(x1), np.array(x2))
        for a, (d1, d2) in enumerate(((h, 0), (0, h))):
            fd = (g.F(x1 + d1, x2 + d2) - g.F(x1 - d1, x2 - d2)) / (2 * h)
            assert np.allclose(fd, DF[:, a], atol=1e-8)
            _, DFp, _ = g.derivatives(np.array(x1 + d1), np.array(x2 + d2))
            _, DFm, _ = g.derivatives(np.array(x1 - d1), np.array(x2 - d2))
            assert np.allclose((DFp - DFm) / (2 * h), D2F[:, :, a], atol=1e-7)


def test_area_and_jacobian():
    g = QuarterAnnulus(1.0, 2.0)
    kn = inputs.uniform_open_knots(8, 2)
    x, w, _ = gauss_rule(kn, 10)
    X1, X2 = np.meshgrid(x, x, indexing="xy")
    J = laplacian_coefficients(g, X1, X2)["J"]
    area = np.sum(np.outer(w, w) * J)
    assert abs(area - 0.75 * np.pi) < 1e-13


@pytest.mark.parametrize("name", ["r2", "harm3", "expsin", "xy2"])
def test_chain_rule_laplacian_of_known_functions(name):
    """Pull u(x) back to the parametric square by the forward chain rule and recover Lap_x u."""
    g = QuarterAnnulus(1.0, 2.0)
    rng = np.random.default_rng(1)
    xi1, xi2 = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    F, DF, D2F = g.derivatives(xi1, xi2)
    x, y = F[..., 0], F[..., 1]
    # u, grad_x u, Hess_x u, Lap_x u in closed form
    if name == "r2":
        gu = np.stack([2 * x, 2 * y], -1); H = np.zeros(x.shape + (2, 2)); H[..., 0, 0] = H[..., 1, 1] = 2; lap = 4 + 0 * x
    elif name == "harm3":
        gu = np.stack([3 * x ** 2 - 3 * y ** 2, -6 * x * y], -1)
        H = np.stack([np.stack([6 * x, -6 * y], -1), np.stack([-6 * y, -6 * x], -1)], -2); lap = 0 * x
    elif name == "expsin":
        gu = np.stack([np.exp(x) * np.sin(y), np.exp(x) * np.cos(y)], -1)
        H = np.stack([np.stack([np.exp(x) * np.sin(y), np.exp(x) * np.cos(y)], -1),
                      np.stack([np.exp(x) * np.cos(y), -np.exp(x) * np.sin(y)], -1)], -2); lap = 0 * x
    else:
        gu = np.stack([y ** 2, 2 * x * y], -1)
        H = np.stack([np.stack([0 * x, 2 * y], -1), np.stack([2 * y, 2 * x], -1)], -2); lap = 2 * x
    # forward chain rule: parametric gradient and Hessian of u(F(xi))
    g_xi = np.einsum("...ka,...k->...a", DF, gu)
    H_xi = np.einsum("...ka,...kl,...lb->...ab", DF, H, DF) + np.einsum("...k,...kab->...ab", gu, D2F)
    cf = laplacian_coefficients(g, xi1, xi2)
    got = (cf["a11"] * H_xi[..., 0, 0] + cf["a12"] * H_xi[..., 0, 1] + cf["a22"] * H_xi[..., 1, 1]
           + cf["b1"] * g_xi[..., 0] + cf["b2"] * g_xi[..., 1])
    assert np.max(np.abs(got - lap)) < 1e-11


@pytest.mark.parametrize("with_V", [False, True])
def test_identity_map_reproduces_unit_square_factors(with_V):
    kn = [inputs.uniform_open_knots(5, 3), inputs.graded_open_knots(6, 3, 1.2)]
    V = inputs.gaussian_potential(2, 31) if with_V else None
    ref = system_spatial_factors(kn, 3, 1.3, V, sparse=True)
    got = mapped_spatial_factors(kn, 3, 1.3, IdentityMap(), V)
    for a, b in zip(got, ref):
        assert abs(a - b).max() <= 1e-12 * abs(b).max()


def test_gradient_form_equals_minus_laplacian_form():
    """Integration by parts on the annulus: int phi_I Lap phi_J dx = - int grad phi_I . grad phi_J dx,
    read off S_2 with V = 1 (K_V = int phi_I Lap phi_J) against S_3 with V = 0 (fine quadrature)."""
    g = QuarterAnnulus(1.0, 2.0)
    kn = [inputs.uniform_open_knots(4, 3)] * 2
    one = lambda x, y: np.ones_like(x)  # noqa: E731
    S1, S2_0, S3_0 = mapped_spatial_factors(kn, 3, 1.0, g, None, q=14)
    _, S2_1, S3_1 = mapped_spatial_factors(kn, 3, 1.0, g, one, q=14)
    KKt = (S1 - (S2_1 - S2_0)).toarray()         # K + K^T
    L = S3_0.toarray()
    assert np.max(np.abs(KKt + 2 * L)) < 1e-9 * np.max(np.abs(L))
    assert np.max(np.abs((S3_1 - S3_0).toarray() - S1.toarray())) < 1e-14


def test_annulus_system_is_hermitian_positive_definite():
    g = QuarterAnnulus(1.0, 2.0)
    kn = inputs.uniform_open_knots(3, 3)
    V = lambda x, y: 20 * np.exp(-((x - 1) ** 2 + (y - 1) ** 2) / 0.1)  # noqa: E731
    pr = Problem(kn, [kn, kn], 3, 3, 1.0, V, geometry=g)
    A = pr.dense_A()
    assert np.max(np.abs(A - A.conj().T)) < 1e-12 * np.max(np.abs(A))
    assert np.linalg.eigvalsh(A).min() > 0
    for S in pr.S:
        Sd = S.toarray()
        assert np.max(np.abs(Sd - Sd.T)) < 1e-12 * np.max(np.abs(Sd))


def test_mapped_fd_inverts_the_dense_mapped_preconditioner():
    """The oracle's mapped FD (one dense 2D eigenproblem) equals the inverse of eq. prec_definition
    written with the physical M and L."""
    from oracle.operators import MappedFastDiagonalization, dense_P_mapped
    g = QuarterAnnulus(1.0, 2.0)
    kn = inputs.uniform_open_knots(3, 3)
    pr = Problem(kn, [kn, kn], 3, 3, 1.0, None, geometry=g)
    P = dense_P_mapped(pr)
    r = inputs.random_complex(pr.N, 4)
    s = MappedFastDiagonalization(pr).apply(r)
    assert np.linalg.norm(P @ s - r) < 1e-11 * np.linalg.norm(r)
    assert np.max(np.abs(P - P.conj().T)) < 1e-12 * np.max(np.abs(P))


# ---------------------------------------------------------------------------------------------
# Mapped-domain right-hand side (Section 2.2 lifting, Section 4.3 load vector) by brute force.
# Nothing below uses the oracle's chain rule, Jacobian or Kronecker assembly: the map and its
# inverse are written here from the arc's definition (rational quadratic Bernstein form with
# weights 1, 1/sqrt(2), 1), every physical Laplacian is a fourth-order finite difference in
# physical coordinates through the inverse map, and the measure is the determinant of a
# finite-difference Jacobian.  Only the 1D B-spline values (pinned in test_oracle_bspline) and
# NumPy's Gauss-Legendre nodes are shared.
# ---------------------------------------------------------------------------------------------

_W = 1.0 / np.sqrt(2.0)


def _arc_point(t):
    """Quarter circle as a rational quadratic: control points (1,0), (1,1), (0,1), weights 1, w, 1."""
    b0, b1, b2 = (1 - t) ** 2, 2 * t * (1 - t) * _W, t ** 2
    den = b0 + b1 + b2
    return (b0 + b1) / den, (b1 + b2) / den


def _map(xi1, xi2, r0=1.0, r1=2.0):
    cx, cy = _arc_point(xi2)
    r = r0 + (r1 - r0) * xi1
    return r * cx, r * cy


def _inverse_map(x, y, r0=1.0, r1=2.0):
    """xi = F^{-1}(x): radius gives xi_1; the arc parameter solves tan(angle) = c_y(t) / c_x(t), which
    with s = t / (1 - t) is the quadratic s^2 + sqrt(2) (1 - T) s - T = 0, T = y / x."""
    xi1 = (np.hypot(x, y) - r0) / (r1 - r0)
    T = y / x
    s = 0.5 * (-np.sqrt(2.0) * (1 - T) + np.sqrt(2.0 * (1 - T) ** 2 + 4 * T))
    return xi1, s / (1 + s)


def _spatial_values(kn, p, xi1, xi2):
    """phi_{i1,i2}(xi) for every spatial B-spline, shape (m2, m1) + xi.shape."""
    sh = np.shape(xi1)
    b1 = basis(kn, p, np.ravel(xi1), 0)[0]
    b2 = basis(kn, p, np.ravel(xi2), 0)[0]
    return np.einsum("jq,iq->jiq", b2, b1).reshape((b2.shape[0], b1.shape[0]) + sh)


def _physical_laplacian(kn, p, x, y, h=1e-3):
    """Lap_x of phi(F^{-1}(x)) by the fourth-order five-point second difference along x and y."""
    c = (-1.0 / 12, 4.0 / 3, -5.0 / 2, 4.0 / 3, -1.0 / 12)
    lap = 0.0
    for dx, dy in ((1.0, 0.0), (0.0, 1.0)):
        for k, ck in zip(range(-2, 3), c):
            a, b = _inverse_map(x + k * h * dx, y + k * h * dy)
            lap = lap + ck * _spatial_values(kn, p, a, b)
    return lap / (h * h)


def _jacobian_det(xi1, xi2, h=1e-4):
    c = (1.0 / 12, -2.0 / 3, 0.0, 2.0 / 3, -1.0 / 12)
    D = np.zeros(np.shape(xi1) + (2, 2))
    for a, (d1, d2) in enumerate(((1.0, 0.0), (0.0, 1.0))):
        for k, ck in zip(range(-2, 3), c):
            fx, fy = _map(xi1 + k * h * d1, xi2 + k * h * d2)
            D[..., 0, a] += ck * fx / h
            D[..., 1, a] += ck * fy / h
    return np.abs(np.linalg.det(D))


def _element_gauss(kn, q):
    z = np.unique(kn)
    g, w = np.polynomial.legendre.leggauss(q)
    pts = (0.5 * (z[:-1] + z[1:]))[:, None] + (0.5 * np.diff(z))[:, None] * g[None, :]
    return pts.ravel(), ((0.5 * np.diff(z))[:, None] * w[None, :]).ravel()


def test_annulus_right_hand_side_brute_force():
    """f_bar_I = int (f - S_V u_bar) conj(S_V B_I) dx dt on the quarter annulus, with f = 0 and the lifting
    u_bar of a wave packet, against the oracle's sum-factorised assembly (chain rule, Kronecker lifting)."""
    from oracle.rhs import SpaceTimeBasis, assemble_rhs, fixed_mask
    p, n_el_s, n_el_t, nu = 3, 3, 2, 1.0
    ks = inputs.uniform_open_knots(n_el_s, p)
    kt = inputs.uniform_open_knots(n_el_t, p)
    V, u0 = inputs.annulus_sample(5003)
    u0.sigma = 0.4  # a broad packet: every spatial function sees the datum on this coarse grid
    stb = SpaceTimeBasis(kt, [ks, ks], p, p, geometry=QuarterAnnulus(1.0, 2.0))
    fbar, G = assemble_rhs(stb, nu, u0=u0, V=V)

    # 1) the lifting: joint L2 projection onto the functions not vanishing on Gamma (initial face and
    #    lateral faces), parametric measure, data u0 at the mapped points, zero lateral data; dense
    m, mt = len(ks) - p - 1, len(kt) - p - 1
    mask = fixed_mask([m, m], mt)                       # (m2, m1, mt)
    fixed = np.argwhere(mask)
    xq, wq = _element_gauss(ks, p + 1)
    tq, wt = _element_gauss(kt, p + 1)
    Bt = basis(kt, p, tq, 1)                            # (2, mt, Qt)
    X1, X2 = np.meshgrid(xq, xq, indexing="xy")         # (Q2, Q1)
    Ws = np.outer(wq, wq)
    phi = _spatial_values(ks, p, X1, X2)                # (m2, m1, Q2, Q1)
    b0 = basis(kt, p, np.array([0.0]), 0)[0][:, 0]      # time functions at t = 0
    nf = len(fixed)
    Gram = np.zeros((nf, nf))
    rhs = np.zeros(nf, dtype=np.complex128)
    ux, uy = _map(X1, X2)
    u0v = u0(ux, uy)
    for a, (j2, j1, jt) in enumerate(fixed):
        va = phi[j2, j1] * b0[jt]
        rhs[a] = np.sum(Ws * u0v * va)
        for b, (k2, k1, kt_) in enumerate(fixed):
            g = np.sum(Ws * va * phi[k2, k1] * b0[kt_])     # initial face
            # lateral faces xi_l in {0, 1}: trace of phi times the time Gram
            mt_gram = np.sum(wt * Bt[0, jt] * Bt[0, kt_])
            for l in range(2):
                for side in (0, m - 1):
                    if (j1 if l == 0 else j2) != side or (k1 if l == 0 else k2) != side:
                        continue
                    other_j, other_k = (j2, k2) if l == 0 else (j1, k1)
                    bo = basis(ks, p, xq, 0)[0]
                    g += mt_gram * np.sum(wq * bo[other_j] * bo[other_k])
            Gram[a, b] = g
    g_ref = np.linalg.solve(Gram, rhs)
    assert np.max(np.abs(G[mask] - g_ref)) < 1e-12 * np.max(np.abs(g_ref))

    # 2) the load vector by brute force over the space-time Gauss grid
    J = _jacobian_det(X1, X2)
    lap = _physical_laplacian(ks, p, ux, uy)            # (m2, m1, Q2, Q1)
    Vq = V(ux, uy)
    # S_V u_bar = i u_bar_t - nu Lap u_bar + V u_bar at (q2, q1, qt)
    coef = np.where(mask, G, 0.0)
    Su = (1j * np.einsum("jit,jiab,tc->abc", coef, phi, Bt[1])
          - nu * np.einsum("jit,jiab,tc->abc", coef, lap, Bt[0])
          + Vq[..., None] * np.einsum("jit,jiab,tc->abc", coef, phi, Bt[0]))
    w = (Ws * J)[..., None] * wt[None, None, :]
    out = np.zeros((m - 2, m - 2, mt - 1), dtype=np.complex128)
    for i2 in range(1, m - 1):
        for i1 in range(1, m - 1):
            for it in range(1, mt):
                conj_SB = (-1j * phi[i2, i1][..., None] * Bt[1, it] - nu * lap[i2, i1][..., None] * Bt[0, it]
                           + (Vq * phi[i2, i1])[..., None] * Bt[0, it])
                out[i2 - 1, i1 - 1, it - 1] = np.sum(w * (-Su) * conj_SB)
    err = np.max(np.abs(fbar - out.ravel())) / np.max(np.abs(out))
    assert err < 1e-7, err
    assert np.max(np.abs(out)) > 1e-3  # the datum reaches the free functions
