"""Pins of the oracle's mapped-domain operators (quarter annulus, Section 3.1 mapped domains).

The map and its derivatives are pinned by closed forms and finite differences, the chain
rule by functions with known Laplacians, the assembly by the identity map (where it must
equal the unit-square operators) and by the integration-by-parts identity that links the
gradient form of S_3 to the Laplacian form of K_V.
"""
import numpy as np
import pytest

from oracle.bspline import gauss_rule
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
