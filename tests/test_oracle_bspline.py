"""Pins of the oracle's B-spline basis and 1D Gram matrices (paper Sections 3.1, 4.3, 5.1).

Each check uses a fact fixed outside the oracle: a textbook identity, SciPy's
independent B-spline implementation, a closed form of cardinal B-splines, or
the paper's Table 1.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.interpolate import BSpline

from oracle.bspline import basis, gauss_rule, greville
from oracle.matrices import gram_1d, space_1d, time_1d
from paper_2311_18461_amd.inputs import graded_open_knots, uniform_open_knots

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

KNOTS = [(uniform_open_knots(7, 2), 2), (uniform_open_knots(5, 3), 3), (graded_open_knots(6, 4), 4),
         (np.array([0, 0, 0, 0.2, 0.5, 0.5, 0.8, 1, 1, 1.0]), 2), (uniform_open_knots(4, 1), 1)]


@pytest.mark.parametrize("kn,p", KNOTS)
def test_basis_matches_scipy(kn, p):
    """Cox-de Boor values and de Boor derivatives agree with scipy.interpolate.BSpline."""
    x = np.linspace(0.0, 1.0, 57)
    B = basis(kn, p, x, nder=2)
    m = len(kn) - p - 1
    interior_knots = np.asarray(kn)[p + 1:-p - 1]
    max_mult = max([np.sum(interior_knots == z) for z in interior_knots] + [0])
    for r in range(min(2, p - max_mult + 1, p) + 1):
        ref = np.array([BSpline(kn, np.eye(m)[i], p).derivative(r)(x) if r else
                        BSpline(kn, np.eye(m)[i], p)(x) for i in range(m)])
        interior = (x > 0) & (x < 1)
        if r == 2 and p == 2:
            # second derivatives jump at C^1 knots: compare away from breakpoints
            brk = np.unique(kn)
            interior &= np.min(np.abs(x[:, None] - brk[None, :]), axis=1) > 1e-9
        np.testing.assert_allclose(B[r][:, interior], ref[:, interior], atol=1e-10 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("kn,p", KNOTS)
def test_partition_of_unity_and_integrals(kn, p):
    """sum_i b_i = 1 and int b_i = (xi_{i+p+1} - xi_i)/(p+1) (de Boor)."""
    x = np.linspace(0.0, 1.0, 101)
    B = basis(kn, p, x, nder=1)
    np.testing.assert_allclose(B[0].sum(0), 1.0, atol=1e-14)
    np.testing.assert_allclose(B[1].sum(0), 0.0, atol=1e-11)
    M = gram_1d(kn, p)["M"]
    m = M.shape[0]
    integrals = np.array([(kn[i + p + 1] - kn[i]) / (p + 1) for i in range(m)])
    np.testing.assert_allclose(M.sum(1), integrals, rtol=1e-13)


def test_hat_functions_p1():
    """Degree 1 on uniform knots gives hat functions; mass row h(1,4,1)/6, stiffness (-1,2,-1)/h."""
    n = 6
    kn = uniform_open_knots(n, 1)
    h = 1.0 / n
    x = np.array([0.5 * h, 1.5 * h])
    B = basis(kn, 1, x, nder=1)
    np.testing.assert_allclose(B[0][1], [0.5, 0.5], atol=1e-15)
    g = gram_1d(kn, 1)
    np.testing.assert_allclose(g["M"][2, 1:4], h * np.array([1, 4, 1]) / 6, rtol=1e-14)
    np.testing.assert_allclose(g["L"][2, 1:4], np.array([-1, 2, -1]) / h, rtol=1e-13)


def test_derivatives_vs_central_differences():
    kn, p = graded_open_knots(5, 3), 3
    x = np.array([0.13, 0.41, 0.77])
    e = 1e-6
    B = basis(kn, p, x)
    Bp, Bm = basis(kn, p, x + e, 0)[0], basis(kn, p, x - e, 0)[0]
    np.testing.assert_allclose(B[1], (Bp - Bm) / (2 * e), atol=1e-7)


def _cardinal(n, x, r=0):
    """r-th derivative of the cardinal B-spline of order n on knots 0..n (truncated-power form)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for k in range(n + 1):
        out += (-1) ** k * math.comb(n, k) * np.where(x > k, (x - k), 0.0) ** (n - 1 - r)
    return out / math.factorial(n - 1 - r)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_interior_rows_closed_form(p):
    """Uniform interior rows: M = h N(p+1+k), L = -N''(p+1+k)/h, J = N''''(p+1+k)/h^3,
    N = cardinal B-spline of order 2p+2 (autocorrelation of B-splines)."""
    n_el = 3 * p + 4
    h = 1.0 / n_el
    g = gram_1d(uniform_open_knots(n_el, p), p)
    i = 2 * p  # this function and its 2p neighbours avoid the repeated end knots
    k = np.arange(-p, p + 1)
    N = 2 * p + 2
    np.testing.assert_allclose(g["M"][i, i + k], h * _cardinal(N, p + 1 + k), rtol=1e-12)
    np.testing.assert_allclose(g["L"][i, i + k], -_cardinal(N, p + 1 + k, 2) / h, rtol=1e-11)
    np.testing.assert_allclose(g["J"][i, i + k], _cardinal(N, p + 1 + k, 4) / h ** 3, rtol=1e-10, atol=1e-9 / h ** 3)
    if p == 2:
        np.testing.assert_allclose(g["M"][i, i + k], h * np.array([1, 26, 66, 26, 1]) / 120, rtol=1e-13)
    if p == 3:
        np.testing.assert_allclose(g["M"][i, i + k], h * np.array([1, 120, 1191, 2416, 1191, 120, 1]) / 5040,
                                   rtol=1e-13)


@pytest.mark.parametrize("kn,p", KNOTS[:3])
def test_full_basis_kernels(kn, p):
    """L 1 = 0, J 1 = J g = 0 (Greville abscissae reproduce x), G 1 = 0 with G[i,j] = int b_j' b_i."""
    g = gram_1d(kn, p)
    one = np.ones(g["M"].shape[0])
    s = np.abs(g["L"]).max()
    np.testing.assert_allclose(g["L"] @ one, 0, atol=1e-12 * s)
    np.testing.assert_allclose(g["G"] @ one, 0, atol=1e-12)
    if p >= 2:
        sj = np.abs(g["J"]).max()
        np.testing.assert_allclose(g["J"] @ one, 0, atol=1e-11 * sj)
        np.testing.assert_allclose(g["J"] @ greville(kn, p), 0, atol=1e-11 * sj)


def test_gauss_rule_exact():
    x, w, _ = gauss_rule(graded_open_knots(4, 2), 3)
    for deg in range(6):
        assert abs(np.sum(w * x ** deg) - 1.0 / (deg + 1)) < 1e-14


def test_time_pencil_closed_form():
    """W_t + W_t^* = i K with K[i,j] = 2 int b_j' b_i - delta_{i,n} delta_{j,n} (integration by parts,
    b_i(0) = 0 on the reduced time basis and only the last function equals 1 at T)."""
    T = 1.7
    kn = uniform_open_knots(6, 3, T)
    t = time_1d(kn, 3)
    G = gram_1d(kn, 3)["G"][1:, 1:]
    K = 2 * G
    K[-1, -1] -= 1.0
    np.testing.assert_allclose(t["T3"], 1j * K, atol=1e-13)
    assert np.abs(t["T3"].real).max() == 0.0
    # time scaling b_i(t) = b_hat(t / T): M_t = T M_hat, L_t = L_hat / T
    th = time_1d(uniform_open_knots(6, 3), 3)
    np.testing.assert_allclose(t["M"], T * th["M"], rtol=1e-13)
    np.testing.assert_allclose(t["L"], th["L"] / T, rtol=1e-13)


def test_table1_kappa(golden_dir):
    """Table 1: kappa_2(U_l) = sqrt(kappa_2(M_l)) for the Dirichlet-reduced mass matrix."""
    ref = json.load(open(os.path.join(golden_dir, "table1_kappa.json")))
    for n_el in ref["n_el"]:
        for p, kap in zip(ref["p"], ref["kappa_U"]):
            s = space_1d(uniform_open_knots(n_el, p), p)
            ev = np.linalg.eigvalsh(s["M"])
            k_m = math.sqrt(ev[-1] / ev[0])
            assert float(f"{k_m:.2g}") == kap, (n_el, p, k_m)
            if n_el <= 128:
                _, U = sla.eigh(s["L"], s["M"])
                sv = np.linalg.svd(U, compute_uv=False)
                assert abs(sv[0] / sv[-1] - k_m) < 1e-8 * k_m


@pytest.mark.parametrize("p", [2, 3, 4])
def test_generalized_eigs(p):
    """U^T M U = I, U^T L U = Lambda, and lambda_k -> (k pi)^2 from above under refinement."""
    prev = None
    for n_el in (16, 32, 64):
        s = space_1d(uniform_open_knots(n_el, p), p)
        lam, U = sla.eigh(s["L"], s["M"])
        np.testing.assert_allclose(U.T @ s["M"] @ U, np.eye(len(lam)), atol=1e-12)
        np.testing.assert_allclose(U.T @ s["L"] @ U, np.diag(lam), atol=1e-9 * lam.max())
        exact = (np.arange(1, 4) * np.pi) ** 2
        assert np.all(lam[:3] >= exact * (1 - 1e-12))
        if prev is not None:
            assert np.all(lam[:3] - exact <= prev - exact + 1e-12)
        prev = lam[:3]
