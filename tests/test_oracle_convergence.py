"""Discretisation pins: V-norm convergence of order p - 1 (Theorem 2 and the remark after it).

For smooth solutions with p_t = p_s = p and h_t = h_s = h the error in
||v||_V^2 = ||v||^2 + ||S v||^2 decays like h^{p-1}.  The potential case
(S_V = S + V) has no statement in the paper; it is checked against the same
rate ("parity unpinned" by the paper; pinned here by the rate only).
"""
import numpy as np
import pytest

from oracle.operators import FastDiagonalization, Problem
from oracle.pcg import pcg
from oracle.rhs import SpaceTimeBasis, assemble_rhs, errors, full_coefficients
from paper_2311_18461_amd.inputs import (ComplexGaussian1D, GaussianSum, HighModeSeries1D, SineMode1D,
                                         uniform_open_knots)


def _solve(p, n, nu, V=None, T=1.0):
    m = SineMode1D(nu)
    f = m.f if V is None else (lambda t, x: m.f(t, x) + V(x) * m.u(t, x))
    kt, ks = uniform_open_knots(n, p, T), [uniform_open_knots(n, p)]
    pr = Problem(kt, ks, p, p, nu, V)
    stb = SpaceTimeBasis(kt, ks, p, p)
    fb, G = assemble_rhs(stb, nu, f=f, u0=m.u0, V=V)
    x, info = pcg(pr.matvec, FastDiagonalization(pr).apply, fb, tol=1e-12, maxit=300)
    assert info["converged"]
    C = full_coefficients(G, x, pr.n_s, pr.n_t)
    return errors(kt, ks, p, p, C, nu, m.u, f, V)


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("with_V", [False, True])
def test_v_norm_rate(p, with_V):
    V = GaussianSum(np.array([[0.4]]), np.array([0.15]), np.array([30.0])) if with_V else None
    ns = [8, 16, 32]
    ev = [_solve(p, n, 1.0, V)[1] for n in ns]
    rates = np.log2(np.array(ev[:-1]) / np.array(ev[1:]))
    assert rates[-1] > (p - 1) - 0.2, rates


def test_config1_sine_solution_accuracy():
    """1D, p = 2, 16 x 16 elements, u = sin(pi x) exp(-i pi^2 t), tol 1e-10."""
    l2, vn = _solve(2, 16, 1.0)
    assert l2 < 1e-2 and vn < 1.0


@pytest.mark.parametrize("name", ["gaussian", "high_mode"])
def test_section61_data_satisfy_the_equation(name):
    """The Section 6.1 solutions and right-hand sides: f = S u = i u_t - u_xx, checked by fourth-order
    central differences at random points (independent of the closed forms of f)."""
    m = ComplexGaussian1D() if name == "gaussian" else HighModeSeries1D(M=8)
    rng = np.random.default_rng(5)
    t, x = rng.uniform(0.2, 1.8, 20), rng.uniform(0.1, 0.9, 20)
    h = 1e-3 if name == "gaussian" else 1e-5
    c1 = np.array([1.0, -8.0, 0.0, 8.0, -1.0]) / 12.0
    c2 = np.array([-1.0, 16.0, -30.0, 16.0, -1.0]) / 12.0
    k = np.arange(-2, 3)
    ut = sum(c * m.u(t + kk * h, x) for c, kk in zip(c1, k)) / h
    uxx = sum(c * m.u(t, x + kk * h) for c, kk in zip(c2, k)) / h ** 2
    err = np.max(np.abs(1j * ut - uxx - m.f(t, x))) / np.max(np.abs(m.f(t, x)))
    assert err < (1e-8 if name == "gaussian" else 1e-4), err
    if name == "high_mode":
        assert np.max(np.abs(m.u(0.0, x))) == 0.0 and np.max(np.abs(m.u(t, 0.0 * x))) < 1e-12


def test_separable_errors_equal_pointwise_errors():
    """errors_separable (the exact series through its per-mode factors on the tensor grid) against
    errors (the series evaluated point by point) for the high-mode data with M = 40 on a coarse
    solve, and the separable sampling of f against f itself."""
    from oracle.rhs import errors_separable
    p, n, T = 3, 6, 2.0
    m = HighModeSeries1D(M=40)
    kt, ks = uniform_open_knots(2 * n, p, T), [uniform_open_knots(n, p)]
    pr = Problem(kt, ks, p, p, 1.0, None)
    fb, G = assemble_rhs(SpaceTimeBasis(kt, ks, p, p), 1.0, f=m.f, u0=m.u0, dirichlet=m.u)
    x, info = pcg(pr.matvec, FastDiagonalization(pr).apply, fb, tol=1e-12, maxit=300)
    C = full_coefficients(G, x, pr.n_s, pr.n_t)
    l2, vn = errors(kt, ks, p, p, C, 1.0, m.u, m.f)
    l2s, vns = errors_separable(kt, ks, p, p, C, 1.0, m.space_factors, m.time_factors_u, m.time_factors_f)
    assert abs(l2s - l2) <= 1e-12 * l2 and abs(vns - vn) <= 1e-12 * vn
    rng = np.random.default_rng(6)
    t, xx = rng.uniform(0.0, T, 7), rng.uniform(0.0, 1.0, 5)
    want = m.f(t[None, :], xx[:, None])
    assert np.max(np.abs(m.f_grid(t, xx) - want)) <= 1e-12 * np.max(np.abs(want))
