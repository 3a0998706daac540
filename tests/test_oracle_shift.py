"""Pins of the preconditioner shifted by the mean potential (an extension: the paper's P-hat has no
potential, Section 5).

P-hat_c is P-hat built for S + c with a constant c: nu L_s becomes H_c = nu L_s + c M_s, which the
spatial eigenvectors U diagonalise with the scalars nu lambda_i + c, so Algorithm 1 runs unchanged
with mu_i = nu lambda_i + c.  Independent references:
  * the dense inverse of P-hat_c assembled from its definition (Kronecker products of the dense 1D
    matrices, no eigenvectors);
  * for the constant potential V = c, A_c - P-hat_c = nu^2 (B_s - L_s M_s^-1 L_s) (x) M_t >= 0,
    the same Loewner bound as for V = 0 (eig(P-hat_c^-1 A_c) >= 1), with A_c the brute-force-pinned
    system matrix of the potential c;
  * the mean of V by the Gauss rule against closed-form integrals.
"""
import numpy as np
import pytest

from oracle.operators import FastDiagonalization, Problem, mean_potential
from oracle.pcg import pcg
from paper_2311_18461_amd.inputs import gaussian_potential, random_complex, uniform_open_knots


def _problem(d, n, p, V=None):
    kt = uniform_open_knots(n + 1, p)
    ks = [uniform_open_knots(n + l, p) for l in range(d)]
    return Problem(kt, ks, p, p, 0.9, V), kt, ks


@pytest.mark.parametrize("d,n,p,c", [(1, 6, 3, 7.5), (2, 3, 2, 12.0), (2, 4, 3, -3.0), (3, 2, 2, 20.0)])
def test_shifted_fd_is_exact_inverse(d, n, p, c):
    pr, *_ = _problem(d, n, p)
    fd = FastDiagonalization(pr, shift=c)
    r = random_complex(pr.N, 21)
    ref = np.linalg.solve(pr.dense_P(shift=c), r)
    assert np.linalg.norm(fd.apply(r) - ref) <= 1e-11 * np.linalg.norm(ref)
    for H in fd.H(np.arange(pr.N_s)):
        np.linalg.cholesky(H)


@pytest.mark.parametrize("d,n,p,c", [(1, 8, 2, 10.0), (2, 3, 3, 25.0), (2, 4, 2, 4.0)])
def test_shifted_preconditioner_below_constant_potential_system(d, n, p, c):
    """V = c: A_c - P-hat_c = nu^2 (B_s - L_s M_s^-1 L_s) (x) M_t >= 0."""
    pr, *_ = _problem(d, n, p, V=lambda *x: np.full(np.broadcast(*x).shape, c))
    A, P = pr.dense_A(), pr.dense_P(shift=c)
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() >= 1 - 1e-10
    # and the unshifted P-hat is not below A_c (the shift is what makes the bound hold)
    ev0 = np.linalg.eigvals(np.linalg.solve(pr.dense_P(), A)).real
    assert ev0.max() > ev.real.max()


def test_mean_potential_closed_forms():
    ks = [uniform_open_knots(5, 3), uniform_open_knots(7, 3)]
    assert abs(mean_potential(ks, 3, lambda x, y: 0 * x + 4.0) - 4.0) < 1e-14
    # int_0^1 x + y^2 = 1/2 + 1/3; cubic x^3 y exact as well (1/8)
    assert abs(mean_potential(ks, 3, lambda x, y: x + y * y) - (0.5 + 1.0 / 3.0)) < 1e-14
    assert abs(mean_potential(ks, 3, lambda x, y: x ** 3 * y) - 0.125) < 1e-14


def test_shift_by_mean_potential_cuts_iterations():
    """The 8-Gaussian potential at 16^3, p = 3: PCG with P-hat_c, c = mean V, takes fewer iterations
    than with the V-free P-hat (a property, not a paper figure)."""
    V = gaussian_potential(2, 2000)
    kt = uniform_open_knots(16, 3)
    ks = [uniform_open_knots(16, 3)] * 2
    pr = Problem(kt, ks, 3, 3, 1.0, V)
    f = random_complex(pr.N, 22)
    c = mean_potential(ks, 3, V)
    _, i0 = pcg(pr.matvec, FastDiagonalization(pr).apply, f, tol=1e-8, maxit=500)
    _, ic = pcg(pr.matvec, FastDiagonalization(pr, shift=c).apply, f, tol=1e-8, maxit=500)
    print(f"mean V {c:.3f}: iterations {i0['iters']} -> {ic['iters']}")
    assert ic["converged"] and ic["iters"] < 0.8 * i0["iters"]
