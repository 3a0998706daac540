"""Pins of the oracle's system matrix, preconditioner, FD apply, matvec, lifting and PCG.

Independent references used here:
  * a brute-force space-time quadrature of (S_V B_J, S_V B_I) over the full
    (d+1)-dimensional Gauss grid, which never uses the Kronecker split, the
    integration by parts behind the time pencil, or the potential expansion;
  * dense linear algebra (solve, Cholesky, eigenvalues);
  * exact reproduction of a discrete solution (Theorem 1: u in V_h gives u_h = u);
  * the derived Loewner bound P-hat <= A for V = 0 (eigenvalues of P^-1 A >= 1).
"""
import numpy as np
import pytest

from oracle.bspline import basis, gauss_rule
from oracle.operators import FastDiagonalization, Problem, dense_fd_factorization
from oracle.pcg import pcg
from oracle.rhs import SpaceTimeBasis, assemble_rhs, full_coefficients
from oracle.spatial import kron_operators, kron_seq, quadrature_operator
from paper_2311_18461_amd.inputs import (gaussian_potential, graded_open_knots, random_complex,
                                         uniform_open_knots)

CASES = [(1, 6, 2, None), (1, 5, 3, "gauss"), (2, 3, 2, None), (2, 3, 3, "gauss"), (3, 2, 2, None),
         (2, 4, 2, "graded")]


def _problem(d, n, p, kind, nu=1.0, T=1.0):
    kt = uniform_open_knots(n + 1, p, T)  # different time mesh than space
    if kind == "graded":
        ks = [graded_open_knots(n, p, 1.25 + 0.1 * l) for l in range(d)]
    else:
        ks = [uniform_open_knots(n + l, p) for l in range(d)]
    V = gaussian_potential(d, 17, count=3, a_range=(5.0, 40.0)) if kind == "gauss" else None
    return Problem(kt, ks, p, p, nu, V), kt, ks, V


def brute_force_A(kt, ks, p, nu, V):
    """A[I,J] = sum_q w_q (S_V B_J)(q) conj(S_V B_I)(q) over the free basis (space-time Gauss grid)."""
    d = len(ks)
    xt, wt, _ = gauss_rule(kt, p + 1)
    Bt = basis(kt, p, xt, 1)[:, 1:]  # free time functions: drop the first
    xs, ws, Bs = [], [], []
    for kn in ks:
        x, w, _ = gauss_rule(kn, p + 1)
        xs.append(x)
        ws.append(w)
        Bs.append(basis(kn, p, x, 2)[:, 1:-1])
    # spatial functions on the spatial tensor grid (x_1 fastest both for index and point)
    val = kron_seq([B[0] for B in Bs])
    lap = sum(kron_seq([Bs[j][2 if j == l else 0] for j in range(d)]) for l in range(d))
    wsp = kron_seq([w[None, :] for w in ws]).ravel()
    grids = np.meshgrid(*reversed(xs), indexing="ij")
    Vq = V(*reversed(grids)).ravel() if V is not None else np.zeros(val.shape[1])
    spat_SV = -nu * lap + Vq[None, :] * val  # (N_s, Qs)
    # space-time: index (i_s, i_t) -> i_t + n_t i_s, point (q_s, q_t)
    SB = (1j * np.einsum("sa,tb->stab", val, Bt[1]) + np.einsum("sa,tb->stab", spat_SV, Bt[0]))
    N_s, n_t = val.shape[0], Bt.shape[1]
    SB = SB.reshape(N_s * n_t, -1)
    w = np.einsum("a,b->ab", wsp, wt).ravel()
    return (SB.conj() * w) @ SB.T


@pytest.mark.parametrize("d,n,p,kind", CASES)
def test_system_matches_spacetime_quadrature(d, n, p, kind):
    pr, kt, ks, V = _problem(d, n, p, kind, nu=0.7)
    A = pr.dense_A()
    Ab = brute_force_A(kt, ks, p, 0.7, V)
    np.testing.assert_allclose(A, Ab, atol=1e-11 * np.abs(Ab).max())
    x = random_complex(pr.N, 5)
    np.testing.assert_allclose(pr.matvec(x), Ab @ x, atol=1e-11 * np.abs(Ab @ x).max())


@pytest.mark.parametrize("d,n,p,kind", CASES)
def test_hermitian_positive_definite(d, n, p, kind):
    pr, *_ = _problem(d, n, p, kind)
    A, P = pr.dense_A(), pr.dense_P()
    assert np.abs(A - A.conj().T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)
    np.linalg.cholesky(P)
    fd = FastDiagonalization(pr)
    for H in fd.H(np.arange(pr.N_s)):
        np.linalg.cholesky(H)


@pytest.mark.parametrize("d,n,p", [(1, 8, 2), (1, 6, 4), (2, 4, 2), (2, 3, 3), (3, 2, 2), (2, 5, 4)])
def test_preconditioner_below_system(d, n, p):
    """V = 0, F = Id: A - P-hat = nu^2 (B_s - L_s M_s^-1 L_s) (x) M_t >= 0, so eig(P^-1 A) >= 1."""
    pr, *_ = _problem(d, n, p, None, nu=1.3)
    A, P = pr.dense_A(), pr.dense_P()
    ev = np.linalg.eigvals(np.linalg.solve(P, A))
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() >= 1 - 1e-10


def test_bs_kronecker_identity_2d():
    """Reduced basis, d = 2: B_s = M_2 (x) J_1 + J_2 (x) M_1 + 2 L_2 (x) L_1 (integration by parts)."""
    ks = [uniform_open_knots(4, 3), graded_open_knots(5, 3)]
    pr = Problem(uniform_open_knots(3, 3), ks, 3, 3)
    s1, s2 = pr.space1d
    ident = np.kron(s2["M"], s1["J"]) + np.kron(s2["J"], s1["M"]) + 2 * np.kron(s2["L"], s1["L"])
    brute = quadrature_operator(ks, 3, "bilap").toarray()
    np.testing.assert_allclose(brute, ident, atol=1e-10 * np.abs(ident).max())
    np.testing.assert_allclose(kron_operators(pr.space1d)["B"], ident, atol=1e-10 * np.abs(ident).max())


@pytest.mark.parametrize("d,n,p,kind", CASES)
def test_fd_apply_is_exact_inverse(d, n, p, kind):
    """Algorithm 1 solves P-hat s = r exactly (eq. preconditioner_str2) - dense brute force."""
    pr, *_ = _problem(d, n, p, kind)
    P = pr.dense_P()
    fd = FastDiagonalization(pr)
    r = random_complex(pr.N, 11)
    s = fd.apply(r)
    ref = np.linalg.solve(P, r)
    assert np.linalg.norm(s - ref) <= 1e-11 * np.linalg.norm(ref)
    np.testing.assert_allclose(dense_fd_factorization(fd), P, atol=1e-11 * np.abs(P).max())
    # M_s^-1 = U_s U_s^T
    Us = kron_seq(fd.U)
    Ms = kron_operators(pr.space1d)["M"]
    np.testing.assert_allclose(Us @ Us.T @ Ms, np.eye(pr.N_s), atol=1e-11)
    # streamed (no stored inverses) path agrees
    fd2 = FastDiagonalization(pr, precompute_inverse=False)
    np.testing.assert_allclose(fd2.apply(r), s, atol=1e-12 * np.abs(s).max())


@pytest.mark.parametrize("d,n,p,kind", CASES[:4])
def test_pcg_solution_vs_dense(d, n, p, kind):
    pr, *_ = _problem(d, n, p, kind)
    A = pr.dense_A()
    fd = FastDiagonalization(pr)
    f = random_complex(pr.N, 3)
    tol = 1e-10
    x, info = pcg(pr.matvec, fd.apply, f, tol=tol, maxit=500)
    assert info["converged"] and info["true_rel_res"] <= 10 * tol
    ref = np.linalg.solve(A, f)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - ref) <= kappa * 10 * tol * np.linalg.norm(ref)
    # residual identity: ||f - A x|| / ||f||
    assert abs(np.linalg.norm(f - A @ x) / np.linalg.norm(f) - info["true_rel_res"]) < 1e-12


def test_pcg_warm_start_and_zero_rhs():
    pr, *_ = _problem(2, 3, 2, None)
    fd = FastDiagonalization(pr)
    f = random_complex(pr.N, 4)
    x, info = pcg(pr.matvec, fd.apply, f, tol=1e-12)
    x2, info2 = pcg(pr.matvec, fd.apply, f, x0=x, tol=1e-8)
    assert info2["iters"] == 0
    x3, info3 = pcg(pr.matvec, fd.apply, f, x0=x + 1e-3 * random_complex(pr.N, 9), tol=1e-8)
    assert info3["converged"] and info3["iters"] < info["iters"]


class _Spline:
    """u = sum_I C_I B_I over the full space-time basis, and S_V u, evaluated pointwise."""

    def __init__(self, kt, ks, p, C, nu, V):
        self.kt, self.ks, self.p, self.C, self.nu, self.V = kt, ks, p, C, nu, V

    def _eval(self, t, xs, der_t=0, der_x=None):
        t = np.asarray(t, dtype=np.float64)
        shp = t.shape
        Bt = basis(self.kt, self.p, t.ravel(), 1)[der_t]
        vals = []
        for l, (kn, x) in enumerate(zip(self.ks, xs)):
            vals.append(basis(kn, self.p, np.asarray(x, dtype=np.float64).ravel(), 2)[der_x[l] if der_x else 0])
        d = len(self.ks)
        letters = "abc"[:d]
        expr = "".join(reversed(letters)) + "z," + ",".join(c + "p" for c in letters) + ",zp->p"
        return np.einsum(expr, self.C, *vals, Bt).reshape(shp)

    def u(self, t, *xs):
        t, *xs = np.broadcast_arrays(t, *xs)
        return self._eval(t, xs)

    def f(self, t, *xs):
        t, *xs = np.broadcast_arrays(t, *xs)
        d = len(xs)
        out = 1j * self._eval(t, xs, der_t=1)
        for l in range(d):
            out = out - self.nu * self._eval(t, xs, der_x=[2 if j == l else 0 for j in range(d)])
        if self.V is not None:
            out = out + self.V(*xs) * self._eval(t, xs)
        return out


@pytest.mark.parametrize("d,n,p,kind", [(1, 5, 2, None), (1, 4, 3, "gauss"), (2, 3, 2, "gauss"), (2, 3, 3, None)])
def test_discrete_solution_reproduced(d, n, p, kind):
    """A spline u in the discrete space is reproduced exactly (Theorem 1), which pins the load
    vector, the lifting, the matvec, the FD apply and PCG together."""
    nu = 0.9
    pr, kt, ks, V = _problem(d, n, p, kind, nu=nu, T=1.4)
    mt = len(kt) - p - 1
    ms = [len(k) - p - 1 for k in ks]
    g = np.random.default_rng(8)
    C = g.standard_normal(tuple(reversed(ms)) + (mt,)) + 1j * g.standard_normal(tuple(reversed(ms)) + (mt,))
    spl = _Spline(kt, ks, p, C, nu, V)
    stb = SpaceTimeBasis(kt, ks, p, p)
    fb, G = assemble_rhs(stb, nu, f=spl.f, u0=lambda *x: spl.u(0.0, *x), dirichlet=spl.u, V=V)
    fixed = G != 0
    np.testing.assert_allclose(G[fixed], C[fixed], atol=1e-10)
    fd = FastDiagonalization(pr)
    x, info = pcg(pr.matvec, fd.apply, fb, tol=1e-13, maxit=300)
    full = full_coefficients(G, x, pr.n_s, pr.n_t)
    np.testing.assert_allclose(full, C, atol=1e-8 * np.abs(C).max())
