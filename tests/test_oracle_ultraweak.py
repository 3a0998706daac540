"""Pins of the ultraweak method's oracle (Section 4.4, eq. uw-discrete-system).

Independent references:
  * the system matrix against a brute-force space-time quadrature of (S_V B_J, S_V B_I) over the
    final-condition basis (no Kronecker split, no integration by parts);
  * the right-hand side (f, B_I) + i (u_0, B_I(0)) against a brute-force quadrature of
    (u, S_V B_I) for a smooth u that vanishes on the spatial boundary but not at T: the two agree
    only through the integration by parts behind the method (sign and conjugation of the
    initial-data term);
  * exact reproduction: for u = S_V z* with z* in W_h the method returns z_h = z* (u_h is the
    L2(Q) projection of u onto S_V(W_h));
  * the fast-diagonalisation apply against the dense inverse of P-hat on the final-condition basis.
"""
import numpy as np
import pytest

from oracle import ultraweak as uw
from oracle.bspline import basis, gauss_rule
from oracle.operators import FastDiagonalization, Problem
from oracle.pcg import pcg
from oracle.rhs import SpaceTimeBasis
from oracle.spatial import kron_seq
from paper_2311_18461_amd.inputs import gaussian_potential, random_complex, uniform_open_knots


def _spacetime_test_functions(kt, ks, p, nu, V, q):
    """S_V B_I at the space-time Gauss grid (q points per element) for the free basis of W_h,
    rows I = i_t + n_t i_s, columns (spatial point, time point); and the weights."""
    d = len(ks)
    xt, wt, _ = gauss_rule(kt, q)
    Bt = basis(kt, p, xt, 1)[:, :-1]  # final condition: drop the last time function
    xs, ws, Bs = [], [], []
    for kn in ks:
        x, w, _ = gauss_rule(kn, q)
        xs.append(x)
        ws.append(w)
        Bs.append(basis(kn, p, x, 2)[:, 1:-1])
    val = kron_seq([B[0] for B in Bs])
    lap = sum(kron_seq([Bs[j][2 if j == l else 0] for j in range(d)]) for l in range(d))
    wsp = kron_seq([w[None, :] for w in ws]).ravel()
    grids = np.meshgrid(*reversed(xs), indexing="ij")
    Vq = V(*reversed(grids)).ravel() if V is not None else np.zeros(val.shape[1])
    spat = -nu * lap + Vq[None, :] * val
    SB = 1j * np.einsum("sa,tb->stab", val, Bt[1]) + np.einsum("sa,tb->stab", spat, Bt[0])
    SB = SB.reshape(val.shape[0] * Bt.shape[1], -1)
    w = np.einsum("a,b->ab", wsp, wt).ravel()
    pts = [np.repeat(g.ravel(), len(xt)) for g in reversed(grids)]  # x_1 .. x_d per column
    tt = np.tile(xt, val.shape[1])
    return SB, w, tt, pts


def _problem(d, n, p, with_V, nu=0.8):
    kt = uniform_open_knots(n + 1, p)
    ks = [uniform_open_knots(n + l, p) for l in range(d)]
    V = gaussian_potential(d, 23, count=2, a_range=(5.0, 30.0)) if with_V else None
    return kt, ks, V, Problem(kt, ks, p, p, nu, V, final=True)


class _Smooth:
    """u = prod_l sin(pi x_l) g(t), g = (1 + t + 2 t^2) e^{i t}; f = S_V u."""

    def __init__(self, d, nu, V):
        self.d, self.nu, self.V = d, nu, V

    def u(self, t, *x):
        s = np.prod([np.sin(np.pi * xi) for xi in x], axis=0)
        return s * (1 + t + 2 * t * t) * np.exp(1j * t)

    def f(self, t, *x):
        s = np.prod([np.sin(np.pi * xi) for xi in x], axis=0)
        g = (1 + t + 2 * t * t) * np.exp(1j * t)
        dg = (1 + 4 * t) * np.exp(1j * t) + 1j * g
        out = s * (1j * dg + self.nu * self.d * np.pi ** 2 * g)
        if self.V is not None:
            out = out + self.V(*x) * s * g
        return out

    def u0(self, *x):
        return self.u(0.0 * x[0], *x)


@pytest.mark.parametrize("d,n,p,with_V", [(1, 5, 2, False), (1, 4, 3, True), (2, 3, 2, True), (2, 3, 3, False)])
def test_matrix_matches_spacetime_quadrature(d, n, p, with_V):
    kt, ks, V, pr = _problem(d, n, p, with_V)
    SB, w, _, _ = _spacetime_test_functions(kt, ks, p, pr.nu, V, p + 1)
    Ab = (SB.conj() * w) @ SB.T
    A = pr.dense_A()
    np.testing.assert_allclose(A, Ab, atol=1e-11 * np.abs(Ab).max())
    np.linalg.cholesky(A)


@pytest.mark.parametrize("d,n,p,with_V", [(1, 5, 2, False), (1, 4, 3, True), (2, 3, 3, True)])
def test_load_vector_equals_projection_of_the_solution(d, n, p, with_V):
    """(f, B_I) + i (u_0, B_I(0)) = (u, S_V B_I): brute force with 8 Gauss points per element."""
    kt, ks, V, pr = _problem(d, n, p, with_V)
    m = _Smooth(d, pr.nu, V)
    stb = SpaceTimeBasis(kt, ks, p, p, q=8)  # both sides with the same 8-point rule
    F = uw.load_vector(stb, f=m.f, u0=m.u0).reshape(-1)
    SB, w, tt, pts = _spacetime_test_functions(kt, ks, p, pr.nu, V, 8)
    ref = (SB.conj() * w) @ m.u(tt, *pts)
    assert np.max(np.abs(F - ref)) <= 1e-11 * np.max(np.abs(ref))
    # the initial-data term alone is not small: dropping it (or its factor i) breaks the identity
    F0 = uw.load_vector(stb, f=m.f).reshape(-1)
    assert np.max(np.abs(F0 - ref)) > 1e-3 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,n,p,with_V", [(1, 6, 4, False), (2, 3, 4, True)])
def test_exact_reproduction_of_the_trial_space(d, n, p, with_V):
    """u = S_V z* with z* in W_h: the discrete solution is z* (the method is the L2(Q) projection
    onto S_V(W_h)); the right-hand side is taken as (u, S_V B_I) by quadrature of u itself."""
    kt, ks, V, pr = _problem(d, n, p, with_V)
    z_star = random_complex(pr.N, 3)
    stb = SpaceTimeBasis(kt, ks, p, p)
    Vq = V(*stb.space_grid()) if V is not None else None
    u_q = uw.solution_values(stb, z_star, pr.nu, Vq)  # u on the grid of stb (p+1 points)
    SB, w, _, _ = _spacetime_test_functions(kt, ks, p, pr.nu, V, p + 1)
    # reorder u_q (x_d..x_1, t) to the columns of SB (spatial point x_1 fastest, then time)
    rhs = (SB.conj() * w) @ u_q.reshape(-1)
    z, info = pcg(pr.matvec, FastDiagonalization(pr).apply, rhs, tol=1e-13, maxit=500)
    assert info["converged"]
    assert np.linalg.norm(z - z_star) <= 1e-9 * np.linalg.norm(z_star)


@pytest.mark.parametrize("d,n,p", [(1, 6, 3), (2, 3, 2), (3, 2, 2)])
def test_fd_apply_inverts_p_hat_on_the_final_condition_basis(d, n, p):
    kt, ks, V, pr = _problem(d, n, p, False)
    fd = FastDiagonalization(pr)
    for H in fd.H(np.arange(pr.N_s)):
        np.linalg.cholesky(H)
    r = random_complex(pr.N, 7)
    ref = np.linalg.solve(pr.dense_P(), r)
    assert np.linalg.norm(fd.apply(r) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_l2_convergence_1d():
    """||u - u_h||_{L2(Q)} for the smooth solution decreases at order >= p - 1 (p = 3, 1D)."""
    p, nu = 3, 1.0
    errs = []
    for n in (4, 8, 16):
        kt, ks = uniform_open_knots(n, p), [uniform_open_knots(n, p)]
        pr = Problem(kt, ks, p, p, nu, final=True)
        m = _Smooth(1, nu, None)
        F = uw.load_vector(SpaceTimeBasis(kt, ks, p, p), f=m.f, u0=m.u0).reshape(-1)
        z, info = pcg(pr.matvec, FastDiagonalization(pr).apply, F, tol=1e-13, maxit=500)
        assert info["converged"]
        errs.append(uw.l2_error(kt, ks, p, p, z, nu, m.u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("ultraweak L2 errors", errs, "rates", rates)
    assert rates[-1] > p - 1 - 0.2
