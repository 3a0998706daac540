"""Convergence studies of Section 6.1 on the GPU solver (1D space + time, T = 2, h_t = h_s = h,
p_t = p_s = p, uniform knots).

The library assembles the right-hand side with lifting and solves to a relative residual of 1e-12;
the errors ||u - u_h||_{L2(Q)} and ||S(u - u_h)||_{L2(Q)} (the V-norm squared is their sum of
squares, Section 2.1) are evaluated with the oracle's quadrature (p + 2 Gauss points per element)
from the library's lifting and solution.  The paper prints no error values (its figures are not
in the text), so the pins are the rates: V-norm order p - 1 for the smooth complex Gaussian
(Theorem 2), and for the non-smooth high-mode series (M = 625) only that refinement reduces the
error, plus agreement with the oracle's own solve on a coarse grid.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from oracle.rhs import SpaceTimeBasis, assemble_rhs, errors, full_coefficients  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 2.0


def gpu_solve(m, p, n, tol=1e-12):
    """Library right-hand side (f, u0 and the Dirichlet trace of u sampled on its Gauss grids) and
    PCG solve; returns the full coefficient tensor (lifting + free solution) and the iterations."""
    from paper_2311_18461_amd import stfd
    kt, ks = inputs.uniform_open_knots(2 * n, p), [inputs.uniform_open_knots(n, p)]
    lib = stfd.Problem(kt, ks, p, p, T, 1.0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    fb = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    lift = lib.load_vector(fb, f_q=to(lib.sample_spacetime(m.f)), u0_q=to(lib.sample_space(m.u0)),
                           dirichlet_q=[to(a) for a in lib.sample_faces(m.u)], return_lift=True)
    u = torch.empty_like(fb)
    rc, info = lib.pcg_solve(fb, u, rtol=tol, maxit=1000)
    assert rc == 0 and info[0]["true_rel_res"] < 10 * tol
    G = lift.reshape(lib.m_full[1], lib.m_full[0])
    C = full_coefficients(G, u.cpu().numpy(), lib.n_s, lib.n_t)
    lib.close()
    return C, info[0]["iters"], kt, ks


def study(m, p, ns):
    rows = []
    for n in ns:
        C, its, kt, ks = gpu_solve(m, p, n)
        l2, vn = errors(np.asarray(kt) * T, ks, p, p, C, 1.0, m.u, m.f)
        rows.append((n, its, l2, vn))
    return rows


def rates(rows, col):
    return [np.log(a[col] / b[col]) / np.log(b[0] / a[0]) for a, b in zip(rows[:-1], rows[1:])]


@pytest.mark.parametrize("p", [2, 3, 4])
def test_complex_gaussian_v_norm_rate(p):
    """Section 6.1, first test: u = a b / sqrt(b^2 - i g t) exp(-x^2 / (b^2 - i g t)), a = b = 1.5,
    g = 2.5, non-homogeneous Dirichlet and initial data from u, f = S u."""
    rows = study(inputs.ComplexGaussian1D(), p, [8, 16, 32, 60])
    rv, rl = rates(rows, 3), rates(rows, 2)
    for n, its, l2, vn in rows:
        print(f"p={p} n_el={n} (time {2 * n}): PCG {its} iterations, L2 error {l2:.3e}, V-norm error {vn:.3e}")
    print(f"p={p}: V-norm rates {np.round(rv, 2)}, L2 rates {np.round(rl, 2)}")
    assert rv[-1] > (p - 1) - 0.2
    # the L2(Q) error stays below the residual part ||S e|| of the V-norm (the remark of Section 6.1)
    assert all(l2 < np.sqrt(vn ** 2 - l2 ** 2) for _, _, l2, vn in rows)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_high_mode_series(p):
    """Section 6.1, second test: the M = 625 high-mode series (homogeneous data, non-smooth solution);
    the grids here are far coarser than the shortest wavelength, so only the error reduction under
    refinement is asserted and the rates are printed."""
    m = inputs.HighModeSeries1D(625)
    rows = study(m, p, [8, 16, 32])
    for n, its, l2, vn in rows:
        print(f"p={p} n_el={n}: PCG {its} iterations, L2 error {l2:.3e}, V-norm error {vn:.3e}")
    print(f"p={p}: V-norm rates {np.round(rates(rows, 3), 2)}")
    assert rows[-1][3] < rows[0][3]


def test_high_mode_series_matches_oracle_solve():
    """The same data solved by the oracle (its own right-hand side and FD-preconditioned CG)."""
    p, n = 3, 8
    m = inputs.HighModeSeries1D(625)
    C, _, kt, ks = gpu_solve(m, p, n)
    ktp = np.asarray(kt) * T
    ref = OProblem(ktp, ks, p, p, 1.0, None)
    fb, G = assemble_rhs(SpaceTimeBasis(ktp, ks, p, p), 1.0, f=m.f, u0=m.u0, dirichlet=m.u)
    x, info = pcg(ref.matvec, FastDiagonalization(ref).apply, fb, tol=1e-12, maxit=500)
    C_ref = full_coefficients(G, x, ref.n_s, ref.n_t)
    err = np.max(np.abs(C - C_ref)) / np.max(np.abs(C_ref))
    print(f"GPU vs oracle full coefficients (p={p}, n_el={n}): {err:.2e}")
    assert err < 1e-9
