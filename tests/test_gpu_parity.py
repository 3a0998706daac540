"""GPU parity of the C ABI library against the CPU oracle.

Tolerances (FP64 path).  The matvec is a sum of at most a few hundred FP64
products per entry, so each entry agrees with the dense product to
1e-13 * sum_j |A_ij x_j|.  The FD apply is backward stable in each factor:
the mode products carry kappa(U_l)^2 <= 60 (Table 1, p <= 4) and the banded
time solves carry kappa(H_i) <= ~1e4 (dominated by L_t, ~n_t^2), so two
independent FP64 implementations agree to ~kappa * eps ~ 1e-12; the tests use
1e-11 against the oracle's FD and a backward-error test against dense P-hat.
PCG solutions are compared through the residual (<= rtol) and the distance to
the oracle's solution.  With a potential the V-free preconditioner needs many
more iterations than the paper's V = 0 cases (228 at 64^3 with the
8-Gaussian potential), so those solves use maxit = 1000.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402
from parity import abs_matvec, fiber_rel, max_rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stfd():
    from paper_2311_18461_amd import stfd
    return stfd


def make_pair(d, n_el, p, V=None, T=1.0, nu=1.0, graded=False, max_nrhs=1, n_el_t=None, oracle=True):
    stfd = _stfd()
    kt = inputs.uniform_open_knots(n_el_t or n_el, p)
    if graded:
        ks = [inputs.graded_open_knots(n_el + l, p, 1.2 + 0.05 * l) for l in range(d)]
    else:
        ks = [inputs.uniform_open_knots(n_el + l, p) for l in range(d)]
    Vq = stfd.sample_on_quad_grid(V, ks, p) if V is not None else None
    lib = stfd.Problem(kt, ks, p, p, T, nu, V_quad=Vq, max_nrhs=max_nrhs)
    ref = OProblem(inputs.uniform_open_knots(n_el_t or n_el, p, T), ks, p, p, nu, V) if oracle else None
    return lib, ref


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_mfma_lane_layout():
    """The lane layout the mode-product kernel assumes (16x16xK, one block): lane l supplies
    A[l%16][(K/4)(l/16)+e] and B[(K/4)(l/16)+e][l%16]; register v holds D[4(l/16)+v][l%16]
    for the FP32-accumulating instructions and D[4v+l/16][l%16] for the FP64 one.
    Probe: A[m][k] = m + 16k, B[k][n] = (k == n mod K), so D[m][n] = m + 16 (n mod K)."""
    o64, o32, obf = _stfd().debug_mfma_layout()
    lane = np.arange(64)[:, None]
    v = np.arange(4)[None, :]
    n = lane % 16
    m_f64 = 4 * v + lane // 16
    m_f32 = 4 * (lane // 16) + v
    got = {"f64": o64.reshape(64, 4), "f32": o32.reshape(64, 4), "bf16": obf.reshape(64, 4)}
    want = {"f64": m_f64 + 16 * (n % 4), "f32": m_f32 + 16 * (n % 4), "bf16": m_f32 + 16 * n}
    bad = [k for k in got if not np.array_equal(got[k], want[k])]
    for k in bad:
        print(k, "lanes 0-3, 16-19:", got[k][[0, 1, 2, 3, 16, 17, 18, 19]].tolist())
    assert not bad, bad


@pytest.mark.parametrize("d,n_el,p", [(1, 30, 2), (2, 12, 3), (3, 6, 4), (2, 64, 3)])
def test_generalized_eigendecomposition(d, n_el, p):
    """U_l^T M_l U_l = I and U_l^T L_l U_l = Lambda_l (eq. space_eig) with the oracle's matrices."""
    lib, ref = make_pair(d, n_el, p)
    fd = FastDiagonalization(ref)
    for l in range(d):
        U, lam = lib.get_pencil(l)
        M, L = ref.space1d[l]["M"], ref.space1d[l]["L"]
        np.testing.assert_allclose(U.T @ M @ U, np.eye(len(lam)), atol=1e-12)
        np.testing.assert_allclose(U.T @ L @ U, np.diag(lam), atol=1e-12 * lam.max())
        np.testing.assert_allclose(lam, fd.lam1d[l], rtol=1e-12)


TINY = [(1, 8, 2, None, False), (1, 5, 4, "gauss", True), (2, 3, 2, None, False), (2, 4, 3, "gauss", False),
        (2, 3, 4, None, True), (3, 2, 2, None, False), (3, 2, 3, "gauss", False), (1, 17, 3, None, False)]


def _V(kind, d):
    return inputs.gaussian_potential(d, 31, count=4, a_range=(5.0, 40.0)) if kind == "gauss" else None


@pytest.mark.parametrize("d,n_el,p,kind,graded", TINY)
def test_apply_fp64_vs_dense_inverse(d, n_el, p, kind, graded):
    """FD apply on the GPU equals the dense solve with P-hat (brute force, eq. prec_definition)."""
    lib, ref = make_pair(d, n_el, p, _V(kind, d), graded=graded, T=1.3, nu=0.8)
    P = ref.dense_P()
    r = inputs.random_complex(lib.N, 7)
    out = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    lib.apply_preconditioner(to_dev(r), out)
    torch.cuda.synchronize()
    s = out.cpu().numpy()
    # backward error against P-hat, and forward error within the conditioning of the dense reference
    assert np.linalg.norm(P @ s - r) / (np.linalg.norm(P, 2) * np.linalg.norm(s)) < 1e-15
    assert rel(s, np.linalg.solve(P, r)) < max(1e-12, 50 * np.linalg.cond(P) * 2.2e-16)


@pytest.mark.parametrize("d,n_el,p,kind,graded", TINY)
def test_matvec_vs_dense(d, n_el, p, kind, graded):
    lib, ref = make_pair(d, n_el, p, _V(kind, d), graded=graded, T=1.3, nu=0.8)
    A = ref.dense_A()
    x = inputs.random_complex(lib.N, 8)
    out = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    lib.matvec(to_dev(x), out)
    torch.cuda.synchronize()
    y = A @ x
    # entrywise: |y_gpu - y| <= c eps sum_j |A_ij||x_j| (FP64 dot products of at most a few hundred terms)
    bound = 1e-13 * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(out.cpu().numpy() - y) <= bound + 1e-300)


MEDIUM = [(2, 64, 3, "gauss2000"), (2, 37, 2, None), (3, 12, 3, None), (3, 9, 4, "harm"), (1, 120, 4, None),
          (2, 64, 4, None)]


def _Vm(kind, d):
    if kind == "gauss2000":
        return inputs.gaussian_potential(d, 2000)
    if kind == "harm":
        return inputs.harmonic_potential(d, 3000)
    return None


@pytest.mark.parametrize("d,n_el,p,kind", MEDIUM)
def test_apply_and_matvec_vs_oracle(d, n_el, p, kind):
    """Config-scale grids (2D p=3 64^3 elements is the Gaussian-potential workload): GPU vs oracle."""
    lib, ref = make_pair(d, n_el, p, _Vm(kind, d))
    fd = FastDiagonalization(ref, precompute_inverse=False)
    r = inputs.random_complex(lib.N, 9)
    rd = to_dev(r)
    out = torch.empty_like(rd)
    lib.apply_preconditioner(rd, out)
    torch.cuda.synchronize()
    s, s_ref = out.cpu().numpy(), fd.apply(r)
    e_max, e_fib = max_rel(s, s_ref), fiber_rel(s, s_ref, lib.n_t)
    lib.matvec(rd, out)
    torch.cuda.synchronize()
    y = out.cpu().numpy()
    # entrywise: |y_gpu - y| <= c eps (|A| |x|)_i at every entry
    e_mv = float(np.max(np.abs(y - ref.matvec(r)) / abs_matvec(ref, r)))
    print(f"d={d} n_el={n_el} p={p}: apply max {e_max:.2e} per-fibre {e_fib:.2e}; matvec / (|A||x|) {e_mv:.2e}")
    assert e_max < 1e-11 and e_fib < 1e-10
    assert e_mv < 1e-13


@pytest.mark.parametrize("d,n_el,p,kind", [(1, 8, 2, None), (2, 4, 3, "gauss"), (3, 2, 2, None)])
def test_pcg_vs_dense_solve(d, n_el, p, kind):
    lib, ref = make_pair(d, n_el, p, _V(kind, d))
    A = ref.dense_A()
    f = inputs.random_complex(lib.N, 12)
    u = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    rc, info = lib.pcg_solve(to_dev(f), u, rtol=1e-10, maxit=300)
    assert rc == 0 and info[0]["status"] == 0
    x = u.cpu().numpy()
    true = np.linalg.norm(f - A @ x) / np.linalg.norm(f)
    assert true <= 2e-10 and abs(true - info[0]["true_rel_res"]) < 1e-12
    ustar = np.linalg.solve(A, f)
    assert rel(x, ustar) <= np.linalg.cond(A) * 2e-10


@pytest.mark.parametrize("d,n_el,p,kind", [(2, 64, 3, "gauss2000"), (2, 32, 4, None), (3, 10, 3, "harm")])
def test_pcg_vs_oracle_pcg(d, n_el, p, kind):
    lib, ref = make_pair(d, n_el, p, _Vm(kind, d))
    fd = FastDiagonalization(ref)
    f = inputs.random_complex(lib.N, 13)
    u = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    tol = 1e-8
    rc, info = lib.pcg_solve(to_dev(f), u, rtol=tol, maxit=1000)
    # the oracle runs on to tol / 3 so that its residual history brackets the stopping point
    x_ref, info_ref = pcg(ref.matvec, fd.apply, f, tol=tol / 3, maxit=1000, record=True)
    assert rc == 0
    hist = np.asarray(info_ref["history"])
    k_ora = int(np.argmax(hist <= tol))
    k_gpu = info[0]["iters"]
    # finite-precision CG fixes the stopping iteration only up to a rounding-induced delay
    # (fresh relative noise of 1e-15 in each operator application moves the oracle's residual at a
    # given late iteration of the 8-Gaussian workload by a factor 2): the GPU must stop where the
    # oracle's own residual is within a factor 3 of the tolerance (or within 2% of the oracle's
    # count, whichever window is wider)
    k_lo, k_hi = int(np.argmax(hist <= 3 * tol)), int(np.argmax(hist <= tol / 3))
    slack = max(1, k_ora // 50)
    print(f"iterations gpu {k_gpu} oracle {k_ora} (oracle residual within [tol/3, 3 tol]: {k_lo}..{k_hi})")
    assert min(k_lo, k_ora - slack) <= k_gpu <= max(k_hi, k_ora + slack)
    x = u.cpu().numpy()
    assert np.linalg.norm(f - ref.matvec(x)) / np.linalg.norm(f) <= 1.2e-8
    assert rel(x, x_ref) < 1e-5


@pytest.mark.parametrize("prec,bound", [("fp32", 2e-5), ("bf16", 5e-2)])
@pytest.mark.parametrize("d,n_el,p", [(2, 64, 3), (3, 12, 3), (2, 20, 4)])
def test_mixed_precision_apply_error(prec, bound, d, n_el, p):
    """Relative error of the FP32 / BF16-MFMA apply against the FP64 oracle apply (reported, bounded)."""
    lib, ref = make_pair(d, n_el, p)
    fd = FastDiagonalization(ref)
    r = inputs.random_complex(lib.N, 14)
    rd = to_dev(r)
    out = torch.empty_like(rd)
    lib.apply_preconditioner(rd, out, precision=prec)
    torch.cuda.synchronize()
    z, z_ref = out.cpu().numpy(), fd.apply(r)
    err, err_max = rel(z, z_ref), max_rel(z, z_ref)
    print(f"{prec} apply rel err d={d} n_el={n_el} p={p}: 2-norm {err:.3e}, max-norm {err_max:.3e}")
    assert err < bound and err_max < bound


@pytest.mark.parametrize("prec", ["fp32", pytest.param("bf16", marks=pytest.mark.xfail(
    reason="plain BF16 operands (apply error ~7e-3) stall flexible PCG on the 226-iteration "
           "8-Gaussian potential workload within 1000 iterations", strict=False))])
def test_mixed_precision_pcg_reaches_fp64_tolerance(prec):
    lib, ref = make_pair(2, 64, 3, _Vm("gauss2000", 2))
    f = inputs.random_complex(lib.N, 15)
    fd64 = torch.empty(lib.N, dtype=torch.complex128, device=DEV)
    rc64, info64 = lib.pcg_solve(to_dev(f), fd64, rtol=1e-8, maxit=1000)
    u = torch.empty_like(fd64)
    rc, info = lib.pcg_solve(to_dev(f), u, rtol=1e-8, maxit=1000, precision=prec)
    assert rc == 0 and info[0]["true_rel_res"] <= 1.2e-8
    x = u.cpu().numpy()
    assert np.linalg.norm(f - ref.matvec(x)) / np.linalg.norm(f) <= 1.2e-8
    print(f"{prec}: iters {info[0]['iters']} vs fp64 {info64[0]['iters']}, "
          f"|u - u64|/|u64| = {rel(x, fd64.cpu().numpy()):.2e}")
    # the inexact preconditioner costs iterations on this potential workload (FP32: ~1.4x)
    assert info[0]["iters"] <= 2 * info64[0]["iters"]


def test_batched_equals_single():
    """nrhs stacked vectors give bitwise the same result as one call per vector."""
    lib, _ = make_pair(2, 16, 3, _V("gauss", 2), max_nrhs=3, oracle=False)
    N = lib.N
    rs = [inputs.random_complex(N, 20 + k) for k in range(3)]
    stacked = to_dev(np.concatenate(rs))
    out = torch.empty_like(stacked)
    for prec in ("fp64", "fp32", "bf16"):
        lib.apply_preconditioner(stacked, out, nrhs=3, precision=prec)
        single = torch.empty(N, dtype=torch.complex128, device=DEV)
        for k in range(3):
            lib.apply_preconditioner(to_dev(rs[k]), single, precision=prec)
            assert torch.equal(out[k * N:(k + 1) * N], single)
    lib.matvec(stacked, out, nrhs=3)
    single = torch.empty(N, dtype=torch.complex128, device=DEV)
    for k in range(3):
        lib.matvec(to_dev(rs[k]), single)
        assert torch.equal(out[k * N:(k + 1) * N], single)
    # PCG: each system converges on its own; scale one rhs so it needs fewer iterations
    u = torch.empty_like(stacked)
    rc, infos = lib.pcg_solve(stacked, u, nrhs=3, rtol=1e-9)
    assert rc == 0
    for k in range(3):
        rc1, info1 = lib.pcg_solve(to_dev(rs[k]), single, rtol=1e-9)
        assert info1[0]["iters"] == infos[k]["iters"]
        assert torch.equal(u[k * N:(k + 1) * N], single)


def test_pcg_edge_cases():
    stfd = _stfd()
    lib, ref = make_pair(2, 6, 3, _V("gauss", 2), max_nrhs=2)
    N = lib.N
    zero = torch.zeros(N, dtype=torch.complex128, device=DEV)
    u = torch.full((N,), 3.0 + 1j, dtype=torch.complex128, device=DEV)
    rc, info = lib.pcg_solve(zero, u)
    assert rc == 0 and info[0]["iters"] == 0 and torch.count_nonzero(u) == 0
    f = to_dev(inputs.random_complex(N, 30))
    rc, info = lib.pcg_solve(f, u, maxit=1)
    assert rc == stfd.NOT_CONVERGED and info[0]["iters"] == 1 and info[0]["status"] == stfd.NOT_CONVERGED
    # warm start at the solution: zero iterations
    rc, info = lib.pcg_solve(f, u, rtol=1e-12, maxit=200)
    rc2, info2 = lib.pcg_solve(f, u, rtol=1e-8, x0_given=True)
    assert rc2 == 0 and info2[0]["iters"] == 0
    # non-finite right-hand side
    bad = f.clone()
    bad[5] = float("nan")
    rc, info = lib.pcg_solve(bad, u, check=False)
    assert rc == stfd.EBREAKDOWN and info[0]["status"] == stfd.EBREAKDOWN
    # one good and one non-finite system in a batch: the good one still converges
    both = torch.cat([f, bad])
    ub = torch.empty_like(both)
    rc, info = lib.pcg_solve(both, ub, nrhs=2, check=False)
    assert rc == stfd.EBREAKDOWN and info[0]["status"] == 0 and info[1]["status"] == stfd.EBREAKDOWN
    # argument errors (nrhs above max_nrhs = 2 is rejected by the library)
    big = torch.zeros(3 * N, dtype=torch.complex128, device=DEV)
    with pytest.raises(stfd.StfdError):
        lib.apply_preconditioner(big, big.clone(), nrhs=3)
    with pytest.raises(stfd.StfdError):
        lib.apply_preconditioner(f, u, precision=7)
    with pytest.raises(stfd.StfdError):
        lib.matvec(f, f)
    # the apply may run in place
    s1 = torch.empty_like(f)
    lib.apply_preconditioner(f, s1)
    g = f.clone()
    lib.apply_preconditioner(g, g)
    assert torch.equal(g, s1)


def test_repeatable_bitwise():
    lib, _ = make_pair(3, 8, 3, None, oracle=False)
    f = to_dev(inputs.random_complex(lib.N, 40))
    u1, u2 = torch.empty_like(f), torch.empty_like(f)
    lib.pcg_solve(f, u1)
    lib.pcg_solve(f, u2)
    assert torch.equal(u1, u2)
