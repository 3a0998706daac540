"""GPU parity of the preconditioner shifted by the mean potential (STFD_SHIFT_MEAN_POTENTIAL).

The library computes c = mean of V on its Gauss grid and refactorises the time pencils with
nu lambda_i + c; the oracle applies P-hat_c (pinned against its dense inverse on CPU).  Bounds as
for the unshifted apply: 1e-11 entrywise and 1e-10 per time fibre.  The solve is checked through
the oracle's residual, and the iteration count against the unshifted preconditioner.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem, mean_potential  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402
from parity import fiber_rel, max_rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _make(d, n_el, p, V, shift, oracle=True):
    from paper_2311_18461_amd import stfd
    kt = inputs.uniform_open_knots(n_el, p)
    ks = [inputs.uniform_open_knots(n_el, p) for _ in range(d)]
    lib = stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=stfd.sample_on_quad_grid(V, ks, p),
                       precond_shift=stfd.SHIFT_MEAN_POTENTIAL if shift else stfd.SHIFT_NONE)
    return lib, (OProblem(kt, ks, p, p, 1.0, V) if oracle else None), ks


@pytest.mark.parametrize("d,n_el,p,kind", [(2, 64, 3, "gauss"), (2, 20, 4, "gauss"), (3, 12, 3, "harm"),
                                           (3, 32, 4, "harm")])
def test_shifted_apply_vs_oracle(d, n_el, p, kind):
    V = inputs.gaussian_potential(d, 2000) if kind == "gauss" else inputs.harmonic_potential(d, 3000)
    lib, ref, ks = _make(d, n_el, p, V, True)
    c = mean_potential(ks, p, V)
    # the two means sum the same samples in different orders (and the library's points come from its
    # own Gauss rule): agreement to rounding; the apply is compared with the library's constant
    assert abs(lib.precond_shift - c) <= 1e-10 * abs(c)
    c = lib.precond_shift
    r = inputs.random_complex(lib.N, 71)
    rd = torch.from_numpy(r).to(DEV)
    out = torch.empty_like(rd)
    lib.apply_preconditioner(rd, out)
    torch.cuda.synchronize()
    s, s_ref = out.cpu().numpy(), FastDiagonalization(ref, precompute_inverse=False, shift=c).apply(r)
    e_max, e_fib = max_rel(s, s_ref), fiber_rel(s, s_ref, lib.n_t)
    print(f"shifted apply d={d} n_el={n_el} p={p} c={c:.3f}: max {e_max:.2e} fibre {e_fib:.2e}")
    assert e_max < 1e-11 and e_fib < 1e-10
    lib.apply_preconditioner(rd, out, precision="fp32")
    torch.cuda.synchronize()
    assert max_rel(out.cpu().numpy(), s_ref) < 2e-5


def test_shift_cuts_pcg_iterations_on_the_gaussian_workload():
    """2D p = 3 64^3 with the 8-Gaussian potential: the shifted preconditioner reaches the same
    residual (checked with the oracle's matvec) in far fewer iterations."""
    V = inputs.gaussian_potential(2, 2000)
    lib, ref, _ = _make(2, 64, 3, V, True)
    plain, _, _ = _make(2, 64, 3, V, False, oracle=False)
    f = inputs.random_complex(lib.N, 72)
    fd = torch.from_numpy(f).to(DEV)
    u, u0 = torch.empty_like(fd), torch.empty_like(fd)
    rc, info = lib.pcg_solve(fd, u, rtol=1e-8, maxit=1000)
    rc0, info0 = plain.pcg_solve(fd, u0, rtol=1e-8, maxit=1000)
    print(f"iterations: shifted {info[0]['iters']}, plain {info0[0]['iters']}")
    assert rc == 0 and rc0 == 0
    assert info[0]["iters"] < 0.6 * info0[0]["iters"]
    x = u.cpu().numpy()
    assert np.linalg.norm(f - ref.matvec(x)) / np.linalg.norm(f) <= 1.2e-8
    assert np.linalg.norm(x - u0.cpu().numpy()) / np.linalg.norm(x) < 1e-6
