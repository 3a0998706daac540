"""Precision of the FD apply on the 3D workloads at their full size, against the CPU oracle.

The 3D space + time configurations (unit cube, p = 3 at 48^4 elements with about 5.9 million
complex unknowns, and p = 4 at 32^4 with about 1.4 million) run the mode products in FP64, in FP32
and in BF16 with FP32 accumulation (the eigendecomposition, the time factors and everything
outside the apply stay FP64).  The preconditioner is the V-free fast diagonalisation (Section 5,
Algorithm 1), so it is the same for V = 0 and for the harmonic potential.

Bounds.  FP64: two independent FP64 implementations of a backward-stable apply agree to
kappa * eps (see test_gpu_parity).  FP32: one rounding of each mode-product operand and of the
stored intermediates per direction (unit roundoff 6e-8, three directions there and back, growth
kappa(U_l)^2 <= 60) gives a few 1e-6 at most; BF16 operands (unit roundoff 3.9e-3) give a few
1e-2 at most.  The measured errors are printed.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402
from parity import fiber_rel, max_rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("n_el,p", [(48, 3), (32, 4)])
def test_apply_3d_full_size_vs_oracle(n_el, p):
    from paper_2311_18461_amd import stfd
    print(f"3D apply precision: n_el={n_el} p={p}", flush=True)
    kn = inputs.uniform_open_knots(n_el, p)
    lib = stfd.Problem(kn, [kn] * 3, p, p, 1.0, 1.0, rhs_workspace=False)
    ref = OProblem(kn, [kn] * 3, p, p, 1.0, None)
    fd = FastDiagonalization(ref, precompute_inverse=False)
    r = inputs.random_complex(lib.N, 3999)
    z_ref = fd.apply(r)
    rd = torch.from_numpy(r).to(DEV)
    out = torch.empty_like(rd)
    errs = {}
    for prec, bound in (("fp64", 1e-11), ("fp32", 2e-5), ("bf16", 5e-2)):
        lib.apply_preconditioner(rd, out, precision=prec)
        torch.cuda.synchronize()
        z = out.cpu().numpy()
        errs[prec] = max_rel(z, z_ref)
        assert errs[prec] < bound, (prec, errs[prec])
        if prec == "fp64":
            e_fib = fiber_rel(z, z_ref, lib.n_t)
            assert e_fib < 1e-10, e_fib
    print(f"N={lib.N}: max-norm relative error vs the FP64 oracle "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) + f"; fp64 per-fibre {e_fib:.2e}", flush=True)
    lib.close()


def test_pcg_3d_large_products_converge():
    """FP64 PCG to 1e-8 on the 3D p = 4, 32^4 harmonic workload (about 1.4 million unknowns).

    At this size the library runs its x_1 mode products with two 16-row groups per wave, the
    last backward one included, whose fused partial sums give <r, z_new> and <r, z_old> for the
    direction update.  A wrong partial changes beta and with it the iteration count: with one
    row group per wave this solve took 57 iterations.  The final residual is recomputed here
    with the library matvec (itself checked against the oracle in test_gpu_parity)."""
    from paper_2311_18461_amd import stfd
    print("3D PCG: n_el=32 p=4 harmonic potential", flush=True)
    w = inputs.harmonic_3d_workload(0, n_el=32, p=4, with_potential=True)
    ks = [w.knots_s()] * 3
    prob = stfd.Problem(w.knots_t(), ks, 4, 4, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, 4))
    f = torch.empty(prob.N, dtype=torch.complex128, device=DEV)
    prob.load_vector(f, u0_q=torch.from_numpy(prob.sample_space(w.u0)).to(DEV))
    u = torch.empty_like(f)
    rc, info = prob.pcg_solve(f, u, rtol=1e-8, maxit=200)
    q = torch.empty_like(f)
    prob.matvec(u, q)
    torch.cuda.synchronize()
    res = float(torch.linalg.vector_norm(f - q) / torch.linalg.vector_norm(f))
    print(f"iterations {info[0]['iters']}, relative residual {res:.2e}", flush=True)
    assert rc == stfd.OK
    assert res <= 1.05e-8
    assert info[0]["iters"] <= 70
    prob.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pcg_3d_p3_n48_harmonic(prec):
    """PCG to 1e-8 on the 3D p = 3, 48^4 harmonic workload (about 5.9 million unknowns) per
    preconditioner precision, FP64 outer loop.  The true residual is recomputed with the library
    matvec (checked against the oracle entry by entry in test_gpu_sumfac and test_gpu_parity)."""
    from paper_2311_18461_amd import stfd
    print(f"3D PCG: n_el=48 p=3 harmonic potential, {prec} preconditioner", flush=True)
    w = inputs.harmonic_3d_workload(0, n_el=48, p=3, with_potential=True)
    ks = [w.knots_s()] * 3
    prob = stfd.Problem(w.knots_t(), ks, 3, 3, w.T, w.nu, V_quad=stfd.sample_on_quad_grid(w.potential, ks, 3))
    f = torch.empty(prob.N, dtype=torch.complex128, device=DEV)
    prob.load_vector(f, u0_q=torch.from_numpy(prob.sample_space(w.u0)).to(DEV))
    u = torch.empty_like(f)
    rc, info = prob.pcg_solve(f, u, rtol=1e-8, maxit=400, precision=prec)
    q = torch.empty_like(f)
    prob.matvec(u, q)
    torch.cuda.synchronize()
    res = float(torch.linalg.vector_norm(f - q) / torch.linalg.vector_norm(f))
    print(f"{prec}: iterations {info[0]['iters']}, relative residual {res:.2e}", flush=True)
    prob.close()
    assert rc == stfd.OK and res <= 1.2e-8
    assert info[0]["iters"] <= {"fp64": 110, "fp32": 140}[prec]
