"""The allocation-free apply (stfd_apply_preconditioner_static) against stfd_apply_preconditioner,
called through the C ABI.

Both run the same kernels on the same operands, so the outputs must agree bit for bit; the
static variant keeps its intermediates in the library's fixed device scratch, which every call
on the GPU shares, so two calls in a row (the second smaller) must not see each other's data.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_18461_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(d, n_el, p, max_nrhs=1):
    from paper_2311_18461_amd import stfd
    kt, ks = inputs.uniform_open_knots(n_el, p), [inputs.uniform_open_knots(n_el + l, p) for l in range(d)]
    return stfd.Problem(kt, ks, p, p, max_nrhs=max_nrhs, rhs_workspace=False)


def _call_static(prob, r, s, nrhs, prec):
    """Direct C-ABI call (no binding helper between the test and the library)."""
    from paper_2311_18461_amd import stfd
    lib = stfd._lib()
    return lib.stfd_apply_preconditioner_static(prob._h, ctypes.c_void_p(r.data_ptr()),
                                                ctypes.c_void_p(s.data_ptr()), nrhs, stfd.PRECISIONS[prec],
                                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_static_apply_matches_apply_twice(prec):
    print(f"static apply {prec}: 2D p=3 64^3 nrhs=3, then 3D p=3 6^4 nrhs=1", flush=True)
    big = _problem(2, 64, 3, max_nrhs=3)
    small = _problem(3, 6, 3)
    for prob, nrhs, seed in ((big, 3, 50), (small, 1, 51)):
        r = torch.from_numpy(np.concatenate([inputs.random_complex(prob.N, seed + k) for k in range(nrhs)])).to(DEV)
        want = torch.empty_like(r)
        got = torch.full_like(r, float("nan"))
        prob.apply_preconditioner(r, want, nrhs=nrhs, precision=prec)
        assert _call_static(prob, r, got, nrhs, prec) == 0
        torch.cuda.synchronize()
        assert torch.equal(got, want), prec


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_apply_with_the_fused_last_direction(prec):
    """The fused last-direction launch works in place in the scratch's intermediate: the static
    apply equals the regular one with the fused form on, twice (3D 13 x 14 x 15 x 11, then 9^3 x 8)."""
    print(f"static apply {prec} with the fused last direction", flush=True)
    for n_el, seed in ((12, 52), (8, 53)):
        prob = _problem(3, n_el, 3)
        prob.set_fused_time(True)
        r = torch.from_numpy(inputs.random_complex(prob.N, seed)).to(DEV)
        want = torch.empty_like(r)
        got = torch.full_like(r, float("nan"))
        prob.apply_preconditioner(r, want, precision=prec)
        assert _call_static(prob, r, got, 1, prec) == 0
        torch.cuda.synchronize()
        assert torch.equal(got, want), (prec, n_el)


def test_static_apply_rejects_sizes_above_the_scratch():
    from paper_2311_18461_amd import stfd
    prob = _problem(2, 64, 3)
    r = torch.zeros(prob.N * 8, dtype=torch.complex128, device=DEV)
    s = torch.empty_like(r)
    # FP64: each intermediate holds 16 N bytes per right-hand side in a 32 MiB half -> nrhs <= 7
    assert _call_static(prob, r, s, 8, "fp64") == stfd.EINVAL
    assert _call_static(prob, r, s, 0, "fp64") == stfd.EINVAL
    assert _call_static(prob, r, s, 7, "fp64") == 0
    torch.cuda.synchronize()
