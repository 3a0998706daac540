"""Setup-time autotuning of the launch shapes (stfd_setup_desc.autotune, stfd_get_tuning).

The tuned shapes change only how the work is cut: the mode products compute every output with the
same K-step order whatever the row groups (bitwise equal applies when only those change), and the
time solve's segment length and transfer mode change the rounding of the segmented recurrences
(FP64 parity with the oracle as for the heuristic shapes).  PCG with the tuned shapes takes the
heuristic's iteration count up to the rounding-induced delay of one.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402
from parity import fiber_rel, max_rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _make(d, n_el, p, V, autotune, oracle=False):
    from paper_2311_18461_amd import stfd
    kt = inputs.uniform_open_knots(n_el, p)
    ks = [inputs.uniform_open_knots(n_el, p) for _ in range(d)]
    Vq = stfd.sample_on_quad_grid(V, ks, p) if V is not None else None
    lib = stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=Vq, autotune=autotune)
    return lib, (OProblem(kt, ks, p, p, 1.0, V) if oracle else None)


@pytest.mark.parametrize("d,n_el,p,kind", [(2, 64, 3, "gauss"), (2, 16, 3, None), (3, 12, 3, "harm"),
                                           (3, 20, 4, None)])
def test_tuned_shapes_valid_and_apply_matches_oracle(d, n_el, p, kind):
    V = inputs.gaussian_potential(d, 2000) if kind == "gauss" else (
        inputs.harmonic_potential(d, 3000) if kind == "harm" else None)
    lib, ref = _make(d, n_el, p, V, True, oracle=True)
    heur, _ = _make(d, n_el, p, V, False)
    t, h = lib.get_tuning(), heur.get_tuning()
    print(f"d={d} n_el={n_el} p={p}: tuned {t}, heuristic {h}")
    assert t["autotuned"] and not h["autotuned"]
    for prec, rts in t["mode_product_row_groups"].items():
        for l, rt in enumerate(rts):
            assert rt in (1, 2) and (rt == 1 or lib.n_s[l] <= 80)
    assert t["time_segment_length"] >= p and (lib.n_t + t["time_segment_length"] - 1) // t["time_segment_length"] <= 64
    r = inputs.random_complex(lib.N, 51)
    rd = torch.from_numpy(r).to(DEV)
    out, out_h = torch.empty_like(rd), torch.empty_like(rd)
    lib.apply_preconditioner(rd, out)
    heur.apply_preconditioner(rd, out_h)
    torch.cuda.synchronize()
    s, s_ref = out.cpu().numpy(), FastDiagonalization(ref, precompute_inverse=False).apply(r)
    assert max_rel(s, s_ref) < 1e-11 and fiber_rel(s, s_ref, lib.n_t) < 1e-10
    if (t["time_segment_length"], t["time_transfers_in_kernel"]) == (h["time_segment_length"],
                                                                      h["time_transfers_in_kernel"]):
        assert torch.equal(out, out_h)  # only the row groups differ: same arithmetic
    for prec in ("fp32", "bf16"):
        lib.apply_preconditioner(rd, out, precision=prec)
        heur.apply_preconditioner(rd, out_h, precision=prec)
        torch.cuda.synchronize()
        assert max_rel(out.cpu().numpy(), out_h.cpu().numpy()) < (1e-5 if prec == "fp32" else 2e-2)


def test_tuned_pcg_matches_heuristic():
    V = inputs.gaussian_potential(2, 2000)
    lib, _ = _make(2, 64, 3, V, True)
    heur, _ = _make(2, 64, 3, V, False)
    f = torch.from_numpy(inputs.random_complex(lib.N, 52)).to(DEV)
    u, u_h = torch.empty_like(f), torch.empty_like(f)
    for prec in ("fp64", "fp32"):
        rc, info = lib.pcg_solve(f, u, rtol=1e-8, maxit=1000, precision=prec)
        rc_h, info_h = heur.pcg_solve(f, u_h, rtol=1e-8, maxit=1000, precision=prec)
        assert rc == 0 and rc_h == 0
        assert abs(info[0]["iters"] - info_h[0]["iters"]) <= max(1, info_h[0]["iters"] // 50)
        assert (torch.linalg.vector_norm(u - u_h) / torch.linalg.vector_norm(u_h)).item() < 1e-6
