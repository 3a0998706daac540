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


def _time_solve_key(t):
    """What fixes the rounding of the time solves: the fused launch's segment length and form, or
    the separate launch's."""
    if t["fused_time"]:
        return ("fused", t["fused_segment_length"], t["fused_factors_in_kernel"])
    return ("separate", t["time_segment_length"], t["time_transfers_in_kernel"], t["time_factors_in_kernel"])


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
            assert rt in (1, 2, 3) and (rt == 1 or lib.n_s[l] <= 80)
    assert t["time_segment_length"] >= p and (lib.n_t + t["time_segment_length"] - 1) // t["time_segment_length"] <= 64
    r = inputs.random_complex(lib.N, 51)
    rd = torch.from_numpy(r).to(DEV)
    out, out_h = torch.empty_like(rd), torch.empty_like(rd)
    lib.apply_preconditioner(rd, out)
    heur.apply_preconditioner(rd, out_h)
    torch.cuda.synchronize()
    s, s_ref = out.cpu().numpy(), FastDiagonalization(ref, precompute_inverse=False).apply(r)
    assert max_rel(s, s_ref) < 1e-11 and fiber_rel(s, s_ref, lib.n_t) < 1e-10
    if _time_solve_key(t) == _time_solve_key(h):
        assert torch.equal(out, out_h)  # only the row groups differ: same arithmetic
    for prec in ("fp32", "bf16"):
        lib.apply_preconditioner(rd, out, precision=prec)
        heur.apply_preconditioner(rd, out_h, precision=prec)
        torch.cuda.synchronize()
        # two applies each within the FP32 bound of the oracle (2e-5; the time solves may differ in
        # form, e.g. FP32 factor rows computed in the solve against FP32 copies of FP64 tables)
        assert max_rel(out.cpu().numpy(), out_h.cpu().numpy()) < (4e-5 if prec == "fp32" else 2e-2)


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


@pytest.mark.parametrize("d,n_el,p,n_el_t", [(2, 64, 3, 64), (2, 15, 3, 21), (3, 16, 2, 11), (3, 31, 3, 7),
                                             (3, 48, 3, 9), (3, 32, 4, 35)])
def test_every_shape_gives_the_same_apply(d, n_el, p, n_el_t):
    """Shapes 1, 2 (one column group per wave, 1 or 2 row groups) and 3 (every column group per wave,
    U' in LDS) accumulate every output over the same K steps in the same order: the applies agree
    bit for bit in every precision, and the FP64 one matches the oracle.  The PCG with the fused dot
    products (whose partials depend on the shape) takes the same iteration count up to one.  The
    last direction runs as separate launches here, so that every direction takes every shape.
    48 x 48 x 48 x 9 (n = 49) has one remainder column in x_1, 32^3 x 35 at p = 4 (n = 34, n_t = 38)
    two in every direction: launches of at least 16,384 one-group waves compute them with vector
    FMAs, by the same sequence in every shape (FP64 and FP32; BF16 keeps its MFMA group)."""
    from paper_2311_18461_amd import stfd
    kt = inputs.uniform_open_knots(n_el_t, p)
    ks = [inputs.uniform_open_knots(n_el, p) for _ in range(d)]
    lib = stfd.Problem(kt, ks, p, p, 1.0, 1.0)
    lib.set_fused_time(False)
    r = inputs.random_complex(lib.N, 61)
    rd = torch.from_numpy(r).to(DEV)
    outs = {}
    for shape in (1, 2, 3):
        lib.set_mode_product_shapes({prec: [shape] * d for prec in ("fp64", "fp32", "bf16")})
        assert all(v == [shape] * d for v in lib.get_tuning()["mode_product_row_groups"].values())
        for prec in ("fp64", "fp32", "bf16"):
            out = torch.empty_like(rd)
            lib.apply_preconditioner(rd, out, precision=prec)
            outs[(shape, prec)] = out
    torch.cuda.synchronize()
    for prec in ("fp64", "fp32", "bf16"):
        assert torch.equal(outs[(1, prec)], outs[(2, prec)]) and torch.equal(outs[(1, prec)], outs[(3, prec)])
    if lib.N <= 400_000:
        ref = OProblem(kt, ks, p, p, 1.0)
        s_ref = FastDiagonalization(ref, precompute_inverse=False).apply(r)
        s = outs[(3, "fp64")].cpu().numpy()
        assert max_rel(s, s_ref) < 1e-11 and fiber_rel(s, s_ref, lib.n_t) < 1e-10
    its = []
    f = torch.from_numpy(inputs.random_complex(lib.N, 62)).to(DEV)
    u = torch.empty_like(f)
    for shape in (1, 3):
        lib.set_mode_product_shapes({prec: [shape] * d for prec in ("fp64", "fp32", "bf16")})
        rc, info = lib.pcg_solve(f, u, rtol=1e-9, maxit=500)
        assert rc == 0
        its.append(info[0]["iters"])
    assert abs(its[0] - its[1]) <= 1


def test_set_tuning_rejects_invalid_shapes():
    from paper_2311_18461_amd import stfd
    kt = inputs.uniform_open_knots(6, 3)
    lib = stfd.Problem(kt, [inputs.uniform_open_knots(90, 3), kt], 3, 3)  # n_1 = 91 > 80
    with pytest.raises(stfd.StfdError):
        lib.set_mode_product_shapes({"fp64": [2, 1]})
    with pytest.raises(stfd.StfdError):
        lib.set_mode_product_shapes({"fp64": [1, 4]})
    lib.set_mode_product_shapes({"fp64": [1, 3]})


def test_time_mode_product_measures_and_checks_arguments():
    """stfd_time_mode_product: a positive average per launch for every direction and precision,
    no longer than one launch bracketed by its own events (which also enclose the dispatch), and
    argument errors.  The applies afterwards are unchanged (it only uses the work buffers)."""
    from paper_2311_18461_amd import stfd
    kt = inputs.uniform_open_knots(16, 3)
    lib = stfd.Problem(kt, [kt, kt], 3, 3)
    r = torch.from_numpy(inputs.random_complex(lib.N, 63)).to(DEV)
    before, after = torch.empty_like(r), torch.empty_like(r)
    lib.apply_preconditioner(r, before)
    for l in range(2):
        for prec in ("fp64", "fp32", "bf16"):
            ms = lib.time_mode_product(l, prec, reps=50)
            assert 0.0 < ms < 1.0, (l, prec, ms)
    lib.timing_begin(capacity=8)
    lib.apply_preconditioner(r, after)
    tot, n = lib.timing_end()
    assert n == 4 and lib.time_mode_product(0, "fp64", reps=200) <= 1.5 * tot / n
    lib.apply_preconditioner(r, after)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    for bad in ((2, "fp64"), (-1, "fp64"), (0, 7)):
        with pytest.raises(stfd.StfdError) as ei:
            lib.time_mode_product(bad[0], bad[1], reps=5)
        assert ei.value.code == stfd.EINVAL
    with pytest.raises(stfd.StfdError):
        lib.time_mode_product(0, "fp64", reps=0)
