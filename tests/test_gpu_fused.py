"""GPU parity of the fused last direction (the products along x_d and the time solves of Algorithm 1
in one launch, one block per spatial column; stfd_tuning.fused_time).

The fused apply is compared element by element with the oracle's fast diagonalisation (bounds of
the separate-launch parity tests: FP64 1e-11 entrywise and 1e-10 per time fibre, FP32 2e-5) and
with the separate launches on the same handle: the MFMA chains run in the same order, and the time
solves differ only in their segment length (a rounding-level change: 1e-13 of the largest entry in
FP64).  Shapes cover ragged column groups (n_d not a multiple of 16), ragged last time segments,
p = 3 and 4, several right-hand sides with converged ones skipped, and PCG through the fused apply.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import FastDiagonalization, Problem as OProblem  # noqa: E402
from paper_2311_18461_amd import inputs  # noqa: E402
from parity import fiber_rel, max_rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _make(n_el, p, n_el_t=None, kind="harm", oracle=True, **kw):
    from paper_2311_18461_amd import stfd
    V = inputs.harmonic_potential(3, 3000) if kind == "harm" else None
    kt = inputs.uniform_open_knots(n_el_t or n_el, p)
    ks = [inputs.uniform_open_knots(n_el + l, p) for l in range(3)]
    Vq = stfd.sample_on_quad_grid(V, ks, p) if V is not None else None
    lib = stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=Vq, **kw)
    ref = OProblem(kt, ks, p, p, 1.0, V) if oracle else None
    return lib, ref


def _apply(lib, r, fused, precision="fp64"):
    lib.set_fused_time(fused)
    rd = torch.from_numpy(r).to(DEV)
    out = torch.empty_like(rd)
    lib.apply_preconditioner(rd, out, precision=precision, nrhs=r.size // lib.N)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n_el,p,n_el_t", [(12, 3, 9), (14, 3, 47), (10, 4, 13), (20, 4, 7)])
def test_fused_apply_vs_oracle_and_separate(n_el, p, n_el_t):
    lib, ref = _make(n_el, p, n_el_t)
    t = lib.get_tuning()
    print(f"fused n_s={lib.n_s} n_t={lib.n_t} p={p}: segment {t['fused_segment_length']}, "
          f"factor in kernel {t['fused_factors_in_kernel']}", flush=True)
    assert t["fused_segment_length"] > 0
    r = inputs.random_complex(lib.N, 81)
    s_ref = FastDiagonalization(ref, precompute_inverse=False).apply(r)
    s_f = _apply(lib, r, True)
    s_s = _apply(lib, r, False)
    e_max, e_fib = max_rel(s_f, s_ref), fiber_rel(s_f, s_ref, lib.n_t)
    d_sep = np.max(np.abs(s_f - s_s)) / np.max(np.abs(s_s))
    print(f"  fp64: max {e_max:.2e} fibre {e_fib:.2e}; vs separate launches {d_sep:.2e}", flush=True)
    assert e_max < 1e-11 and e_fib < 1e-10
    assert d_sep < 1e-13
    f32 = _apply(lib, r, True, "fp32")
    s32 = _apply(lib, r, False, "fp32")
    d32 = np.max(np.abs(f32 - s32)) / np.max(np.abs(s32))
    print(f"  fp32: max {max_rel(f32, s_ref):.2e}; vs separate launches {d32:.2e}", flush=True)
    assert max_rel(f32, s_ref) < 2e-5
    assert d32 < 1e-5


def test_fused_several_rhs_equal_single():
    lib, _ = _make(12, 3, 11, oracle=False, max_nrhs=3)
    r = inputs.random_complex(3 * lib.N, 82)
    s3 = _apply(lib, r, True)
    for k in range(3):
        s1 = _apply(lib, r[k * lib.N:(k + 1) * lib.N], True)
        assert np.array_equal(s1, s3[k * lib.N:(k + 1) * lib.N])


def test_fused_pcg_matches_separate():
    """PCG to 1e-10 through the fused apply: the oracle's residual, and the same solution as with
    the separate launches."""
    lib, ref = _make(10, 3, 12)
    f = inputs.random_complex(lib.N, 83)
    fd = torch.from_numpy(f).to(DEV)
    sols, its = [], []
    for fused in (True, False):
        lib.set_fused_time(fused)
        u = torch.empty_like(fd)
        rc, info = lib.pcg_solve(fd, u, rtol=1e-10, maxit=500)
        assert rc == 0
        sols.append(u.cpu().numpy())
        its.append(info[0]["iters"])
        if fused:
            # replayed from captured iterations (twice: capture, then the cached graphs)
            ug = torch.empty_like(fd)
            for _ in range(2):
                ug.fill_(float("nan"))
                rcg, infog = lib.pcg_solve(fd, ug, rtol=1e-10, maxit=500, graph=True)
                torch.cuda.synchronize()
                assert rcg == 0 and infog[0]["iters"] == its[-1] and torch.equal(ug, u)
    x = sols[0]
    res = np.linalg.norm(f - ref.matvec(x)) / np.linalg.norm(f)
    print(f"fused PCG: {its[0]} iterations (separate {its[1]}), residual {res:.2e}", flush=True)
    assert res <= 1.2e-10
    assert abs(its[0] - its[1]) <= 1
    assert np.linalg.norm(x - sols[1]) <= 1e-8 * np.linalg.norm(x)


def test_fused_not_available_is_rejected():
    """d = 1 (one column) has no fused form: its segment field is 0 and switching it on fails."""
    from paper_2311_18461_amd import stfd
    kn = inputs.uniform_open_knots(16, 3)
    lib = stfd.Problem(kn, [kn], 3, 3, 1.0, 1.0)
    t = lib.get_tuning()
    assert t["fused_segment_length"] == 0 and not t["fused_time"]
    with pytest.raises(stfd.StfdError) as ei:
        lib.set_fused_time(True)
    assert ei.value.code == stfd.EINVAL
    lib.set_fused_time(False)


def test_fused_bitwise_equal_with_the_same_segment_length():
    """21 x 22 x 23 x 50 (p = 3): the separate time solve takes segments of 8 computed from the entry
    states (a grid of more than 4 blocks per CU); with the fused segment length set to 8 the two
    paths run the same arithmetic in the same order, FP64 and FP32."""
    lib, _ = _make(20, 3, 48, oracle=False, fused_segment_length=8)
    t = lib.get_tuning()
    assert (t["time_segment_length"], t["time_factors_in_kernel"]) == (8, True)
    assert (t["fused_segment_length"], t["fused_factors_in_kernel"]) == (8, True)
    r = inputs.random_complex(lib.N, 84)
    for prec in ("fp64", "fp32"):
        a, b = _apply(lib, r, True, prec), _apply(lib, r, False, prec)
        assert np.array_equal(a, b), prec


def test_fused_segment_length_that_does_not_fit_is_rejected():
    from paper_2311_18461_amd import stfd
    with pytest.raises(stfd.StfdError) as ei:
        _make(6, 3, 5, oracle=False, fused_segment_length=5)
    assert ei.value.code == stfd.EINVAL


@pytest.mark.parametrize("n_el,p", [(48, 3), (32, 4)])
def test_fused_full_size_3d_equals_separate(n_el, p):
    """The 3D workloads at full size (49^3 x 50 and 34^3 x 35): the fused launch against the
    separate launches (themselves checked against the oracle at this size in
    test_gpu_precision3d)."""
    from paper_2311_18461_amd import stfd
    print(f"fused full size n_el={n_el} p={p}", flush=True)
    kn = inputs.uniform_open_knots(n_el, p)
    lib = stfd.Problem(kn, [kn] * 3, p, p, 1.0, 1.0, rhs_workspace=False)
    assert lib.get_tuning()["fused_segment_length"] > 0
    r = inputs.random_complex(lib.N, 85)
    for prec, bound in (("fp64", 1e-13), ("fp32", 2e-5)):
        a, b = _apply(lib, r, True, prec), _apply(lib, r, False, prec)
        d = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print(f"  {prec}: fused vs separate {d:.2e}", flush=True)
        assert d < bound
    lib.close()
