"""Host-only checks of the C ABI library: it loads, exports every declared
symbol, its Gauss rule matches the oracle's, and invalid setups are rejected
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.bspline import gauss_rule
from paper_2311_18461_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2311_18461_amd import stfd
    return stfd


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(stfd_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    stfd = _lib()
    lib = stfd._lib()
    names = _declared_functions()
    assert len(names) >= 25 and "stfd_fno_forward" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in stfd.SIGNATURES, name


def test_strerror():
    stfd = _lib()
    assert stfd._lib().stfd_strerror(stfd.EINVAL) == b"invalid argument"
    assert stfd._lib().stfd_strerror(1234) == b"unknown status"


@pytest.mark.parametrize("n_el,p,q,scale", [(5, 2, 0, 1.0), (7, 3, 0, 2.0), (4, 4, 6, 1.0)])
def test_quad_points_match_oracle(n_el, p, q, scale):
    stfd = _lib()
    kn = inputs.uniform_open_knots(n_el, p)
    pts, wts = stfd.quad_points(kn, p, q, scale)
    x, w, _ = gauss_rule(kn * scale, q or p + 1)
    np.testing.assert_allclose(pts, x, atol=1e-15 * scale)
    np.testing.assert_allclose(wts, w, rtol=1e-13)


def test_quad_points_graded_and_repeated():
    stfd = _lib()
    kn = np.array([0, 0, 0, 0.2, 0.5, 0.5, 0.8, 1, 1, 1.0])
    pts, wts = stfd.quad_points(kn, 2)
    x, w, _ = gauss_rule(kn, 3)
    np.testing.assert_allclose(pts, x, atol=1e-15)
    np.testing.assert_allclose(wts, w, rtol=1e-13)


BAD = {
    "p_s < 2": dict(p_s=1),
    "p_t < 1": dict(p_t=0),
    "nu <= 0": dict(nu=0.0),
    "T <= 0": dict(T=-1.0),
    "non-open knots": dict(knots_s=[np.array([0, 0, 0.1, 0.5, 1, 1, 1.0])]),
    "decreasing knots": dict(knots_s=[np.array([0, 0, 0, 0.6, 0.4, 1, 1, 1.0])]),
    "space not C1": dict(knots_s=[np.array([0, 0, 0, 0.5, 0.5, 1, 1, 1.0])]),
    "time not C0": dict(knots_t=np.array([0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1.0])),
    "knots outside [0,1]": dict(knots_t=np.array([0, 0, 0, 0.5, 1.5, 1.5, 1.5])),
}


@pytest.mark.parametrize("case", sorted(BAD))
def test_setup_rejects_invalid(case):
    stfd = _lib()
    args = dict(knots_t=inputs.uniform_open_knots(3, 2), knots_s=[inputs.uniform_open_knots(3, 2)],
                p_t=2, p_s=2, T=1.0, nu=1.0)
    args.update(BAD[case])
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(args["knots_t"], args["knots_s"], args["p_t"], args["p_s"], args["T"], args["nu"])
    assert ei.value.code == stfd.EINVAL


def test_setup_rejects_bad_d_and_nrhs():
    stfd = _lib()
    kn = inputs.uniform_open_knots(3, 2)
    with pytest.raises(stfd.StfdError):
        stfd.Problem(kn, [kn] * 4, 2, 2)
    with pytest.raises(stfd.StfdError):
        stfd.Problem(kn, [kn], 2, 2, max_nrhs=0)


def test_setup_rejects_sizes_above_the_limits():
    """n_l, n_t <= 128 for d = 2, 3 (one 16-column block of U_l per wave, one time line per point in
    the matvec's LDS); n_1 <= 1024 and n_t <= 2048 for d = 1 (the long-axis kernels).  Rejected from
    the knot counts, before any host or device work."""
    stfd = _lib()
    for kt, ks in ((inputs.uniform_open_knots(4, 2), [inputs.uniform_open_knots(130, 2)] * 2),
                   (inputs.uniform_open_knots(130, 2), [inputs.uniform_open_knots(4, 2)] * 2),
                   (inputs.uniform_open_knots(4, 2), [inputs.uniform_open_knots(1030, 2)]),
                   (inputs.uniform_open_knots(2050, 2), [inputs.uniform_open_knots(4, 2)])):
        with pytest.raises(stfd.StfdError) as ei:
            stfd.Problem(kt, ks, 2, 2)
        assert ei.value.code == stfd.EINVAL


def test_handle_entry_points_reject_null_handle():
    """Every entry point that takes a handle validates it before touching the device."""
    stfd = _lib()
    lib = stfd._lib()
    assert lib.stfd_load_vector(None, None, None, None, None, None, 1, None) == stfd.EINVAL
    assert lib.stfd_matvec(None, None, None, 1, None) == stfd.EINVAL
    assert lib.stfd_apply_preconditioner(None, None, None, 1, 0, None) == stfd.EINVAL
    assert lib.stfd_pcg_solve(None, None, None, 1, 1e-8, 10, 0, 0, None, None) == stfd.EINVAL
    assert lib.stfd_set_lift_max_iterations(None, 10) == stfd.EINVAL
    assert lib.stfd_get_tuning(None, ctypes.byref(stfd.Tuning())) == stfd.EINVAL
    assert lib.stfd_set_tuning(None, ctypes.byref(stfd.Tuning())) == stfd.EINVAL
    assert lib.stfd_get_precond_shift(None, ctypes.byref(ctypes.c_double())) == stfd.EINVAL


def test_fno_rejects_invalid_descriptors():
    """The network's shape checks run before any device work."""
    stfd = _lib()
    for kw in [dict(modes1=40), dict(modes2=7), dict(modes2=80), dict(width=0), dict(max_batch=0)]:
        args = dict(H=66, W=66, c_in=5, width=8, modes1=16, modes2=16, layers=2, proj=8, c_out=4, max_batch=1)
        args.update(kw)
        with pytest.raises(stfd.StfdError) as ei:
            stfd.Fno(**args)
        assert ei.value.code == stfd.EINVAL


def test_sumfac_matvec_rejected_where_it_does_not_apply():
    """STFD_MATVEC_SUMFAC needs the unit cube, d >= 2 and a potential that is a sum of 1D functions;
    the check runs on the host before any device work."""
    stfd = _lib()
    kn = inputs.uniform_open_knots(4, 3)
    cases = [dict(knots_s=[kn]),                                            # d = 1
             dict(knots_s=[kn, kn], geometry=stfd.GEOM_QUARTER_ANNULUS),    # mapped domain
             dict(knots_s=[kn] * 3, V=inputs.gaussian_potential(3, 31, count=3))]  # not separable
    for c in cases:
        ks = c["knots_s"]
        Vq = stfd.sample_on_quad_grid(c["V"], ks, 3) if "V" in c else None
        with pytest.raises(stfd.StfdError) as ei:
            stfd.Problem(kn, ks, 3, 3, V_quad=Vq, geometry=c.get("geometry", stfd.GEOM_UNIT_CUBE),
                         matvec=stfd.MATVEC_SUMFAC)
        assert ei.value.code == stfd.EINVAL
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(kn, [kn] * 2, 3, 3, matvec=7)
    assert ei.value.code == stfd.EINVAL


def test_time_condition_rejected_where_it_does_not_apply():
    """The ultraweak method (final time condition) runs on the unit cube only; unknown values of
    the time condition are rejected."""
    stfd = _lib()
    kn = inputs.uniform_open_knots(4, 3)
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(kn, [kn, kn], 3, 3, geometry=stfd.GEOM_QUARTER_ANNULUS, time_condition=stfd.TIME_FINAL)
    assert ei.value.code == stfd.EINVAL
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(kn, [kn], 3, 3, time_condition=2)
    assert ei.value.code == stfd.EINVAL


def test_precond_shift_rejected_where_it_does_not_apply():
    """The mean-potential shift runs on the unit cube only; unknown values are rejected."""
    stfd = _lib()
    kn = inputs.uniform_open_knots(4, 3)
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(kn, [kn, kn], 3, 3, geometry=stfd.GEOM_QUARTER_ANNULUS,
                     precond_shift=stfd.SHIFT_MEAN_POTENTIAL)
    assert ei.value.code == stfd.EINVAL
    with pytest.raises(stfd.StfdError) as ei:
        stfd.Problem(kn, [kn], 3, 3, precond_shift=3)
    assert ei.value.code == stfd.EINVAL


def test_time_mode_product_rejects_null_handle():
    stfd = _lib()
    ms = ctypes.c_double()
    assert stfd._lib().stfd_time_mode_product(None, 0, 0, 10, None, ctypes.byref(ms)) == stfd.EINVAL
