"""Learned warm start: the scaled initial guess of PCG and a small end-to-end training run."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_18461_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stfd():
    from paper_2311_18461_amd import stfd
    return stfd


def test_scaled_initial_guess():
    """alpha = Re<x0,f>/<x0,A x0>: a multiple of the solution is rescaled onto it; a guess pointing
    away from it is replaced by the cold start."""
    stfd = _stfd()
    kn = inputs.uniform_open_knots(10, 3)
    V = inputs.gaussian_potential(2, 2000)
    pr = stfd.Problem(kn, [kn, kn], 3, 3, V_quad=stfd.sample_on_quad_grid(V, [kn, kn], 3))
    f = torch.from_numpy(inputs.random_complex(pr.N, 1)).to(DEV)
    u = torch.empty_like(f)
    rc, cold = pr.pcg_solve(f, u, rtol=1e-12, maxit=1000)
    sol = u.clone()
    x = 0.5 * sol
    rc, info = pr.pcg_solve(f, x, rtol=1e-8, maxit=1000, x0_scaled=True)
    assert abs(info[0]["x0_scale"] - 2.0) < 1e-8 and info[0]["iters"] <= 1
    x = -0.7 * sol
    rc, info = pr.pcg_solve(f, x, rtol=1e-8, maxit=1000, x0_scaled=True)
    _, cold8 = pr.pcg_solve(f, u, rtol=1e-8, maxit=1000)
    assert info[0]["x0_scale"] == 0.0 and info[0]["iters"] == cold8[0]["iters"]
    x = torch.from_numpy(inputs.random_complex(pr.N, 2)).to(DEV)
    rc, info = pr.pcg_solve(f, x, rtol=1e-8, maxit=1000, x0_scaled=True)
    assert rc == 0 and info[0]["true_rel_res"] <= 1.2e-8 and 0.0 <= info[0]["x0_scale"] < 1.0


def test_warm_start_pipeline_small():
    """Solver-generated data, FNO training on the device, evaluation with the scaled warm start
    (annulus, p = 4, 8^3 elements): the training loss falls and every warm solve meets the tolerance."""
    from paper_2311_18461_amd import warmstart
    wl = warmstart.AnnulusWorkload(n_el=8)
    feats, targets, iters = warmstart.generate(wl, warmstart.TRAIN_SEED0, 24)
    assert feats.shape == (24, wl.ns, wl.ns, 5) and targets.shape == (24, 2 * wl.N)
    net, hist = warmstart.train(wl, feats, targets, epochs=40, batch=8, lr=3e-3)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.8 * hist[0]
    rows = warmstart.evaluate(wl, net, warmstart.TEST_SEED0, 3)
    for r in rows:
        assert r["warm_true_rel_res"] <= 1.2e-8 and r["solution_diff"] < 1e-6
