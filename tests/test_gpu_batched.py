"""Batched PCG over uneven grids (stfd_pcg_solve_batched) and graph-replayed iterations.

Every kernel of the batched path is the single-problem kernel, each job on its own stream
inside one captured graph per iteration parity, so each system's iterate must equal the
one of a single-problem solve bit for bit (reductions are deterministic), and every graph
replay of a solve is checked by that comparison.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_18461_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stfd():
    from paper_2311_18461_amd import stfd
    return stfd


def _problem(n_el, p=3, V=None, max_nrhs=1):
    stfd = _stfd()
    kt, ks = inputs.uniform_open_knots(n_el, p), [inputs.uniform_open_knots(n_el, p)] * 2
    Vq = stfd.sample_on_quad_grid(V, ks, p) if V is not None else None
    return stfd.Problem(kt, ks, p, p, 1.0, 1.0, V_quad=Vq, max_nrhs=max_nrhs)


def _rhs(prob, packets):
    """Stacked load vectors of wave-packet initial data (f = 0)."""
    u0 = np.concatenate([prob.sample_space(w) for w in packets])
    fb = torch.empty(prob.N * len(packets), dtype=torch.complex128, device=DEV)
    prob.load_vector(fb, u0_q=torch.from_numpy(u0).to(DEV), nrhs=len(packets))
    return fb


@pytest.mark.parametrize("nrhs", [1, 3])
def test_graph_replay_equals_direct(nrhs):
    """PCG with every iteration replayed from a captured graph gives the direct launch's iterates."""
    prob = _problem(16, V=inputs.gaussian_potential(2, 2000), max_nrhs=nrhs)
    f = torch.from_numpy(inputs.random_complex(prob.N * nrhs, 11)).to(DEV)
    u1, u2 = torch.empty_like(f), torch.empty_like(f)
    rc1, i1 = prob.pcg_solve(f, u1, nrhs=nrhs, rtol=1e-9, maxit=1000)
    scratch = torch.randn(1 << 20, device=DEV)  # eager work between the solves
    scratch.mul_(2.0).sum().item()
    rc2, i2 = prob.pcg_solve(f, u2, nrhs=nrhs, rtol=1e-9, maxit=1000, graph=True)
    assert rc1 == rc2 == 0
    assert [a["iters"] for a in i1] == [b["iters"] for b in i2]
    assert torch.equal(u1, u2)


def test_batched_uneven_grids_equal_single_solves():
    """64 wave-packet systems over 16^3, 24^3, 32^3, 48^3, 64^3 (p = 3, V = 0) in one batched call:
    each system's solution and iteration count equal its own single-system solve."""
    stfd = _stfd()
    work = inputs.batched_2d_workload()
    probs, fs, us, nr = [], [], [], []
    for n_el, packets in work.items():
        pr = _problem(n_el, max_nrhs=len(packets))
        probs.append(pr)
        fs.append(_rhs(pr, packets))
        us.append(torch.empty_like(fs[-1]))
        nr.append(len(packets))
    assert sum(nr) == 64 and nr == [13, 13, 13, 13, 12]
    rc, info = stfd.pcg_solve_batched(probs, fs, us, nr, rtol=1e-8, maxit=200)
    assert rc == 0
    k = 0
    for pr, f, u, n in zip(probs, fs, us, nr):
        for j in range(n):
            fj = f[j * pr.N:(j + 1) * pr.N].clone()
            uj = torch.empty_like(fj)
            rcj, ij = pr.pcg_solve(fj, uj, rtol=1e-8, maxit=200)
            assert rcj == 0 and info[k]["status"] == 0
            assert info[k]["iters"] == ij[0]["iters"], (pr.n_t, j)
            assert info[k]["true_rel_res"] <= 1.2e-8
            assert torch.equal(u[j * pr.N:(j + 1) * pr.N], uj), (pr.n_t, j)
            k += 1
    # a second batched call reuses nothing from the first: same answers
    us2 = [torch.empty_like(u) for u in us]
    rc2, info2 = stfd.pcg_solve_batched(probs, fs, us2, nr, rtol=1e-8, maxit=200)
    assert rc2 == 0 and all(torch.equal(a, b) for a, b in zip(us, us2))
    assert [a["iters"] for a in info] == [b["iters"] for b in info2]


def test_batched_argument_errors():
    stfd = _stfd()
    pr = _problem(8, max_nrhs=2)
    f = torch.zeros(pr.N, dtype=torch.complex128, device=DEV)
    u = torch.empty_like(f)
    with pytest.raises(stfd.StfdError) as ei:  # the same handle twice
        stfd.pcg_solve_batched([pr, pr], [f, f], [u, u], [1, 1])
    assert ei.value.code == stfd.EINVAL
    with pytest.raises(stfd.StfdError) as ei:  # more systems than the handle was set up for
        f3 = torch.zeros(pr.N * 3, dtype=torch.complex128, device=DEV)
        stfd.pcg_solve_batched([pr], [f3], [torch.empty_like(f3)], [3])
    assert ei.value.code == stfd.EINVAL
    rc, info = stfd.pcg_solve_batched([pr], [f], [u], [1])  # f = 0: u = 0 at once
    assert rc == 0 and info[0]["iters"] == 0 and torch.all(u == 0).item()


def test_cached_graphs_replay_across_solves():
    """Captured iterations are kept in the handle and replayed by later solves with the same
    arguments: each replay (with eager work and host synchronisations between) equals the direct
    solve of the data then in the buffers; new launch shapes drop the cache; more argument sets
    than the cache holds evict the oldest."""
    prob = _problem(16, V=inputs.gaussian_potential(2, 2000))
    f = torch.empty(prob.N, dtype=torch.complex128, device=DEV)
    u_ref, u = torch.empty_like(f), torch.empty_like(f)
    extra = [torch.empty_like(f) for _ in range(5)]
    for rep, seed in enumerate((12, 12, 13, 14)):
        f.copy_(torch.from_numpy(inputs.random_complex(prob.N, seed)))
        if rep == 3:
            prob.set_mode_product_shapes({"fp64": [2, 2]})
        rc1, i1 = prob.pcg_solve(f, u_ref, rtol=1e-9, maxit=1000)
        torch.randn(1 << 20, device=DEV).mul_(2.0).sum().item()  # eager work between
        rc2, i2 = prob.pcg_solve(f, u, rtol=1e-9, maxit=1000, graph=True)
        torch.cuda.synchronize()
        assert rc1 == rc2 == 0
        assert i1[0]["iters"] == i2[0]["iters"] and torch.equal(u_ref, u), rep
    for k, x in enumerate(extra + extra[:2]):  # seven argument sets through a cache of four
        rc, info = prob.pcg_solve(f, x, rtol=1e-9, maxit=1000, graph=True)
        assert rc == 0 and torch.equal(x, u_ref), k


def test_batched_graph_replay_equals_streams():
    """The batched driver with cached per-job graphs, called twice, gives the direct batched result."""
    stfd = _stfd()
    work = {n: ps[:3] for n, ps in inputs.batched_2d_workload().items() if n <= 32}
    probs, fs, nr = [], [], []
    for n_el, packets in work.items():
        pr = _problem(n_el, max_nrhs=len(packets))
        probs.append(pr)
        fs.append(_rhs(pr, packets))
        nr.append(len(packets))
    us = [torch.empty_like(f) for f in fs]
    rc, info = stfd.pcg_solve_batched(probs, fs, us, nr, rtol=1e-8, maxit=200)
    assert rc == 0
    for rep in range(2):
        ug = [torch.empty_like(f) for f in fs] if rep == 0 else ug
        torch.randn(1 << 20, device=DEV).mul_(2.0).sum().item()
        rcg, infog = stfd.pcg_solve_batched(probs, fs, ug, nr, rtol=1e-8, maxit=200, graph=True)
        assert rcg == 0 and all(torch.equal(a, b) for a, b in zip(us, ug)), rep
        assert [a["iters"] for a in info] == [b["iters"] for b in infog]
