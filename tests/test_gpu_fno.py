"""GPU parity of the spectral-convolution network kernels against the FP64 oracle.

The library runs in FP32 (FMA GEMMs with K up to a few thousand per partial sum), the
oracle in FP64 with numpy.fft, so outputs agree to a few 1e-6 relative and gradients to
~1e-4 relative per parameter block (the mode-mixing weight gradients sum over the batch and
the spectrum, the largest reductions).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fno as ofno  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stfd():
    from paper_2311_18461_amd import stfd
    return stfd


NET_SHAPES = [
    dict(H=12, W=10, c_in=3, width=6, modes1=4, modes2=6, layers=2, proj=8, c_out=5),
    dict(H=18, W=18, c_in=5, width=8, modes1=6, modes2=6, layers=4, proj=16, c_out=10),
]


def _pair(cfg, batch, seed):
    stfd = _stfd()
    net = stfd.Fno(max_batch=batch, seed=seed, **cfg)
    spec = ofno.Spec(**cfg)
    assert net.n_params == spec.n_params()
    return net, spec


def _blocks(spec):
    """(name, start, stop) of every parameter block of the flat layout."""
    C, M1, M2 = spec.width, spec.M1, spec.M2
    sizes = [("Wp", spec.c_in * C), ("bp", C)]
    for l in range(spec.L):
        sizes += [(f"W{l}", C * C), (f"b{l}", C), (f"Rr{l}", M2 * M1 * C * C), (f"Ri{l}", M2 * M1 * C * C)]
    sizes += [("Q1", C * spec.proj), ("q1", spec.proj), ("Q2", spec.proj * spec.c_out), ("q2", spec.c_out)]
    out, o = [], 0
    for n, k in sizes:
        out.append((n, o, o + k))
        o += k
    return out


@pytest.mark.parametrize("ci", [0, 1])
def test_forward_backward_vs_oracle(ci):
    cfg = NET_SHAPES[ci]
    batch = 3
    net, spec = _pair(cfg, batch, seed=11 + ci)
    theta = net.get_params().astype(np.float64)
    rng = np.random.default_rng(ci)
    x = rng.standard_normal((batch, cfg["H"], cfg["W"], cfg["c_in"]))
    dy = rng.standard_normal((batch, cfg["H"], cfg["W"], cfg["c_out"]))
    xd = torch.from_numpy(x.astype(np.float32)).to(DEV)
    yd = torch.empty(batch * net.n_out, dtype=torch.float32, device=DEV)
    net.forward(xd.view(-1), yd, batch)
    y_ref, cache = ofno.forward(spec, theta, x)
    y = yd.cpu().numpy().reshape(y_ref.shape)
    ey = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
    dxd = torch.empty_like(xd).view(-1)
    net.backward(torch.from_numpy(dy.astype(np.float32)).to(DEV).view(-1), batch, dx=dxd)
    g = net.get_grads().astype(np.float64)
    g_ref, dx_ref = ofno.backward(spec, theta, cache, dy)
    edx = np.linalg.norm(dxd.cpu().numpy().reshape(dx_ref.shape) - dx_ref) / np.linalg.norm(dx_ref)
    print(f"config {ci}: forward {ey:.2e}, dx {edx:.2e}")
    assert ey < 2e-5 and edx < 2e-4
    for name, a, b in _blocks(spec):
        e = np.linalg.norm(g[a:b] - g_ref[a:b]) / max(np.linalg.norm(g_ref[a:b]), 1e-30)
        assert e < 2e-4, (name, e)


def test_rel_l2_and_adam_vs_oracle():
    stfd = _stfd()
    rng = np.random.default_rng(5)
    B, n = 4, 5000
    y, t = rng.standard_normal((B, n)), rng.standard_normal((B, n))
    yd, td = (torch.from_numpy(a.astype(np.float32)).to(DEV).view(-1) for a in (y, t))
    dyd = torch.empty_like(yd)
    loss = stfd.fno_rel_l2(yd, td, n, B, dy=dyd)
    loss_ref, g_ref = ofno.rel_l2(y.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64))
    assert abs(loss - loss_ref) < 1e-5 * loss_ref
    assert np.linalg.norm(dyd.cpu().numpy().reshape(B, n) - g_ref) < 1e-5 * np.linalg.norm(g_ref)
    # Adam: three steps with fixed gradients from one backward
    cfg = NET_SHAPES[0]
    net, spec = _pair(cfg, 2, seed=3)
    x = torch.from_numpy(rng.standard_normal(2 * net.n_in).astype(np.float32)).to(DEV)
    out = torch.empty(2 * net.n_out, dtype=torch.float32, device=DEV)
    net.forward(x, out, 2)
    net.backward(torch.ones_like(out), 2)
    g = net.get_grads().astype(np.float64)
    th = net.get_params().astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 4):
        net.adam_step(1e-3, 0.9, 0.999, 1e-8)
        th, m, v = ofno.adam(th, g, m, v, step, 1e-3, 0.9, 0.999, 1e-8)
    assert np.max(np.abs(net.get_params() - th)) < 1e-6


def test_full_size_forward_vs_oracle():
    """The warm-start network at its real size: 66 x 66 grid, 5 inputs, width 32, 16 x 16 modes,
    4 layers, projection 128 -> 134 outputs."""
    cfg = dict(H=66, W=66, c_in=5, width=32, modes1=16, modes2=16, layers=4, proj=128, c_out=134)
    batch = 2
    net, spec = _pair(cfg, batch, seed=7)
    theta = net.get_params().astype(np.float64)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((batch, 66, 66, 5))
    yd = torch.empty(batch * net.n_out, dtype=torch.float32, device=DEV)
    net.forward(torch.from_numpy(x.astype(np.float32)).to(DEV).view(-1), yd, batch)
    y_ref, cache = ofno.forward(spec, theta, x)
    ey = np.linalg.norm(yd.cpu().numpy().reshape(y_ref.shape) - y_ref) / np.linalg.norm(y_ref)
    dy = rng.standard_normal(y_ref.shape)
    net.backward(torch.from_numpy(dy.astype(np.float32)).to(DEV).view(-1), batch)
    g = net.get_grads().astype(np.float64)
    g_ref, _ = ofno.backward(spec, theta, cache, dy)
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"full size: forward {ey:.2e}, gradient {eg:.2e}")
    assert ey < 2e-5 and eg < 2e-4
