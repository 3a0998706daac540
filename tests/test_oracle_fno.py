"""Pins of the oracle's spectral-convolution network (learned warm start).

The numpy.fft spectral convolution is checked against the truncated transform written out as
explicit sums; the hand-derived backward pass against central finite differences; the
relative-l2 loss gradient likewise.
"""
import numpy as np

from oracle import fno


def small_spec():
    return fno.Spec(H=6, W=7, c_in=3, width=4, modes1=3, modes2=4, layers=2, proj=5, c_out=4)


def test_spectral_conv_matches_explicit_sums():
    spec = small_spec()
    rng = np.random.default_rng(0)
    h = rng.standard_normal((2, spec.H, spec.W, spec.width))
    R = rng.standard_normal((spec.M2, spec.M1, spec.width, spec.width)) + 1j * rng.standard_normal(
        (spec.M2, spec.M1, spec.width, spec.width))
    got, _ = fno.spectral_conv(spec, h, R)
    H, W = spec.H, spec.W
    i2 = np.arange(H)[:, None]
    i1 = np.arange(W)[None, :]
    want = np.zeros_like(got)
    for j in range(spec.M2):
        k2 = j if j < spec.M2 // 2 else j - spec.M2
        for k1 in range(spec.M1):
            e = np.exp(-2j * np.pi * (k1 * i1 / W + k2 * i2 / H))  # (H, W)
            hh = np.einsum("bhwc,hw->bc", h, e)
            g = hh @ R[j, k1]
            wk = 1.0 if k1 == 0 else 2.0
            want += wk * np.real(g[:, None, None, :] * np.conj(e)[None, :, :, None]) / (H * W)
    assert np.max(np.abs(got - want)) < 1e-12


def test_backward_matches_finite_differences():
    spec = small_spec()
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(spec.n_params()) * 0.3
    x = rng.standard_normal((2, spec.H, spec.W, spec.c_in))
    dy = rng.standard_normal((2, spec.H, spec.W, spec.c_out))
    y, cache = fno.forward(spec, theta, x)
    g, dx = fno.backward(spec, theta, cache, dy)
    f = lambda th, xx: np.sum(dy * fno.forward(spec, th, xx)[0])  # noqa: E731
    h = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (f(theta + e, x) - f(theta - e, x)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    for _ in range(10):
        k = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[k] = h
        fd = (f(theta, x + e) - f(theta, x - e)) / (2 * h)
        assert abs(fd - dx[k]) <= 1e-6 * max(1.0, abs(fd))


def test_rel_l2_gradient():
    rng = np.random.default_rng(2)
    y, t = rng.standard_normal((3, 20)), rng.standard_normal((3, 20))
    loss, g = fno.rel_l2(y, t)
    assert abs(loss - np.mean(np.linalg.norm(y - t, axis=1) / np.linalg.norm(t, axis=1))) < 1e-15
    h = 1e-6
    for _ in range(10):
        k = tuple(rng.integers(0, s) for s in y.shape)
        e = np.zeros_like(y)
        e[k] = h
        fd = (fno.rel_l2(y + e, t)[0] - fno.rel_l2(y - e, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8


def test_adam_first_step_moves_by_lr():
    """Bias correction makes the first Adam step lr * sign(g) (for |g| >> eps)."""
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.1])
    th1, m, v = fno.adam(th, g, np.zeros(5), np.zeros(5), 1, 1e-3, 0.9, 0.999, 1e-12)
    assert np.allclose(th1, -1e-3 * np.sign(g), rtol=1e-9)
