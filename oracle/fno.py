"""Spectral-convolution network of the learned warm start: plain FP64 NumPy forward and backward.

Test infrastructure: see the package docstring.

The network and its flat parameter layout are those declared in include/stfd_fno.h.  The
spectral convolution here uses numpy.fft (full 2D transform, then the retained
frequencies), an implementation independent of the library's truncated-DFT GEMMs; the
backward pass is derived by hand and pinned by central finite differences in the tests.
Adam follows Kingma & Ba (2015) with bias correction.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


class Spec:
    def __init__(self, H, W, c_in, width, modes1, modes2, layers, proj, c_out):
        self.H, self.W, self.c_in, self.width = H, W, c_in, width
        self.M1, self.M2, self.L, self.proj, self.c_out = modes1, modes2, layers, proj, c_out

    def k2_index(self):
        """Rows of the full spectrum kept along i_2: j -> k2 = j (j < M2/2) or j - M2."""
        return np.array([j if j < self.M2 // 2 else self.H + j - self.M2 for j in range(self.M2)])

    def split(self, theta):
        """Parameter views (Wp, bp, [(W, b, R complex)], Q1, q1, Q2, q2) of a flat vector."""
        o = 0
        C, M1, M2 = self.width, self.M1, self.M2

        def take(n, shape):
            nonlocal o
            v = theta[o:o + n].reshape(shape)
            o += n
            return v
        Wp = take(self.c_in * C, (self.c_in, C))
        bp = take(C, (C,))
        layers = []
        for _ in range(self.L):
            W = take(C * C, (C, C))
            b = take(C, (C,))
            Rr = take(M2 * M1 * C * C, (M2, M1, C, C))
            Ri = take(M2 * M1 * C * C, (M2, M1, C, C))
            layers.append((W, b, Rr + 1j * Ri))
        Q1 = take(C * self.proj, (C, self.proj))
        q1 = take(self.proj, (self.proj,))
        Q2 = take(self.proj * self.c_out, (self.proj, self.c_out))
        q2 = take(self.c_out, (self.c_out,))
        assert o == theta.size
        return Wp, bp, layers, Q1, q1, Q2, q2

    def n_params(self):
        C = self.width
        return (self.c_in * C + C + self.L * (C * C + C + 2 * self.M2 * self.M1 * C * C)
                + C * self.proj + self.proj + self.proj * self.c_out + self.c_out)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def spectral_conv(spec: Spec, h, R):
    """K(h) for h [B, H, W, C] and complex R [M2, M1, C, C]; returns (out, X) with X the retained
    spectrum [B, M2, M1, C]."""
    F = np.fft.fft2(h, axes=(1, 2))
    rows = spec.k2_index()
    X = F[:, rows, :spec.M1, :]
    Y = np.einsum("bjkc,jkco->bjko", X, R)
    w = np.where(np.arange(spec.M1) == 0, 1.0, 2.0)
    Z = np.zeros(h.shape[:3] + (R.shape[-1],), dtype=np.complex128)
    Z[:, rows, :spec.M1, :] = Y * w[None, None, :, None]
    return np.real(np.fft.ifft2(Z, axes=(1, 2))), X


def spectral_conv_bwd(spec: Spec, X, R, dout):
    """Gradients (dh, dR) of sum(dout * K(h)) given the retained spectrum X of h."""
    H, W = spec.H, spec.W
    rows = spec.k2_index()
    w = np.where(np.arange(spec.M1) == 0, 1.0, 2.0)
    dZ = np.fft.fft2(dout, axes=(1, 2)) / (H * W)
    dY = dZ[:, rows, :spec.M1, :] * w[None, None, :, None]
    dR = np.einsum("bjkc,bjko->jkco", np.conj(X), dY)
    dX = np.einsum("bjko,jkco->bjkc", dY, np.conj(R))
    full = np.zeros(dout.shape[:3] + (X.shape[-1],), dtype=np.complex128)
    full[:, rows, :spec.M1, :] = dX
    dh = np.real(np.fft.ifft2(full, axes=(1, 2))) * (H * W)
    return dh, dR


def forward(spec: Spec, theta, x):
    """y = net(x) for x [B, H, W, c_in]; returns (y, cache)."""
    Wp, bp, layers, Q1, q1, Q2, q2 = spec.split(np.asarray(theta, dtype=np.float64))
    a = x @ Wp + bp
    cache = {"x": x, "a": [a], "z": [], "X": []}
    for l, (W, b, R) in enumerate(layers):
        s, X = spectral_conv(spec, a, R)
        z = a @ W + b + s
        cache["z"].append(z)
        cache["X"].append(X)
        a = gelu(z) if l < spec.L - 1 else z
        cache["a"].append(a)
    p1 = a @ Q1 + q1
    g1 = gelu(p1)
    y = g1 @ Q2 + q2
    cache.update(p1=p1, g1=g1)
    return y, cache


def backward(spec: Spec, theta, cache, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters and to x."""
    theta = np.asarray(theta, dtype=np.float64)
    Wp, bp, layers, Q1, q1, Q2, q2 = spec.split(theta)
    grads = {}
    flat = lambda t: t.reshape(-1, t.shape[-1])  # noqa: E731
    grads["Q2"] = flat(cache["g1"]).T @ flat(dy)
    grads["q2"] = flat(dy).sum(0)
    dp = (dy @ Q2.T) * gelu_prime(cache["p1"])
    aL = cache["a"][-1]
    grads["Q1"] = flat(aL).T @ flat(dp)
    grads["q1"] = flat(dp).sum(0)
    da = dp @ Q1.T
    lg = [None] * spec.L
    for l in reversed(range(spec.L)):
        W, b, R = layers[l]
        dz = da if l == spec.L - 1 else da * gelu_prime(cache["z"][l])
        al = cache["a"][l]
        dWl = flat(al).T @ flat(dz)
        dbl = flat(dz).sum(0)
        dh, dR = spectral_conv_bwd(spec, cache["X"][l], R, dz)
        da = dz @ W.T + dh
        lg[l] = (dWl, dbl, dR)
    grads["Wp"] = flat(cache["x"]).T @ flat(da)
    grads["bp"] = flat(da).sum(0)
    dx = da @ Wp.T
    parts = [grads["Wp"], grads["bp"]]
    for dWl, dbl, dR in lg:
        parts += [dWl, dbl, np.real(dR), np.imag(dR)]
    parts += [grads["Q1"], grads["q1"], grads["Q2"], grads["q2"]]
    return np.concatenate([p.ravel() for p in parts]), dx


def rel_l2(y, t):
    """(1/B) sum_b ||y_b - t_b|| / ||t_b|| and its gradient with respect to y ([B, n])."""
    e = y - t
    en = np.linalg.norm(e, axis=1)
    tn = np.linalg.norm(t, axis=1)
    B = y.shape[0]
    loss = float(np.mean(en / tn))
    grad = e / (B * en[:, None] * tn[:, None])
    return loss, grad


def adam(theta, g, m, v, step, lr, b1, b2, eps):
    """One Adam update (step counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
