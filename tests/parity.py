"""Element-wise comparison helpers for the GPU parity tests.

A single relative 2-norm over millions of entries dilutes a wrong tile, a padded time segment
or a boundary row by the square root of the size, so the config-size checks here are
element-wise:
  * max_rel: max_i |got_i - want_i| / max_i |want_i|;
  * fiber_rel: the same per time fibre (the n_t coefficients of one spatial point, contiguous in
    the vector layout), each measured against its own largest entry, with fibres whose scale is
    below `floor` times the global maximum measured against that floor instead;
  * abs_matvec: |A| |x| = sum_k (|S_k| (x) |T_k|) |x|, the scale of the rounding error of each
    entry of A x (a sum of products: |fl(y_i) - y_i| <= c eps (|A| |x|)_i).
"""
import numpy as np


def max_rel(got, want):
    got, want = np.asarray(got).ravel(), np.asarray(want).ravel()
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def fiber_rel(got, want, n_t, floor=1e-6):
    g = np.asarray(got).reshape(-1, n_t)
    w = np.asarray(want).reshape(-1, n_t)
    scale = np.max(np.abs(w), axis=1)
    scale = np.maximum(scale, floor * scale.max())
    return float(np.max(np.max(np.abs(g - w), axis=1) / scale))


def abs_matvec(ref, x):
    """|A| |x| for an oracle Problem (Kronecker form, absolute values of every factor)."""
    X = np.abs(np.asarray(x)).reshape(ref.N_s, ref.n_t)
    Y = np.zeros_like(X)
    for S, T in zip(ref.S, ref.T):
        Y += (abs(S) @ X) @ np.abs(T).T
    return Y.reshape(-1)
