"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module describes *problem data only*: knot vectors, random vectors, the
closed-form potentials, initial data and manufactured solutions of the
Schrodinger problem i u_t - nu Lap u + V u = f (Section 2 of the paper, with a
potential added).  It holds none of the discretisation arithmetic (no B-spline
evaluation, no quadrature, no matrices): both the CPU oracle and the HIP
library sample these functions at quadrature points they compute themselves.

All random draws use ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# knot vectors (Section 3.1: open knot vectors on [0,1])
# ----------------------------------------------------------------------------


def uniform_open_knots(n_el: int, p: int, length: float = 1.0) -> np.ndarray:
    """Open uniform knot vector of maximal regularity C^{p-1} on [0, length].

    The first and last p+1 knots are repeated; the interior breakpoints
    k/n_el appear once.  Length m+p+1 with m = n_el + p basis functions.
    """
    interior = np.arange(1, n_el, dtype=np.float64) / n_el
    kn = np.concatenate([np.zeros(p + 1), interior, np.ones(p + 1)])
    return kn * length


def graded_open_knots(n_el: int, p: int, ratio: float = 1.3, length: float = 1.0) -> np.ndarray:
    """Open knot vector with geometrically graded element sizes (test meshes)."""
    h = ratio ** np.arange(n_el, dtype=np.float64)
    z = np.concatenate([[0.0], np.cumsum(h)])
    z /= z[-1]
    kn = np.concatenate([np.zeros(p), z, np.ones(p)])
    return kn * length


# ----------------------------------------------------------------------------
# random vectors
# ----------------------------------------------------------------------------


def random_complex(n: int, seed: int) -> np.ndarray:
    """i.i.d. standard complex normal vector CN(0,1) of length n."""
    g = np.random.default_rng(seed)
    return (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2.0)


def random_real(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


# ----------------------------------------------------------------------------
# potentials
# ----------------------------------------------------------------------------


@dataclass
class GaussianSum:
    """V(x) = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2))."""

    centres: np.ndarray  # (K, d)
    widths: np.ndarray  # (K,)
    amps: np.ndarray  # (K,)

    def __call__(self, *xs):
        x = np.broadcast_arrays(*xs)
        out = np.zeros(x[0].shape)
        for c, w, a in zip(self.centres, self.widths, self.amps):
            r2 = sum((xi - ci) ** 2 for xi, ci in zip(x, c))
            out += a * np.exp(-r2 / (2.0 * w * w))
        return out


@dataclass
class Harmonic:
    """V(x) = 0.5 w^2 |x - c|^2."""

    w: float
    centre: np.ndarray

    def __call__(self, *xs):
        x = np.broadcast_arrays(*xs)
        r2 = sum((xi - ci) ** 2 for xi, ci in zip(x, self.centre))
        return 0.5 * self.w * self.w * r2


def gaussian_potential(d: int, seed: int, count: int = 8, w_range=(0.05, 0.2),
                       a_range=(0.0, 50.0)) -> GaussianSum:
    """Seeded sum of Gaussians: centres U([0,1]^d), widths U(w_range), amplitudes U(a_range)."""
    g = np.random.default_rng(seed)
    return GaussianSum(centres=g.uniform(0.0, 1.0, size=(count, d)),
                       widths=g.uniform(*w_range, size=count),
                       amps=g.uniform(*a_range, size=count))


def harmonic_potential(d: int, seed: int) -> Harmonic:
    """Seeded harmonic potential, w ~ U(5,20), centre ~ U([0.25,0.75]^d)."""
    g = np.random.default_rng(seed)
    return Harmonic(w=float(g.uniform(5.0, 20.0)), centre=g.uniform(0.25, 0.75, size=d))


# ----------------------------------------------------------------------------
# initial data
# ----------------------------------------------------------------------------


@dataclass
class WavePacket:
    """u0(x) = exp(-|x - c|^2 / (2 sigma^2)) exp(i k.x)."""

    centre: np.ndarray
    sigma: float
    k: np.ndarray

    def __call__(self, *xs):
        x = np.broadcast_arrays(*xs)
        r2 = sum((xi - ci) ** 2 for xi, ci in zip(x, self.centre))
        phase = sum(ki * xi for ki, xi in zip(self.k, x))
        return np.exp(-r2 / (2.0 * self.sigma ** 2)) * np.exp(1j * phase)


def wave_packet(d: int, seed: int, kmax: float = 20.0, sigma_range=(0.05, 0.15)) -> WavePacket:
    """Seeded packet: centre U([0.3,0.7]^d), sigma U(sigma_range), |k| <= kmax (area-uniform in 2D)."""
    g = np.random.default_rng(seed)
    c = g.uniform(0.3, 0.7, size=d)
    sigma = float(g.uniform(*sigma_range))
    if d == 1:
        k = np.array([g.uniform(-kmax, kmax)])
    else:
        direction = g.standard_normal(d)
        direction /= np.linalg.norm(direction)
        k = kmax * g.uniform() ** (1.0 / d) * direction
    return WavePacket(centre=c, sigma=sigma, k=k)


# ----------------------------------------------------------------------------
# manufactured / closed-form solutions (nu = 1 unless stated)
# ----------------------------------------------------------------------------


class SineMode1D:
    """u(t,x) = sin(pi x) exp(-i pi^2 t) on (0,1); S u = (1 + nu) pi^2 u (S = i d_t - nu d_xx)."""

    def __init__(self, nu: float = 1.0):
        self.nu = nu

    def u(self, t, x):
        return np.sin(np.pi * x) * np.exp(-1j * np.pi ** 2 * t)

    def f(self, t, x):
        return (1.0 + self.nu) * np.pi ** 2 * self.u(t, x)

    def u0(self, x):
        return np.sin(np.pi * x) + 0j


class TravelingWave:
    """u(t,x) = a exp(-i(|x|^2 + t^2)/w^2), w = 0.2, a = (2/w^2)^(1/4); the paper's right-hand side.

    The right-hand side a(4i/w^2 + 4|x|^2/w^4 + 2t/w^2) exp(...) is S u for nu = 1 in 2D.
    """

    def __init__(self, omega: float = 0.2):
        self.omega = omega
        self.a = (2.0 / omega ** 2) ** 0.25

    def u(self, t, *xs):
        x = np.broadcast_arrays(t, *xs)
        r2 = sum(xi ** 2 for xi in x[1:])
        return self.a * np.exp(-1j * (r2 + x[0] ** 2) / self.omega ** 2)

    def f(self, t, *xs):
        x = np.broadcast_arrays(t, *xs)
        r2 = sum(xi ** 2 for xi in x[1:])
        w2 = self.omega ** 2
        d = len(xs)
        return (2j * d / w2 + 4.0 * r2 / w2 ** 2 + 2.0 * x[0] / w2) * self.u(t, *xs)


class ComplexGaussian1D:
    """u(t,x) = a b / sqrt(b^2 - i g t) exp(-x^2/(b^2 - i g t)) with a = b = 1.5, g = 2.5 (T = 2).

    f = S u with S = i d_t - nu d_xx, derived by hand from the closed form.
    """

    def __init__(self, alpha=1.5, beta=1.5, gamma=2.5, nu=1.0):
        self.alpha, self.beta, self.gamma, self.nu = alpha, beta, gamma, nu

    def u(self, t, x):
        s = self.beta ** 2 - 1j * self.gamma * t
        return self.alpha * self.beta / np.sqrt(s) * np.exp(-x * x / s)

    def u0(self, x):
        return self.u(0.0, x)

    def f(self, t, x):
        s = self.beta ** 2 - 1j * self.gamma * t
        g = self.gamma
        fac = -g / (2 * s) + g * x * x / s ** 2 - self.nu * (4 * x * x / s ** 2 - 2 / s)
        return fac * self.u(t, x)


class HighModeSeries1D:
    """Truncated high-mode series of Section 6.1 (second test, from Demkowicz et al.) on (0,1),
    T = 2, homogeneous Dirichlet data and u(0) = 0: with e_k = sqrt(2) sin(k pi x) and
    w_k = k pi (the Dirichlet eigenpairs of -d_xx),
        f(t,x) = sum_{k<=M} (1/k) exp(i w_k^2 t) e_k(x),
        u(t,x) = sum_{k<=M} (-i t / k) exp(i w_k^2 t) e_k(x),
    and S u = f for S = i d_t - d_xx (nu = 1).  The paper states M = 625 (and once 652); 625 here."""

    def __init__(self, M: int = 625, chunk: int = 64):
        self.M, self.chunk = int(M), int(chunk)

    def _series(self, t, x, coef):
        t, x = np.broadcast_arrays(np.asarray(t, dtype=np.float64), np.asarray(x, dtype=np.float64))
        out = np.zeros(t.shape, dtype=np.complex128)
        for k0 in range(1, self.M + 1, self.chunk):
            k = np.arange(k0, min(self.M, k0 + self.chunk - 1) + 1, dtype=np.float64)
            kk = k.reshape((-1,) + (1,) * t.ndim)
            w2 = (np.pi * kk) ** 2
            out += np.sum(coef(kk, t) * np.exp(1j * w2 * t) * np.sqrt(2.0) * np.sin(np.pi * kk * x), axis=0)
        return out

    def u(self, t, x):
        return self._series(t, x, lambda k, t: -1j * t / k)

    def f(self, t, x):
        return self._series(t, x, lambda k, t: 1.0 / k + 0.0 * t)

    def u0(self, x):
        return np.zeros(np.shape(x), dtype=np.complex128)

    # the same series through its per-mode factors, for tensor grids too fine to sample point by
    # point: u = sum_k a_k(t) e_k(x), f = sum_k c_k(t) e_k(x)
    def space_factors(self, x):
        """e_k(x_q) for the points x (array of length Q): shape (Q, M)."""
        k = np.arange(1, self.M + 1, dtype=np.float64)
        return np.sqrt(2.0) * np.sin(np.pi * np.outer(np.asarray(x, dtype=np.float64), k))

    def time_factors_u(self, t):
        k = np.arange(1, self.M + 1, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)[:, None]
        return -1j * t / k * np.exp(1j * (np.pi * k) ** 2 * t)

    def time_factors_f(self, t):
        k = np.arange(1, self.M + 1, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)[:, None]
        return (1.0 / k) * np.exp(1j * (np.pi * k) ** 2 * t)

    def f_grid(self, t, x):
        """f on the tensor grid t x x, shape (len(x), len(t)) (time fastest)."""
        return self.space_factors(x) @ self.time_factors_f(t).T


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------


@dataclass
class Workload:
    """One synthetic problem: grid, degree, potential and data."""

    name: str
    d: int
    p: int
    n_el: int
    T: float = 1.0
    nu: float = 1.0
    potential: object = None  # callable V(*x) or None
    u0: object = None  # callable u0(*x) or None
    f: object = None  # callable f(t, *x) or None
    dirichlet: object = None  # callable g(t, *x) or None (homogeneous)
    extra: dict = field(default_factory=dict)

    @property
    def n_s(self):
        return self.n_el + self.p - 2

    @property
    def n_t(self):
        return self.n_el + self.p - 1

    @property
    def n_dof(self):
        return self.n_t * self.n_s ** self.d

    def knots_t(self):
        return uniform_open_knots(self.n_el, self.p, self.T)

    def knots_s(self):
        return uniform_open_knots(self.n_el, self.p)


def sine_1d_workload(nu: float = 1.0, n_el: int = 16, p: int = 2) -> Workload:
    """1D space + time, p = 2, 16 x 16 elements, u = sin(pi x) exp(-i pi^2 t)."""
    m = SineMode1D(nu)
    return Workload("sine1d", d=1, p=p, n_el=n_el, nu=nu, u0=m.u0, f=m.f,
                    extra={"exact": m.u})


def gaussian_potential_2d_workload(sample: int = 0, n_el: int = 64, p: int = 3) -> Workload:
    """2D + time, p = 3, 64^3 elements, 8 Gaussians (seed 2000 + s), packet |k| <= 20, f = 0."""
    seed = 2000 + sample
    V = gaussian_potential(2, seed)
    u0 = wave_packet(2, seed + 500, kmax=20.0)
    return Workload("gauss2d", d=2, p=p, n_el=n_el, potential=V, u0=u0)


def harmonic_3d_workload(sample: int = 0, n_el: int = 48, p: int = 3, with_potential=True) -> Workload:
    seed = 3000 + sample
    V = harmonic_potential(3, seed) if with_potential else None
    u0 = wave_packet(3, seed + 500, kmax=20.0)
    return Workload("harm3d", d=3, p=p, n_el=n_el, potential=V, u0=u0)


def traveling_wave_workload(n_el: int, p: int) -> Workload:
    """2D + time traveling wave, T = 1, non-homogeneous Dirichlet and initial data from u."""
    tw = TravelingWave()
    return Workload("travel2d", d=2, p=p, n_el=n_el, f=tw.f,
                    u0=lambda x1, x2: tw.u(0.0, x1, x2), dirichlet=tw.u,
                    extra={"exact": tw.u})


BATCH_GRIDS = (16, 24, 32, 48, 64)


def batched_2d_workload(count: int = 64, grids=BATCH_GRIDS, p: int = 3, seed0: int = 4000):
    """Batched 2D + time, p = 3, V = 0: `count` systems dealt round-robin over the uneven grids
    (64 -> 13, 13, 13, 13, 12), each with a seeded wave-packet initial datum (|k| <= 30).
    Returns {n_el: [WavePacket, ...]} in grid order."""
    out = {n: [] for n in grids}
    for k in range(count):
        out[grids[k % len(grids)]].append(wave_packet(2, seed0 + k, kmax=30.0))
    return out


# ----------------------------------------------------------------------------
# quarter annulus r0 <= |x| <= r1, x_1, x_2 >= 0 (learned warm-start workload)
# ----------------------------------------------------------------------------

ANNULUS_RADII = (1.0, 2.0)


def _annulus_point(g, r0, r1, margin=0.0):
    """Area-uniform point of the quarter annulus at distance >= margin from its boundary."""
    while True:
        r = np.sqrt(g.uniform(r0 * r0, r1 * r1))
        a = g.uniform(0.0, 0.5 * np.pi)
        x = np.array([r * np.cos(a), r * np.sin(a)])
        if margin <= 0.0 or (r - r0 >= margin and r1 - r >= margin and min(x) >= margin):
            return x


def annulus_gaussian_potential(seed: int, radii=ANNULUS_RADII, count_range=(4, 12), w_range=(0.05, 0.2),
                               a_range=(0.0, 50.0)) -> GaussianSum:
    """Seeded sum of 4-12 Gaussians with area-uniform centres in the quarter annulus."""
    g = np.random.default_rng(seed)
    count = int(g.integers(count_range[0], count_range[1] + 1))
    centres = np.array([_annulus_point(g, *radii) for _ in range(count)])
    return GaussianSum(centres=centres, widths=g.uniform(*w_range, size=count),
                       amps=g.uniform(*a_range, size=count))


def annulus_wave_packet(seed: int, radii=ANNULUS_RADII, kmax: float = 20.0,
                        sigma_range=(0.05, 0.15)) -> WavePacket:
    """Seeded packet with |k| <= kmax and a centre at least 3 sigma inside the quarter annulus."""
    g = np.random.default_rng(seed)
    sigma = float(g.uniform(*sigma_range))
    c = _annulus_point(g, *radii, margin=3.0 * sigma)
    direction = g.standard_normal(2)
    direction /= np.linalg.norm(direction)
    k = kmax * np.sqrt(g.uniform()) * direction
    return WavePacket(centre=c, sigma=sigma, k=k)


def annulus_sample(seed: int):
    """(potential, initial datum) of one learned warm-start sample (train 5000-6999, held-out 7000-7199)."""
    return annulus_gaussian_potential(seed), annulus_wave_packet(seed + 100000)
