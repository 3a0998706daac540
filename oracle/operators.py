"""System matrix, preconditioner and their Kronecker-structured application.

Test infrastructure: see the package docstring.

Vector layout (Section 3.3, vec operator): the coefficient of B_{(i_t, i_s)}
sits at i_t + n_t * i_s, time fastest.  As a NumPy array a vector is viewed
as X with shape (N_s, n_t), X[i_s, i_t]; a Kronecker product S (x) T then
acts as X -> S X T^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .geometry import mapped_spatial_factors
from .matrices import space_1d, time_1d
from .spatial import kron_operators, kron_seq, system_spatial_factors


class Problem:
    """Discrete least-squares Schrodinger system on (0,T) x (0,1)^d (Section 4.3).

    Holds the time matrices (eq. time_mat), the spatial factors of the system
    (eq. syst_mat plus potential terms) and the 1D pencils of the
    preconditioner (eq. prec_definition).
    """

    def __init__(self, knots_t, knots_s: list, p_t: int, p_s: int, nu: float = 1.0,
                 V=None, q: int | None = None, geometry=None, final: bool = False):
        """final=True: time basis with the final condition w(T) = 0 (the ultraweak method of
        Section 4.4, whose matrix has the same Kronecker form; see oracle.ultraweak)."""
        self.geometry, self.q, self.final = geometry, q, final
        self.d = len(knots_s)
        self.nu = float(nu)
        self.p_t, self.p_s = p_t, p_s
        self.knots_t = np.asarray(knots_t, dtype=np.float64)
        self.knots_s = [np.asarray(k, dtype=np.float64) for k in knots_s]
        self.time = time_1d(self.knots_t, p_t, None if q is None else q, final=final)
        self.space1d = [space_1d(k, p_s, q) for k in self.knots_s]
        self.n_t = self.time["M"].shape[0]
        self.n_s = [s["M"].shape[0] for s in self.space1d]
        self.N_s = int(np.prod(self.n_s))
        self.N = self.n_t * self.N_s
        if geometry is None:
            self.S = system_spatial_factors(self.knots_s, p_s, self.nu, V, q, sparse=True)
        else:  # mapped domain (V in physical coordinates); P-hat stays the parametric one
            self.S = mapped_spatial_factors(self.knots_s, p_s, self.nu, geometry, V, q)
        self.T = [self.time["L"], self.time["M"], self.time["T3"]]

    # -- eq. syst_mat ---------------------------------------------------------
    def dense_A(self) -> np.ndarray:
        """A = sum_k S_k (x) T_k as a dense matrix (tiny grids only)."""
        return sum(np.kron(S.toarray(), T) for S, T in zip(self.S, self.T))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x using the Kronecker form: Y = sum_k S_k X T_k^T (eq. kron_vec_multi)."""
        X = np.asarray(x).reshape(self.N_s, self.n_t)
        Y = np.zeros_like(X, dtype=np.complex128)
        for S, T in zip(self.S, self.T):
            Y += (S @ X) @ T.T
        return Y.reshape(-1)

    # -- eq. prec_definition --------------------------------------------------
    def dense_P(self, shift: float = 0.0) -> np.ndarray:
        """P-hat = M_s (x) L_t + nu^2 L_s M_s^-1 L_s (x) M_t + nu L_s (x) (W_t + W_t^*).

        shift c: the same construction for S + c (a constant potential), i.e. nu L_s replaced by
        H_c = nu L_s + c M_s in both places: M_s (x) L_t + H_c M_s^-1 H_c (x) M_t + H_c (x) T3."""
        ko = kron_operators(self.space1d)
        Ms, Ls = ko["M"], ko["L"]
        Hc = self.nu * Ls + shift * Ms
        HMH = Hc @ np.linalg.solve(Ms, Hc)
        t = self.time
        return np.kron(Ms, t["L"]) + np.kron(HMH, t["M"]) + np.kron(Hc, t["T3"])


def mean_potential(knots_s, p: int, V, q: int | None = None) -> float:
    """Mean of V over the unit cube by the element Gauss rule of the spatial directions (q = p + 1
    points per element by default): the constant that the shifted preconditioner takes."""
    from .bspline import gauss_rule
    q = p + 1 if q is None else q
    pts, wts = [], []
    for kn in knots_s:
        x, w, _ = gauss_rule(np.asarray(kn, dtype=np.float64), q)
        pts.append(x)
        wts.append(w)
    grids = np.meshgrid(*pts, indexing="ij")
    W = np.ones_like(grids[0])
    for l, w in enumerate(wts):
        shape = [1] * len(wts)
        shape[l] = w.size
        W = W * w.reshape(shape)
    return float(np.sum(W * V(*grids)) / np.sum(W))


def mapped_pencil(prob: Problem):
    """Physical mass and stiffness matrices (M, L) of a mapped domain: S_1 and S_3 / nu of the
    V-free mapped system (dense)."""
    S1, _, S3 = mapped_spatial_factors(prob.knots_s, prob.p_s, prob.nu, prob.geometry, None, prob.q)
    return S1.toarray(), S3.toarray() / prob.nu


def dense_P_mapped(prob: Problem) -> np.ndarray:
    """eq. prec_definition with the physical M and L of a mapped domain (tiny grids only)."""
    M, L = mapped_pencil(prob)
    t = prob.time
    return (np.kron(M, t["L"]) + prob.nu ** 2 * np.kron(L @ np.linalg.solve(M, L), t["M"])
            + prob.nu * np.kron(L, t["T3"]))


class MappedFastDiagonalization:
    """P-hat^{-1} with the physical M and L of a mapped domain, by fast diagonalisation with one
    dense generalised eigenproblem L U = M U Lambda of the whole spatial pencil (scipy eigh),
    then the same time solves as Algorithm 1.  Independent of any separable structure."""

    def __init__(self, prob: Problem):
        self.prob = prob
        M, L = mapped_pencil(prob)
        self.lam, self.U = sla.eigh(L, M)
        t = prob.time
        self.Lt, self.Mt, self.T3 = t["L"], t["M"], t["T3"]

    def apply(self, r: np.ndarray) -> np.ndarray:
        prob = self.prob
        Y = self.U.T @ np.asarray(r, dtype=np.complex128).reshape(prob.N_s, prob.n_t)
        mu = prob.nu * self.lam
        H = self.Lt[None] + (mu ** 2)[:, None, None] * self.Mt[None] + mu[:, None, None] * self.T3[None]
        Z = np.linalg.solve(H, Y[..., None])[..., 0]
        return (self.U @ Z).reshape(-1)


class FastDiagonalization:
    """Algorithm 1: apply P-hat^{-1} by the fast diagonalisation method.

    Step 1 (setup): the generalised eigenproblems L_l U_l = M_l U_l Lambda_l with
    U_l^T M_l U_l = I (eq. space_eig), solved by LAPACK through scipy.linalg.eigh,
    and lambda_i = sum_l lambda_{l,i_l} (Kronecker sum Lambda_s).
    Step 2: y = (U_s^T (x) I_t) r, i.e. mode products with U_l^T.
    Step 3: x_i = H_i^{-1} y_i with H_i = L_t + nu^2 lambda_i^2 M_t + nu lambda_i (W_t + W_t^*)
            (with a shift c: mu_i = nu lambda_i + c in place of nu lambda_i).
    Step 4: s = (U_s (x) I_t) x.
    """

    def __init__(self, prob: Problem, precompute_inverse: bool | None = None, shift: float = 0.0):
        """shift c: P-hat of S + c (see Problem.dense_P); the modes' scalars become nu lambda_i + c."""
        self.prob = prob
        self.shift = float(shift)
        self.U, self.lam1d = [], []
        for s in prob.space1d:
            lam, U = sla.eigh(s["L"], s["M"])
            self.U.append(U)
            self.lam1d.append(lam)
        # Kronecker sum, x_1 fastest
        d = prob.d
        lam = np.zeros(tuple(reversed(prob.n_s)))
        for l, l1 in enumerate(self.lam1d):
            shape = [1] * d
            shape[d - 1 - l] = l1.size
            lam = lam + l1.reshape(shape)
        self.lam = lam.reshape(-1)
        assert self.lam.size == prob.N_s
        t = prob.time
        self.Lt, self.Mt, self.T3 = t["L"], t["M"], t["T3"]
        if precompute_inverse is None:
            precompute_inverse = prob.N_s * prob.n_t ** 2 * 16 < 1.5e9
        self.Hinv = self._inverses(np.arange(prob.N_s)) if precompute_inverse else None

    def H(self, idx) -> np.ndarray:
        """Stack of H_i for the modes in idx (Section 5.2)."""
        mu = self.prob.nu * self.lam[idx] + self.shift
        return (self.Lt[None] + (mu ** 2)[:, None, None] * self.Mt[None]
                + mu[:, None, None] * self.T3[None])

    def _inverses(self, idx):
        return np.linalg.inv(self.H(idx))

    def _mode_products(self, X, mats):
        """Apply mats[l] along spatial direction l of X with shape (n_d, ..., n_1, n_t)."""
        d = self.prob.d
        for l, U in enumerate(mats):
            axis = d - 1 - l
            X = np.moveaxis(np.tensordot(U, X, axes=([1], [axis])), 0, axis)
        return X

    def apply(self, r: np.ndarray) -> np.ndarray:
        prob = self.prob
        X = np.asarray(r, dtype=np.complex128).reshape(tuple(reversed(prob.n_s)) + (prob.n_t,))
        Y = self._mode_products(X, [U.T for U in self.U]).reshape(prob.N_s, prob.n_t)
        if self.Hinv is not None:
            Z = np.einsum("itk,ik->it", self.Hinv, Y)
        else:
            Z = np.empty_like(Y)
            for c0 in range(0, prob.N_s, 4096):
                idx = np.arange(c0, min(prob.N_s, c0 + 4096))
                Z[idx] = np.linalg.solve(self.H(idx), Y[idx][..., None])[..., 0]
        Z = Z.reshape(tuple(reversed(prob.n_s)) + (prob.n_t,))
        return self._mode_products(Z, self.U).reshape(-1)


def dense_fd_factorization(fd: FastDiagonalization) -> np.ndarray:
    """(U_s^T (x) I)^{-1} H (U_s (x) I)^{-1} assembled densely (eq. preconditioner_str2)."""
    Us = kron_seq(fd.U)
    It = np.eye(fd.prob.n_t)
    Hblk = sla.block_diag(*fd.H(np.arange(fd.prob.N_s)))
    left = np.linalg.inv(np.kron(Us.T, It))
    right = np.linalg.inv(np.kron(Us, It))
    return left @ Hblk @ right
