"""d-dimensional spatial operators on the parametric domain (0,1)^d.

Test infrastructure: see the package docstring.

Two independent constructions:
  * ``kron_operators``: M_s, L_s, B_s as sums of Kronecker products of the 1D
    matrices (Section 3.3 eq. kron_vec_multi and the definitions in eq.
    space_mat / prec_definition), valid for F = Id.
  * ``quadrature_operator``: brute-force element-by-element tensor Gauss
    quadrature of int c phi_I phi_J, int c phi_I Lap phi_J, int c grad phi_I .
    grad phi_J or int c Lap phi_I Lap phi_J with an arbitrary weight c sampled
    at the quadrature points.  This is what the potential terms need
    (M_V, M_{V^2}, K_V) and it cross-checks the Kronecker forms.

Ordering: a spatial index is i = i_1 + n_1 (i_2 + n_2 i_3) (x_1 fastest),
so a Kronecker product is written J_d (x) ... (x) J_1.
"""
from __future__ import annotations

import itertools
from functools import reduce

import numpy as np
import scipy.sparse as sp

from .bspline import basis, breakpoints, gauss_rule
from .matrices import gram_1d


def kron_seq(mats, sparse=False):
    """J_d (x) ... (x) J_1 for mats = [J_1, ..., J_d]."""
    if sparse:
        return reduce(lambda acc, m: sp.kron(m, acc, format="csr"), [sp.csr_matrix(m) for m in mats])
    return reduce(lambda acc, m: np.kron(m, acc), mats)


def kron_operators(space1d: list, sparse=False) -> dict:
    """M_s, L_s, B_s on the Dirichlet-reduced tensor basis (F = Id, no potential).

    M_s = (x)_l M_l; L_s = sum_l (M ... L_l ... M) (eq. prec_definition);
    B_s[I,J] = int Lap phi_I Lap phi_J expanded over the second derivative in
    direction l of phi_I and direction k of phi_J:
    B_s = sum_{l,k} (x)_dir X^(a,b) with a = 2 if dir = l else 0, b = 2 if dir = k else 0,
    X^(0,0) = M, X^(2,2) = J, X^(2,0) = D20, X^(0,2) = D20^T.
    """
    d = len(space1d)
    M = [s["M"] for s in space1d]
    Ms = kron_seq(M, sparse)
    Ls = sum(kron_seq([space1d[j]["L"] if j == l else M[j] for j in range(d)], sparse) for l in range(d))

    def X(j, a, b):
        s = space1d[j]
        if a == 0 and b == 0:
            return s["M"]
        if a == 2 and b == 2:
            return s["J"]
        if a == 2:
            return s["D20"]
        return s["D20"].T

    Bs = sum(kron_seq([X(j, 2 if j == l else 0, 2 if j == k else 0) for j in range(d)], sparse)
             for l in range(d) for k in range(d))
    return {"M": Ms, "L": Ls, "B": Bs}


def _direction_data(knots, p, q):
    """Per-element local basis data for one direction.

    Returns (first, Bloc, x, w): first[e] = index of the first non-zero function
    on element e, Bloc[e] = (3, p+1, q) values/1st/2nd derivatives, and the
    quadrature points/weights as (n_el, q) arrays.
    """
    kn = np.asarray(knots, dtype=np.float64)
    x, w, _ = gauss_rule(kn, q)
    z = breakpoints(kn)
    n_el = len(z) - 1
    B = basis(kn, p, x, nder=2)
    first = np.searchsorted(kn, z[:-1], side="right") - 1 - p
    Bloc = np.empty((n_el, 3, p + 1, q))
    for e in range(n_el):
        Bloc[e] = B[:, first[e]:first[e] + p + 1, e * q:(e + 1) * q]
    return first, Bloc, x.reshape(n_el, q), w.reshape(n_el, q)


def quadrature_grid(knots_list, q):
    """Tensor quadrature points per direction, as used by ``quadrature_operator``."""
    return [gauss_rule(kn, q)[0] for kn in knots_list]


def quadrature_operator(knots_list, p: int, kind: str, coef=None, q: int | None = None,
                        reduced: bool = True) -> sp.csr_matrix:
    """Brute-force tensor-quadrature assembly of a spatial bilinear form.

    kind: "mass"  int c phi_I phi_J
          "lap"   int c phi_I Lap phi_J           (K_V when c = V)
          "stiff" int c grad phi_I . grad phi_J
          "bilap" int c Lap phi_I Lap phi_J
    coef: None (c = 1) or an array of c at the tensor quadrature grid with
          shape (Q_d, ..., Q_1) (x_1 fastest), Q_l = n_el_l * q.
    reduced: keep only functions vanishing on the boundary (Section 3.2).
    """
    d = len(knots_list)
    q = p + 1 if q is None else q
    dirs = [_direction_data(kn, p, q) for kn in knots_list]
    m = [len(kn) - p - 1 for kn in knots_list]
    n_el = [dd[1].shape[0] for dd in dirs]
    nl = p + 1
    rows, cols, vals = [], [], []
    # local function offsets and strides (x_1 fastest)
    strides = np.cumprod([1] + m[:-1])
    loc = np.array(list(itertools.product(*[range(nl)] * d)))[:, ::-1]  # (nl^d, d): column l = a_l
    for etuple in itertools.product(*[range(n) for n in reversed(n_el)]):
        e = etuple[::-1]  # e[l] = element index in direction l
        vals_l = [dirs[l][1][e[l]] for l in range(d)]  # (3, nl, q)
        wts = reduce(np.multiply.outer, [dirs[l][3][e[l]] for l in reversed(range(d))]).ravel()
        if coef is not None:
            sl = tuple(slice(e[l] * q, (e[l] + 1) * q) for l in reversed(range(d)))
            wts = wts * np.asarray(coef)[sl].ravel()

        def tens(order):
            # tensor-product local matrix (nl^d, q^d) with derivative order[l] in direction l
            return kron_seq([vals_l[l][order[l]] for l in range(d)])

        val = tens([0] * d)
        if kind == "mass":
            loc_m = (val * wts) @ val.T
        elif kind in ("lap", "bilap"):
            lap = sum(tens([2 if j == l else 0 for j in range(d)]) for l in range(d))
            loc_m = (val * wts) @ lap.T if kind == "lap" else (lap * wts) @ lap.T
        elif kind == "stiff":
            loc_m = sum((g * wts) @ g.T for g in
                        (tens([1 if j == l else 0 for j in range(d)]) for l in range(d)))
        else:
            raise ValueError(kind)
        gidx = ((np.array([dirs[l][0][e[l]] for l in range(d)])[None, :] + loc) * strides[None, :]).sum(1)
        rows.append(np.repeat(gidx, len(gidx)))
        cols.append(np.tile(gidx, len(gidx)))
        vals.append(loc_m.ravel())
    N = int(np.prod(m))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    if reduced:
        keep = interior_indices(m)
        A = A[keep][:, keep]
    return A


def interior_indices(m):
    """Flat indices (x_1 fastest) of the functions vanishing on the boundary."""
    grids = np.meshgrid(*[np.arange(1, mm - 1) for mm in reversed(m)], indexing="ij")
    strides = np.cumprod([1] + list(m[:-1]))
    idx = sum(g * s for g, s in zip(reversed(grids), strides))
    return idx.ravel()


def system_spatial_factors(knots_list, p: int, nu: float, V=None, q: int | None = None,
                           sparse=True) -> list:
    """Spatial factors S_1, S_2, S_3 of the system with potential (F = Id).

    With S_V = i d_t - nu Lap + V the Gram matrix (S_V B_J, S_V B_I) splits as
      S_1 (x) L_t + S_2 (x) M_t + S_3 (x) (W_t + W_t^*),
      S_1 = M_s, S_2 = nu^2 B_s - nu (K_V + K_V^T) + M_{V^2}, S_3 = nu L_s + M_V,
    which reduces to eq. syst_mat for V = 0.  V is a callable V(x_1, ..., x_d)
    (sampled here at the quadrature points) or None.
    """
    q = p + 1 if q is None else q
    s1d = []
    for kn in knots_list:
        full = gram_1d(kn, p, q)
        s1d.append({k: v[1:-1, 1:-1] for k, v in full.items()})
    ko = kron_operators(s1d, sparse=sparse)
    S1, S2, S3 = ko["M"], nu * nu * ko["B"], nu * ko["L"]
    if V is not None:
        pts = quadrature_grid(knots_list, q)
        grid = np.meshgrid(*reversed(pts), indexing="ij")  # arrays (Q_d, ..., Q_1)
        Vq = V(*reversed(grid))
        MV = quadrature_operator(knots_list, p, "mass", Vq, q)
        MV2 = quadrature_operator(knots_list, p, "mass", Vq * Vq, q)
        KV = quadrature_operator(knots_list, p, "lap", Vq, q)
        if not sparse:
            MV, MV2, KV = MV.toarray(), MV2.toarray(), KV.toarray()
        S2 = S2 - nu * (KV + KV.T) + MV2
        S3 = S3 + MV
    return [S1, S2, S3]
