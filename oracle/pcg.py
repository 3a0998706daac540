"""Preconditioned conjugate gradients for the Hermitian positive definite system (Section 5.3).

Test infrastructure: see the package docstring.

The paper solves A u = f by CG with tolerance 1e-8, a zero initial guess and
at most 200 iterations.  Readings taken here: the stopping test is
||f - A x_k||_2 / ||f||_2 <= tol on the recursively updated residual, inner
products are <a, b> = a^H b, and beta uses the Polak-Ribiere form
<r_{k+1}, z_{k+1} - z_k> / <r_k, z_k>, which equals the Fletcher-Reeves form
for an exact fixed preconditioner.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, precond, f, x0=None, tol=1e-8, maxit=200, record=False):
    """Return (x, info) with info = dict(iters, rel_res, true_rel_res, converged, history)."""
    f = np.asarray(f, dtype=np.complex128)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.complex128)
    nf = np.linalg.norm(f)
    r = f - matvec(x) if x0 is not None else f.copy()
    hist = [np.linalg.norm(r) / nf]
    it = 0
    if hist[-1] <= tol:
        return x, {"iters": 0, "rel_res": hist[-1], "true_rel_res": hist[-1], "converged": True,
                   "history": hist}
    z = precond(r)
    p = z.copy()
    rz = np.vdot(r, z).real
    converged = False
    while it < maxit:
        q = matvec(p)
        pq = np.vdot(p, q).real
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / nf)
        if hist[-1] <= tol:
            converged = True
            break
        z_new = precond(r)
        beta = np.vdot(r, z_new - z).real / rz
        rz = np.vdot(r, z_new).real
        p = z_new + beta * p
        z = z_new
    true = np.linalg.norm(f - matvec(x)) / nf
    return x, {"iters": it, "rel_res": hist[-1], "true_rel_res": true, "converged": converged,
               "history": hist if record else None}
