"""CPU FP64 oracle for the space-time least-squares Schrodinger solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
NumPy/SciPy implementation of what the library computes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_2311_18461_amd``) never does, and the two
share no code apart from the seeded problem data in
``paper_2311_18461_amd.inputs``.

Module map (paper sections):
  bspline   - Cox-de Boor B-splines and derivatives (Section 3.1)
  matrices  - 1D Gram matrices in space and time, Dirichlet reduction (Sections 3.2, 4.3)
  spatial   - d-dimensional spatial operators with potential (eq. syst_mat + potential terms)
  operators - dense system matrix A, preconditioner P-hat, Kronecker matvec,
              fast-diagonalisation apply (Section 5, Algorithm 1)
  pcg       - preconditioned conjugate gradients (Section 5.3)
  rhs       - load vector and lifting of initial/boundary data (Section 2.2, 4.3)
  ultraweak - ultraweak method: final-condition test space, right-hand side with the
              initial data, solution u_h = S_V z_h (Section 4.4)
  norms     - L2(Q) and V-norm errors (Section 2.1)

Every function states the passage it follows.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""
