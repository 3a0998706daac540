/*
 * stfd.h - C ABI of the MI355X space-time fast-diagonalisation solver for the
 * linear Schrodinger equation  i u_t - nu Lap u + V u = f  on (0,T) x (0,1)^d,
 * discretised by the least-squares space-time isogeometric method of
 * Bressan, Kushova, Sangalli, Tani, "Space-time least squares approximation
 * for Schrodinger equation and efficient solver" (arXiv 2311.18461).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors.  A space-time coefficient vector is complex FP64, stored as
 *   interleaved (re, im) doubles (the memory layout of std::complex<double>
 *   and torch.complex128).  Entry (i_t, i_1, ..., i_d) of the coefficient
 *   tensor sits at index i_t + n_t * (i_1 + n_1 * (i_2 + n_2 * i_3)): time is
 *   the fastest index, as in the vec operator of Section 3.3 (eq.
 *   kron_vec_multi) and the ordering "space (x) time" of eq. syst_mat.
 *   With nrhs > 1 the vectors are stacked, right-hand side slowest.
 * Degrees of freedom.  n_t = m_t - 1 (the first time function is removed,
 *   u(0) = 0) and n_l = m_l - 2 (first and last spatial functions removed,
 *   homogeneous Dirichlet), Section 3.2; N = n_t * n_1 * ... * n_d.
 * Memory.  Pointers named *_dev are device (HIP) pointers owned by the caller;
 *   the library never frees them.  Every other pointer is host memory.  All
 *   device memory the library needs is allocated in stfd_setup and freed in
 *   stfd_destroy; apply/matvec/pcg allocate nothing.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *   stream).  apply and matvec are asynchronous and stream-ordered; pcg
 *   returns when the solve has finished because it fills host-side info.
 *   One handle must not be used by two streams at the same time (it owns one
 *   set of work buffers).
 * Errors.  Every int-returning function returns a stfd_status; no exception
 *   crosses the ABI.  On STFD_EHIP the HIP error code is available from
 *   stfd_last_hip_error().
 */
#ifndef STFD_H
#define STFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stfd_problem stfd_problem; /* opaque handle, immutable after setup */

typedef enum {
  STFD_OK = 0,
  STFD_NOT_CONVERGED = 1, /* pcg hit maxit; u holds the last iterate */
  STFD_EINVAL = -1,       /* invalid argument (see each function) */
  STFD_ENOTSPD = -2,      /* a pencil or time block is not (Hermitian) positive definite */
  STFD_EBREAKDOWN = -3,   /* pcg: non-finite value, <p,Ap> <= 0 or <r,z> <= 0 */
  STFD_ENOMEM = -4,       /* host or device allocation failed */
  STFD_EHIP = -5          /* HIP runtime error */
} stfd_status;

/* Arithmetic of the preconditioner's mode products and time solves.
 * The matvec, residuals, inner products and PCG updates are always FP64. */
typedef enum {
  STFD_FP64 = 0,  /* FP64 MFMA mode products, FP64 time solves */
  STFD_FP32 = 1,  /* FP32 MFMA mode products, FP32 intermediates and time solves (FP32 tables) */
  STFD_BF16 = 2   /* BF16 MFMA mode products with FP32 accumulation, FP32 time solves */
} stfd_precision;

/* pcg flags: the initial guess (STFD_X0_ZERO, STFD_X0_GIVEN, or STFD_X0_GIVEN |
 * STFD_X0_SCALED), optionally or-ed with STFD_PCG_GRAPH to replay each iteration from a
 * captured HIP graph.  STFD_X0_SCALED replaces the given x0 by alpha x0 with the complex
 * alpha = <x0, f> / <x0, A x0>, the complex multiple closest to the solution in the A-norm (the
 * norm CG minimises; it corrects the modulus and the phase of a guess); alpha = 0 (a cold start)
 * when <x0, A x0> <= 0 or when the residual of alpha x0 exceeds ||f||, so a poor guess (for
 * instance a learned prediction) never starts CG farther from the solution, or with a larger
 * residual, than x0 = 0. */
enum { STFD_X0_ZERO = 0, STFD_X0_GIVEN = 1, STFD_PCG_GRAPH = 2, STFD_X0_SCALED = 4 };

/* Physical domain.  STFD_GEOM_UNIT_CUBE: Omega = (0,1)^d, x = xi.
 * STFD_GEOM_QUARTER_ANNULUS (d = 2): x = (r0 + (r1 - r0) xi_1) c(xi_2) with c the
 * quarter circle written as a rational quadratic arc (control points (1,0), (1,1),
 * (0,1), weights 1, sqrt(2)/2, 1), an exact parametrisation of the domain
 * (Section 3.1 allows a mapped domain Omega = F(Omega_hat); the paper's tests use
 * the unit cube).  The system operator uses the physical Laplacian and measure; the
 * preconditioner is chosen by the precond field (below). */
enum { STFD_GEOM_UNIT_CUBE = 0, STFD_GEOM_QUARTER_ANNULUS = 1 };

/* Preconditioner on a mapped domain.  The paper defines P-hat for the unit cube only
 * (Section 5, eq. prec_definition).  STFD_PRECOND_PARAMETRIC applies that P-hat unchanged on
 * the parametric square.  STFD_PRECOND_AUTO (default) applies the same formula with the
 * physical mass and stiffness matrices M, L of the quarter annulus: its metric is separable,
 * so U^T M U = I, U^T L U = Lambda holds with U = [W_j (x) v_j] from a pencil in theta and one
 * pencil in rho per theta mode, and Algorithm 1 runs with a per-mode matrix along x_1.  On the
 * unit cube both choices are the paper's P-hat. */
enum { STFD_PRECOND_AUTO = 0, STFD_PRECOND_PARAMETRIC = 1 };

/* Potential in the preconditioner (an extension: the paper's P-hat has no potential, Section 5).
 * STFD_SHIFT_NONE: P-hat as defined.  STFD_SHIFT_MEAN_POTENTIAL (unit cube): P-hat built for
 * S + c with c the mean of V_quad over the unit cube (element Gauss rule), i.e. nu L_s replaced by
 * nu L_s + c M_s in eq. prec_definition; the same eigenvectors diagonalise it, and Algorithm 1 runs
 * with the scalars nu lambda_i + c in the time pencils H_i.  For V = c it satisfies P-hat_c <= A
 * as P-hat does for V = 0; with a varying potential it cuts PCG iterations (8-Gaussian potential,
 * p = 3: 92 -> 42 at 32^3).  c is fixed at setup (stfd_update_potential keeps it; see
 * stfd_get_precond_shift). */
enum { STFD_SHIFT_NONE = 0, STFD_SHIFT_MEAN_POTENTIAL = 1 };

/* Form of the system matvec (Section 5.3: the residual is the dominant cost of an iteration).
 * STFD_MATVEC_STENCIL stores the spatial factors S_1..S_3 as (2p_s+1)^d-point stencils with
 * per-point coefficients.  STFD_MATVEC_SUMFAC (unit cube, d = 2 or 3, p_s <= 5, V = 0 or V a
 * sum of one-dimensional functions V(x) = sum_l v_l(x_l), such as the harmonic potential) applies
 * them sum-factorised: with h_l = -nu d_l^2 + v_l the factors are Kronecker sums of the 1D banded
 * matrices M_l, G_l = int (h_l b_j) b_i and Jh_l = int (h_l b_j)(h_l b_i), applied in one pass along
 * x_1 and time and one pass per further direction, each reading 2p_s+1 neighbours per entry.
 * STFD_MATVEC_AUTO picks SUMFAC for d = 3 when it applies, else STENCIL. */
enum { STFD_MATVEC_AUTO = 0, STFD_MATVEC_STENCIL = 1, STFD_MATVEC_SUMFAC = 2 };

/* Time condition of the discrete space (Sections 3.2 and 4.4).
 * STFD_TIME_INITIAL: the least-squares method; the time basis drops its first function
 *   (u(0) = 0 on the free space; the initial data enter through the lifting of stfd_load_vector).
 * STFD_TIME_FINAL: the ultraweak method (eq. uw-discrete-system); the time basis drops its last
 *   function (test space W_h with w(T) = 0).  The system matrix has the same Kronecker form
 *   (eq. syst_mat with the potential terms, on this basis) and the same preconditioner; the
 *   solution x holds the coefficients of z_h in W_h and the discrete solution is u_h = S_V z_h
 *   (i d_t z_h - nu Lap z_h + V z_h).  stfd_load_vector then assembles
 *   (f, B_I) + i (u_0, B_I(., 0)) with no lifting.  Unit cube only (geometry must be
 *   STFD_GEOM_UNIT_CUBE) and homogeneous Dirichlet data. */
enum { STFD_TIME_INITIAL = 0, STFD_TIME_FINAL = 1 };

/* Problem description (Sections 2, 3.1-3.2, 4.3).
 * knots_t / knots_s[l]: open knot vectors on [0,1] (first and last p+1 knots
 *   repeated, non-decreasing), length m + p + 1.  The time basis is
 *   b_i(t) = b_hat_i(t / T).  Interior multiplicity must keep the time space
 *   C^0 (<= p_t) and the spatial spaces C^1 (<= p_s - 1) (Assumption 2).
 * p_t >= 1, p_s >= 2 (Assumption 2).  T > 0, nu > 0.
 * V_quad: NULL (V = 0) or the potential sampled at the spatial tensor Gauss
 *   grid returned by stfd_quad_points for each direction (n_quad points per
 *   element; on a mapped domain at the mapped points, see stfd_map_points),
 *   stored x_1 fastest: V_quad[q_1 + Q_1 (q_2 + Q_2 q_3)].  The
 *   system operator uses S_V = i d_t - nu Lap + V; the preconditioner always
 *   uses V = 0 (it is defined for the parametric domain, Section 5).
 * n_quad: Gauss points per element and direction; 0 means p + 1.
 * max_nrhs: largest nrhs any later call will pass (work buffers are sized now).
 */
typedef struct {
  int d;
  int p_t, p_s;
  const double *knots_t;
  int n_knots_t;
  const double *knots_s[3];
  int n_knots_s[3];
  double T, nu;
  const double *V_quad;
  int n_quad;
  int max_nrhs;
  int geometry;   /* STFD_GEOM_UNIT_CUBE or STFD_GEOM_QUARTER_ANNULUS */
  double geom[2]; /* quarter annulus: inner and outer radius (0 < geom[0] < geom[1]) */
  int precond;    /* STFD_PRECOND_AUTO or STFD_PRECOND_PARAMETRIC */
  int matvec;     /* STFD_MATVEC_AUTO, STFD_MATVEC_STENCIL or STFD_MATVEC_SUMFAC (EINVAL where it
                     does not apply) */
  int no_rhs_workspace; /* 0: allocate the workspace of stfd_load_vector now (the Gauss-grid
                           scratch of one right-hand side, about 16 (prod_a Q_a + 4 m_t
                           prod_l max(m_l, Q_l)) bytes, and max_nrhs lifting tensors); nonzero:
                           skip it, stfd_load_vector then returns STFD_EINVAL on this handle */
  int time_condition; /* STFD_TIME_INITIAL or STFD_TIME_FINAL (see below) */
  int autotune;       /* 0: launch shapes from heuristics; 1: stfd_setup times the candidate shapes
                         on the current device and keeps the fastest (see stfd_get_tuning) */
  int precond_shift;  /* STFD_SHIFT_NONE or STFD_SHIFT_MEAN_POTENTIAL (see below) */
  int fused_segment_length; /* 0: the fused last-direction launch (stfd_tuning.fused_time) takes
                         its segment length from the heuristic or the autotune; > 0: that length
                         (STFD_EINVAL where no compiled fused shape with it fits the problem) */
} stfd_setup_desc;

typedef struct {
  int iters;           /* PCG iterations performed */
  int status;          /* stfd_status of this right-hand side */
  double rel_res;      /* ||r_k||_2 / ||f||_2 of the recursively updated residual */
  double true_rel_res; /* ||f - A u||_2 / ||f||_2 recomputed with the FP64 matvec */
  double x0_scale;     /* modulus |alpha| of the factor applied to the initial guess (0: cold
                          start; 1 for STFD_X0_GIVEN without scaling) */
} stfd_pcg_info;

/* Element-wise Gauss-Legendre rule on the non-empty knot spans of an open
 * knot vector scaled by `scale` (pass T for the time direction, 1 in space).
 * Writes *n_out = n_el * n_quad points and weights (pts/wts may be NULL to
 * query the size).  n_quad = 0 means degree + 1.  Returns STFD_EINVAL for an
 * invalid knot vector. */
int stfd_quad_points(const double *knots, int n_knots, int degree, int n_quad, double scale,
                     double *pts, double *wts, int *n_out);

/* Setup (Algorithm 1 step 1 and the assembly of eq. syst_mat):
 *  - 1D B-spline Gram matrices in space and time (eqs. space_mat, time_mat),
 *  - generalised eigendecompositions L_l U_l = M_l U_l Lambda_l,
 *    U_l^T M_l U_l = I (eq. space_eig), lambda_i = sum_l lambda_{l,i_l},
 *  - factors of the Hermitian banded blocks
 *    H_i = L_t + nu^2 lambda_i^2 M_t + nu lambda_i (W_t + W_t^*) (Section 5.2),
 *  - the spatial factors S_1 = M_s, S_2 = nu^2 B_s - nu (K_V + K_V^T) + M_{V^2},
 *    S_3 = nu L_s + M_V of A = sum_k S_k (x) T_k, T = (L_t, M_t, W_t + W_t^*).
 * Everything is computed in FP64 on the host and uploaded once.
 * Sizes: n_l <= 128 and n_t <= 128 for d = 2, 3; for d = 1, n_1 <= 1024 and n_t <= 2048 (long
 * axes: the mode product walks its K steps in chunks, the matvec sums each entry's neighbours
 * directly, and time axes longer than 64 segments of the compiled lengths are solved by one lane
 * per mode, reported as time_segment_length = 0 by stfd_get_tuning).
 * Errors: STFD_EINVAL (see stfd_setup_desc; sizes beyond the above), STFD_ENOTSPD, STFD_ENOMEM,
 * STFD_EHIP.  On success *out owns all host and device data of the problem. */
int stfd_setup(const stfd_setup_desc *desc, stfd_problem **out);

/* Replace the potential of a set-up problem (same conventions as V_quad in
 * stfd_setup_desc; NULL: V = 0).  The spatial factors S_1..S_3 are rebuilt on
 * the device (one thread per stencil entry, d <= 2; host quadrature for d = 3; the 1D
 * band matrices of a sum-factorised matvec); the potential samples are uploaded again (this
 * call allocates device memory for them).  The preconditioner does not depend on V and is
 * kept.  Synchronises `stream`.
 * Errors: STFD_EINVAL (NULL handle, non-finite V, a V that is not a sum of 1D functions on a
 * handle whose matvec is sum-factorised), STFD_EHIP. */
int stfd_update_potential(stfd_problem *P, const double *V_quad, void *stream);

/* Physical coordinates x = F(xi) of n parametric points (host arrays of n * d
 * doubles, point-major: xi[k * d + l]).  Errors: STFD_EINVAL. */
int stfd_map_points(const stfd_problem *P, const double *xi, int64_t n, double *x);

/* Sizes: n_t, n_s[0..2] (unused directions = 1), N = n_t * prod n_s. */
int stfd_sizes(const stfd_problem *P, int64_t *n_t, int64_t n_s[3], int64_t *n_dof);

/* Right-hand side of the free system with lifting (Section 2.2: u = u_bar +
 * u_bar_0, f_bar = f - S u_bar_0; Section 4.3: load vector f_i = (f, S B_i);
 * here with S_V = S + V):
 *   f_bar_I = integral over (0,T) x Omega of (f - S_V u_bar) conj(S_V B_I),
 * evaluated with the element Gauss rule of the setup (n_quad points per element
 * and direction) by sum factorisation on the device.  u_bar is the joint L2
 * projection of the data onto the B-splines that do not vanish on
 * Gamma = {t = 0} x Omega U (0,T) x boundary(Omega), i.e. the initial face and the
 * lateral faces together (the paper leaves the lifting open); its normal
 * equations are solved on the device by CG, preconditioned face by face with
 * the inverse Kronecker mass matrices, to a relative residual of 1e-14.
 * Grids are the element-wise Gauss points of stfd_quad_points per direction
 * (Q_t points in time, Q_l in x_l).  All samples are complex FP64, interleaved,
 * in device memory, nrhs stacked:
 *   f_q_dev          f on the space-time grid, index q_t + Q_t (q_1 + Q_1 (q_2 + Q_2 q_3));
 *                    NULL: f = 0.
 *   u0_q_dev         u(0, x) on the spatial grid (x_1 fastest); NULL: u0 = 0.
 *   dirichlet_q_dev  host array of 2d device pointers, face x_l = 0 at [2l] and
 *                    x_l = 1 at [2l+1], each the Dirichlet data on the face grid
 *                    (time fastest, then x_k for k != l ascending).  NULL array or
 *                    NULL entry: zero data.
 *   fbar_dev         nrhs free vectors of N complex (output).
 *   lift             host or NULL: nrhs full coefficient tensors of u_bar,
 *                    m_t m_1 ... m_d complex (m_t = n_t + 1, m_l = n_l + 2, time
 *                    fastest), zero at free positions (output).
 * The call uses the workspace allocated by stfd_setup (it allocates nothing), processes the
 * right-hand sides one after the other and returns after the device work has finished; the
 * lifting solve synchronises the stream every 4 iterations to test its convergence.
 * Errors: STFD_EINVAL (NULL handle or output, nrhs < 1 or > max_nrhs, handle set up with
 * no_rhs_workspace), STFD_ENOTSPD (breakdown of the lifting solve), STFD_NOT_CONVERGED (the
 * lifting solve of some right-hand side reached its iteration limit, see
 * stfd_set_lift_max_iterations; that f_bar is assembled from the last lifting iterate),
 * STFD_EHIP.
 * Ultraweak problems (time_condition STFD_TIME_FINAL): fbar = (f, B_I) + i (u_0, B_I(., 0))
 * over the free basis of W_h; dirichlet_q_dev must be NULL or all-NULL (else STFD_EINVAL); no
 * lifting runs and lift, if given, is set to zeros. */
int stfd_load_vector(const stfd_problem *P, const void *f_q_dev, const void *u0_q_dev,
                     const void *const *dirichlet_q_dev, void *fbar_dev, double *lift, int64_t nrhs,
                     void *stream);

/* Iteration limit of the lifting CG inside stfd_load_vector (default 200; about 10 iterations
 * reach its relative residual of 1e-14 on the grids of the paper).  Errors: STFD_EINVAL (NULL
 * handle, max_iter < 1). */
int stfd_set_lift_max_iterations(stfd_problem *P, int max_iter);

/* s = P-hat^{-1} r by fast diagonalisation (Algorithm 1 steps 2-4,
 * eq. preconditioner_str2): mode products with U_l^T, N_s independent banded
 * time solves with H_i, mode products with U_l.  r_dev, s_dev: nrhs stacked
 * complex FP64 vectors (may alias).  precision: stfd_precision.
 * Errors: STFD_EINVAL (nrhs < 1 or > max_nrhs, bad precision), STFD_EHIP. */
int stfd_apply_preconditioner(const stfd_problem *P, const void *r_dev, void *s_dev, int64_t nrhs,
                              int precision, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same operation, kernels and results as
 * stfd_apply_preconditioner, with the two intermediate tensors of Algorithm 1 steps 2-4 in a
 * fixed 64 MiB device array of the library (one per GPU, held until the process ends) instead of
 * the handle's work buffers.  The call allocates nothing.  Limit: each intermediate holds
 * 2 N nrhs reals of the working precision (8 bytes for STFD_FP64, 4 otherwise) in one 32 MiB
 * half, so nrhs <= 32 MiB / (2 N * 8 or 4 bytes) (N = 278,850: nrhs <= 7 in FP64, 15 otherwise);
 * nrhs is not limited by max_nrhs.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two threads, two handles) race and must be ordered by the
 * caller.  Errors: STFD_EINVAL (NULL pointer, nrhs < 1, nrhs above the limit, bad precision),
 * STFD_EHIP. */
int stfd_apply_preconditioner_static(const stfd_problem *P, const void *r_dev, void *s_dev, int64_t nrhs,
                                     int precision, void *stream);

/* y = A x with A = sum_k S_k (x) T_k applied matrix-free (Section 5.3, eq.
 * syst_mat with the potential terms): spatial tensor-banded stencils with
 * (2p_s+1)^d coefficients per row, then the banded time factors.  FP64.
 * x_dev and y_dev must not overlap.  Errors: STFD_EINVAL, STFD_EHIP. */
int stfd_matvec(const stfd_problem *P, const void *x_dev, void *y_dev, int64_t nrhs, void *stream);

/* Preconditioned CG for A u = f (Section 5.3: CG since A is Hermitian positive
 * definite, P-hat applied by Algorithm 1).  Stops when
 * ||f - A u_k||_2 <= rtol ||f||_2 (recursive residual) or after maxit
 * iterations; beta uses the Polak-Ribiere form <r_k+1, z_k+1 - z_k>/<r_k, z_k>.
 * flags: STFD_X0_ZERO (u_dev is overwritten) or STFD_X0_GIVEN (u_dev holds
 * the initial guess), optionally | STFD_PCG_GRAPH (each iteration replayed
 * from a captured HIP graph; same results).  The captured iterations are kept in the handle (up
 * to 4 argument sets: f_dev, u_dev, nrhs, precision, rtol, maxit; the least recently used is
 * dropped) and replayed by later solves with the same arguments, which read the data then in the
 * buffers (a replay touches only the buffers passed to the call that replays it);
 * stfd_set_tuning, stfd_update_potential and stfd_timing_begin / _end drop them.  Each
 * right-hand side converges independently (a
 * converged system is frozen).  info: host array of nrhs entries (may be NULL).
 * precision: arithmetic of the preconditioner (stfd_precision); everything
 * else is FP64.  Returns STFD_OK if all systems converged, STFD_NOT_CONVERGED
 * if some hit maxit, STFD_EBREAKDOWN on breakdown, STFD_EINVAL, STFD_EHIP. */
int stfd_pcg_solve(const stfd_problem *P, const void *f_dev, void *u_dev, int64_t nrhs, double rtol,
                   int maxit, int flags, int precision, stfd_pcg_info *info, void *stream);

/* Batched PCG over several problems (uneven grids), each with its own stack of
 * right-hand sides: job k solves A_k u = f on handle probs[k] for nrhs[k]
 * systems stored at f_dev[k] / u_dev[k] (device, layout as stfd_pcg_solve).
 * Same algorithm and stopping rule as stfd_pcg_solve, per system.  Every job
 * runs on a stream of its handle (created on first use, forked from `stream`
 * and joined back into it), so the small, latency-bound grids run beside the
 * large ones; each job stops launching iterations once all its systems have
 * converged (converged systems of a job still running are masked by their done
 * flags).  flags as stfd_pcg_solve: with STFD_PCG_GRAPH each job's iteration
 * is replayed from its own captured graph on its stream (cached in the job's handle as for
 * stfd_pcg_solve).  The host polls the
 * jobs' progress without blocking.  The handles must be distinct (each owns
 * one set of work buffers and one stream); a handle must not be used
 * concurrently from another thread.  info: host array of sum_k nrhs[k] entries
 * in job order (may be NULL).  count <= 64.  Returns as stfd_pcg_solve. */
int stfd_pcg_solve_batched(const stfd_problem *const *probs, int count, const void *const *f_dev,
                           void *const *u_dev, const int64_t *nrhs, double rtol, int maxit, int flags,
                           int precision, stfd_pcg_info *info, void *stream);

/* Kernel timing for measurement: between stfd_timing_begin and stfd_timing_end every mode-product
 * launch of an apply (Algorithm 1 steps 2 and 4) on this handle is bracketed by two HIP events
 * recorded on its launch stream (up to `capacity` launches; the events are created here).
 * stfd_timing_end waits for the last recorded event and returns the summed event time of the
 * recorded launches and their count, then destroys the events.  Timing adds two event records per
 * launch to the stream and is meant for benchmarks, not for production solves.
 * Errors: STFD_EINVAL (NULL handle, capacity < 1, begin while timing / end while not), STFD_EHIP. */
int stfd_timing_begin(stfd_problem *P, int capacity);
int stfd_timing_end(stfd_problem *P, double *total_ms, int64_t *launches);

/* Kernel timing for measurement: the forward mode product of `direction` (Algorithm 1 step 2)
 * for one right-hand side, in the launch shape the applies use, launched `reps` times back to back
 * on the stream after two untimed launches, from one of the handle's work buffers into the other
 * (their contents are overwritten); *avg_ms = HIP-event time between the first and the last
 * launch divided by reps (back-to-back launches overlap the dispatch of one launch with the
 * previous kernel, as in an apply).  precision FP64: FP64 operand and output (the first product of
 * an FP64 apply); FP32 / BF16: FP32 operand and output.  Synchronises with the stream.
 * Errors: STFD_EINVAL (NULL handle or avg_ms, reps < 1, direction outside 0..d-1, unknown
 * precision), STFD_EHIP. */
int stfd_time_mode_product(stfd_problem *P, int direction, int precision, int reps, void *stream, double *avg_ms);

/* Launch shapes of a problem.  With stfd_setup_desc.autotune = 1 the setup timed on the device
 * (2 untimed and 5 timed launches per candidate on a private stream, median kept):
 *   the shape of every mode product, per precision and direction, for directions with n_l <= 80:
 *   1 or 2 = one 16-column group per wave with 1 or 2 sixteen-row groups (four waves per block on
 *   consecutive row tiles of one column group, its packed operand staged in LDS per block, read
 *   from global memory instead for the per-mode operand of a mapped domain's x_1); 3 = the wide
 *   form (every column group of a 16-row tile in one wave, the packed operand staged in LDS per
 *   block; not for the per-mode operand);
 *   the segment length of the time solve and its form (every table read; rows of L and 1/D read and
 *   the segment transfers computed; or all of them computed, the factor rows from the last P rows
 *   before each segment), every form for problems with N_s n_t <= 2^21, the last form only for
 *   larger ones.  Heuristics without autotune: tables where one right-hand side's grid holds at
 *   most one wave per SIMD, else all computed.
 *   and whether the fused form of the last direction (fused_time) beats the separate launches,
 *   each compiled fused shape that fits timed as a whole FP64 apply.
 * Otherwise the values are the heuristics' (fused form built where it fits, and off).  The BF16
 * applies always run separate launches.  tune_ms: host wall time of the tuning runs. */
typedef struct {
  int autotuned;
  int mode_product_row_groups[3][3]; /* [precision STFD_FP64/FP32/BF16][direction], 0 past d */
  int time_segment_length;           /* rows per lane of the segmented time solve; 0: one lane per
                                        mode over the whole time axis (axes longer than 64 segments) */
  int time_transfers_in_kernel;      /* 1: computed in the solve, 0: read from tables */
  double tune_ms;
  int time_factors_in_kernel;        /* 1: the rows of L and 1/D are factorised in the solve from a
                                        per-segment state (implies transfers in kernel) */
  int fused_time;                    /* 1: the FP64 and FP32 applies run the products along x_d and
                                        the time solves (Algorithm 1 steps 2-4 of direction d and
                                        step 3) as one launch, one block per spatial column
                                        (m_1 .. m_{d-1}) holding its n_d x n_t slab in LDS */
  int fused_segment_length;          /* segment length of that launch's time solves; 0 where the
                                        fused form does not apply (d = 1, mapped domain, no compiled
                                        shape fits) */
  int fused_factors_in_kernel;       /* its time-solve form, as time_factors_in_kernel (else all
                                        tables read) */
} stfd_tuning;
/* Errors: STFD_EINVAL (NULL argument). */
int stfd_get_tuning(const stfd_problem *P, stfd_tuning *out);
/* Sets the mode-product shapes (for instance from a committed tile table) and switches the fused
 * form of the last direction on or off, without timing; the time-solve and fused segment fields
 * must equal the handle's (their tables are built at setup); directions past d are ignored.  The
 * results do not depend on the shapes beyond summation order of the dot-product partials; the
 * fused form rounds as the separate launches with its segment length.  Not to be called while a
 * solve on this handle is in flight.
 * Errors: STFD_EINVAL (NULL argument, a shape outside 1..3 or not allowed for that direction,
 * time-solve or fused segment fields that differ, fused_time not 0 / 1 or 1 where the fused form
 * does not apply). */
int stfd_set_tuning(stfd_problem *P, const stfd_tuning *in);

/* The constant c of the preconditioner (0 unless set up with STFD_SHIFT_MEAN_POTENTIAL).
 * Errors: STFD_EINVAL (NULL argument). */
int stfd_get_precond_shift(const stfd_problem *P, double *c);

/* Host copies of setup data for inspection: U_l (n_l x n_l, row-major,
 * U[j*n_l + k] = entry (j,k), column k = k-th eigenvector) and Lambda_l.
 * Errors: STFD_EINVAL for l outside [0, d). */
int stfd_get_pencil(const stfd_problem *P, int l, double *U, double *lambda);

/* Diagnostic: runs one v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32 and
 * v_mfma_f32_16x16x16bf16_1k with A[m][k] = m + 16 k and B[k][n] = (k == n mod K)
 * on the current device and copies lane l's 4 result registers to
 * out[4 l + v] (host arrays of 256 entries).  Used by tests to pin the
 * operand/result lane layout the mode-product kernel relies on.
 * Errors: STFD_EINVAL (NULL pointer), STFD_EHIP. */
int stfd_debug_mfma_layout(double *out64, float *out32, float *outbf);

void stfd_destroy(stfd_problem *P);
const char *stfd_strerror(int code);
int stfd_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STFD_H */
