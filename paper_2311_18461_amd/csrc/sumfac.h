// Sum-factorised system matvec for separable spatial coefficients (Section 5.3: the residual is the
// dominant cost of a CG iteration and matrix-free assembly is the way to cut it).
//
// On the unit cube with V = 0, or with a potential that is a sum of one-dimensional functions
// V(x) = sum_l v_l(x_l) (the harmonic potential), the operator H = -nu Lap + V is a sum of 1D
// operators h_l = -nu d_l^2 + v_l, and the spatial factors of eq. syst_mat (with the potential
// terms) are Kronecker sums of three 1D banded matrices per direction:
//   M_l,  G_l = int (h_l b_j) b_i = nu L_l + M_l^{v},
//   Jh_l = int (h_l b_j)(h_l b_i) = nu^2 J_l - nu (K_l^{v} + K_l^{v T}) + M_l^{v^2},
// (M^{v} = int v b_i b_j, K^{v} = int v b_i b_j'', reduced Dirichlet basis) as
//   S_1 = M (x) M (x) M,   S_3 = sum_l G_l (x) M_rest,
//   S_2 = sum_l Jh_l (x) M_rest + sum_{l != k} G_l (x) G_k (x) M_rest.
// Grouping the terms by their operators along x_2 and x_3 gives three passes (d = 3):
//   x_1 and time:  Za = (M_1 (x) L_t + G_1 (x) i K_t + Jh_1 (x) M_t) X,
//                  Zb = (M_1 (x) i K_t + 2 G_1 (x) M_t) X,  Zc = (M_1 (x) M_t) X;
//   x_2:           P = M_2 Za + G_2 Zb + Jh_2 Zc,  Q = M_2 Zb + 2 G_2 Zc,  R = M_2 Zc;
//   x_3:           Y = M_3 P + G_3 Q + Jh_3 R
// (d = 2: the last pass runs along x_2 on Za, Zb, Zc).  Each pass reads 2p+1 neighbours per entry
// instead of the (2p+1)^d of the stencil form, and no per-point coefficients.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "host_setup.h"

namespace stfd {

struct SumFacPlan {
  int d = 0, n_t = 0, pt = 0, ps = 0;
  int n[3] = {1, 1, 1};
  int64_t N = 0;               // n_t prod n_l (complex entries per right-hand side)
  double* bands[3] = {};       // device, per direction [3][n_l][2 ps + 1]: M, G, Jh (zero off the matrix)
  const double* tband = nullptr;  // device time bands [n_t][2 pt + 1][4] = (L_t, M_t, K_t, 0)
  double* work = nullptr;      // device: (d == 3 ? 6 : 3) tensors of N max_nrhs complex
  int64_t work_stride = 0;     // reals between the work tensors
  int chunk = 1;               // x_1 rows per block of the first pass (a segment)
  size_t lds = 0;              // LDS bytes of the first pass
  int seg_mid = 1, seg_last = 1;  // rows per thread of the middle and last axis passes
  int last_grid = 1;           // blocks per right-hand side of the last pass (= dot partials)
};

// The 1D band triples (M, G, Jh) of every direction for the potential samples V_quad (NULL:
// V = 0) on the spatial Gauss grid (x_1 fastest).  Returns 0, or 1 when V is not a sum of 1D
// functions to rounding accuracy (then out is left empty).
int sumfac_bands(const HostProblem& hp, const double* V_quad, std::vector<double> out[3]);

// Launch shape for the problem (chunk, LDS, last grid); 0 or -1 if it does not fit.
int sumfac_plan_shape(SumFacPlan& p, size_t max_lds);

// y = A x for nrhs stacked vectors; partial (optional): one Re<x, y> partial per block of the last
// pass, [rhs][last_grid].  done: per right-hand side flags (finished systems skipped) or nullptr.
int sumfac_matvec(const SumFacPlan& p, const double* x, double* y, int64_t nrhs, double* partial, const int* done,
                  hipStream_t s);

}  // namespace stfd
