// Spatial factors of the system operator on the unit cube or on a mapped domain.
//
// The physical domain is x = F(xi) with xi in the parametric unit cube.  With the
// Jacobian determinant J and the physical Laplacian written in parametric
// coordinates as Lap = sum_k c_k(xi) D^k (D^k a parametric derivative), the
// least-squares operator (eq. syst_mat with S_V = i d_t - nu Lap + V) keeps the
// form A = S_1 (x) L_t + S_2 (x) M_t + S_3 (x) (W_t + W_t^*) with
//   S_1 = int phi_I phi_J J,
//   S_3 = nu int grad phi_I . grad phi_J dx + int V phi_I phi_J dx,
//   S_2 = nu^2 int Lap phi_I Lap phi_J dx - nu (K_V + K_V^T) + int V^2 phi_I phi_J dx,
//   K_V = int V phi_I Lap phi_J dx,
// every entry a weighted form  int w(xi) D^a phi_I D^b phi_J dxi  evaluated with the
// element Gauss rule.  On the unit cube the V-free part is assembled from 1D
// matrices (Kronecker identities); everything else is a list of weighted terms.
#pragma once
#include <vector>

#include "host_setup.h"

namespace stfd {

enum { GEOM_UNIT = 0, GEOM_QUARTER_ANNULUS = 1 };

struct Geometry {
  int kind = GEOM_UNIT;
  double r0 = 1.0, r1 = 2.0;  // quarter annulus radii
};

// One weighted form added to a spatial factor:
//   S_target[I][J] += scale * int w(xi) D^a phi_I D^b phi_J dxi,  w = arrays[coef] (coef < 0: w = 1)
struct WeightedTerm {
  int coef = -1;
  int a[3] = {0, 0, 0};
  int b[3] = {0, 0, 0};
  double scale = 1.0;
  int target = 0;  // 0: S_1, 1: S_2, 2: S_3
};

// One term of the physical Laplacian: coefficient arrays[coef] times D^ord (coef < 0: 1),
// coefJ = the same coefficient times J (coefJ < 0: 1).
struct LapTerm {
  int ord[3] = {0, 0, 0};
  int coef = -1;
  int coefJ = -1;
};

// Everything the spatial factors and the load vector need, on the spatial Gauss grid
// (x_1 fastest).
struct SpatialModel {
  std::vector<std::vector<double>> arrays;
  std::vector<WeightedTerm> terms;  // added to the base stencils
  std::vector<LapTerm> lap;         // physical Laplacian
  int J = -1;                       // Jacobian determinant (-1: 1)
  int V = -1;                       // potential (-1: none)
  bool kronecker_base = true;       // V-free unit-cube part assembled from 1D matrices
};

int build_spatial_model(const HostProblem& hp, const Geometry& g, const double* V_quad, SpatialModel& m);

// Physical coordinates of n parametric points (d values each, xi_1 fastest).
void map_points(const Geometry& g, int d, const double* xi, int64_t n, double* x);

// Preconditioner pencils of the quarter annulus.  Its metric is separable: the physical mass
// and stiffness matrices are M = M_r^{dr r} (x) M_t^{s} and
// L = K_r^{r/dr} (x) M_t^{s} + M_r^{dr/r} (x) K_t^{1/s} (superscript: 1D weight).  The theta
// pencil (K_t^{1/s}, M_t^{s}) -> V, mu; then per theta mode j the rho pencil
// (K_r^{r/dr} + mu_j M_r^{dr/r}, M_r^{dr r}) -> W_j, lambda_j: U = [W_j (x) v_j] diagonalises
// both (U^T M U = I, U^T L U = diag(lambda)), so P-hat with these M and L is applied by the
// same fast diagonalisation with a per-mode matrix in the rho direction.  Sets hp.U[1],
// hp.Uslice, hp.lam and the time factors.  0, -1 (not an annulus) or -2.
int geometry_pencils(HostProblem& hp, const Geometry& g);

// Host evaluation of the weighted terms (any d): Sc (layout [k][N_s][stencil]) += terms.
void apply_terms_host(const HostProblem& hp, const SpatialModel& m, double* Sc);

}  // namespace stfd
